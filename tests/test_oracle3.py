"""Pins of the tetrahedral oracle (Sec. 4's extrusion to 3D: coarsening,
refinement and smoothing, no swaps) against what the mathematics fixes:

  - the Kuhn cube grid: counts, conformity, exact volume, Euler characteristic;
  - the mean ratio: 1 for the regular tetrahedron with unit metric edges in
    any metric, (4/3) 2^(-2/3) for the unit corner tetrahedron, invariances,
    an independent matrix-form evaluation;
  - hand cases in exact arithmetic: the centre of a cube collapsing onto the
    smallest-id corner, the strict L^2 < 1/2 threshold, a single bisection
    with its ids and coordinates, a shared face cut the same way from both
    sides, a constant-metric grid as a smoothing fixed point;
  - after every class: conformity, exact volume, Euler characteristic, rows =
    a rebuild, members pairwise non-adjacent, the exact deferred set, every
    member's collapse or move re-derived independently;
  - fixpoints: no long edge after refinement converges, every short legal
    edge blocked after coarsening converges.
"""
import math

import numpy as np
import pytest

from oracle.orc import OracleMesh3, ctx_of, prio
from paper_1505_04694_amd import inputs
from tests import checker3
from tests import independent3 as ind

PH_COARSEN, PH_SMOOTH = 1, 3
MARGIN = 1e-9
REG = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.5, math.sqrt(3.0) / 2.0, 0.0],
                [0.5, math.sqrt(3.0) / 6.0, math.sqrt(2.0 / 3.0)]])


def one_tet(xyz, m6):
    xyz = np.asarray(xyz, float)
    met = np.tile(np.asarray(m6, float), (4, 1))
    return OracleMesh3(xyz, np.array([[0, 1, 2, 3]], np.int32), met, np.zeros(4, np.uint8))


def q_of(xyz, m6):
    return one_tet(xyz, m6).element_quality()[0]


def positive(xyz):
    xyz = np.asarray(xyz, float)
    if checker3.vol6(xyz, np.array([[0, 1, 2, 3]]))[0] < 0:
        xyz = xyz[[0, 2, 1, 3]]
    return xyz


# ---- generator ---------------------------------------------------------------------

@pytest.mark.parametrize("n", [2, 3, 5, 9])
def test_cube_grid_is_a_conforming_tiling(n):
    xyz, tet = inputs.cube_grid(n)
    assert xyz.shape == (n ** 3, 3) and tet.shape == (6 * (n - 1) ** 3, 4)
    s = checker3.check_mesh(dict(xyz=xyz, tet=tet, tags=inputs.unit_cube_tags(xyz)), exact=n <= 5)
    assert s["V"] == n ** 3
    vol = checker3.vol6(xyz, tet)
    assert np.all(vol == vol[0])          # every Kuhn tetrahedron has volume h^3 / 6


# ---- quality -------------------------------------------------------------------------

def test_regular_unit_tetrahedron_is_one():
    assert q_of(REG, [1, 0, 0, 1, 0, 1]) == pytest.approx(1.0, abs=1e-15)


def test_corner_tetrahedron_closed_form():
    # |K| = 1/6, S = 3 * 1 + 3 * 2 = 9, (3 |K|)^(2/3) = 2^(-2/3): q = 12 2^(-2/3) / 9
    q = q_of([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], [1, 0, 0, 1, 0, 1])
    assert q == pytest.approx(4.0 / 3.0 * 2.0 ** (-2.0 / 3.0), rel=1e-15)


@pytest.mark.parametrize("seed", range(5))
def test_regular_tetrahedron_in_metric_space_is_one(seed):
    rng = np.random.default_rng(seed)
    F = rng.normal(size=(3, 3))
    if np.linalg.det(F) < 0:
        F[:, 0] *= -1
    M = F.T @ F
    xyz = np.linalg.solve(F, REG.T).T
    assert q_of(xyz, [M[0, 0], M[0, 1], M[0, 2], M[1, 1], M[1, 2], M[2, 2]]) == pytest.approx(1.0, rel=1e-12)


@pytest.mark.parametrize("seed", range(5))
def test_quality_invariances_and_bound(seed):
    rng = np.random.default_rng(50 + seed)
    xyz = positive(rng.uniform(0, 1, (4, 3)))
    F = rng.normal(size=(3, 3))
    M = F.T @ F + 0.1 * np.eye(3)
    m = [M[0, 0], M[0, 1], M[0, 2], M[1, 1], M[1, 2], M[2, 2]]
    q = q_of(xyz, m)
    assert 0 < q <= 1.0 + 1e-15
    assert q_of(xyz, [7.0 * v for v in m]) == pytest.approx(q, rel=1e-13)
    assert q_of(xyz * 0.25 + 0.3, m) == pytest.approx(q, rel=1e-12)
    L = np.linalg.cholesky(M).T
    assert q_of((L @ xyz.T).T, [1, 0, 0, 1, 0, 1]) == pytest.approx(q, rel=1e-12)


def test_quality_matches_the_matrix_form_on_a_jittered_grid():
    mi = inputs.make_mesh3(5, jitter_seed=3)
    om = OracleMesh3.from_input(mi)
    d = om.export()
    np.testing.assert_allclose(om.element_quality(), checker3.mean_ratio(d["xyz"], d["metric"], d["tet"]),
                               rtol=1e-12)
    Q, qmin = om.quality()
    assert Q == pytest.approx(om.element_quality().sum(), rel=1e-14) and qmin == om.element_quality().min()


def test_invalid_meshes_are_rejected():
    met = np.tile([1.0, 0, 0, 1.0, 0, 1.0], (4, 1))
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    with pytest.raises(ValueError):
        OracleMesh3(xyz, np.array([[0, 2, 1, 3]], np.int32), met)       # negative volume
    with pytest.raises(ValueError):
        OracleMesh3(xyz, np.array([[0, 1, 2, 4]], np.int32), met)       # id out of range
    with pytest.raises(ValueError):
        OracleMesh3(xyz, np.array([[0, 1, 2, 3]], np.int32), np.tile([1.0, 2.0, 0, 1.0, 0, 1.0], (4, 1)))


# ---- hand cases -----------------------------------------------------------------------

def centred_cube(m6):
    """The unit cube's 8 corners (id = x + 2y + 4z) and its centre (id 8), each
    face split along the diagonal through its smallest corner, every face
    triangle joined to the centre."""
    xyz = np.array([[i & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)] + [[0.5, 0.5, 0.5]], float)
    faces = [(0, 2, 6, 4), (1, 5, 7, 3), (0, 4, 5, 1), (2, 3, 7, 6), (0, 1, 3, 2), (4, 6, 7, 5)]
    tets = []
    for a, b, c, d in faces:
        for tri in ((a, b, c), (a, c, d)):
            t = [tri[0], tri[1], tri[2], 8]
            if checker3.vol6(xyz, np.array([t]))[0] < 0:
                t = [tri[0], tri[2], tri[1], 8]
            tets.append(t)
    tet = np.array(tets, np.int32)
    return OracleMesh3(xyz, tet, np.tile(np.asarray(m6, float), (9, 1))), xyz, tet


def test_centre_collapses_onto_the_smallest_corner():
    # every centre edge has L^2 = 0.75 * 0.5 (a tie), corners never move: the
    # centre goes onto corner 0, the four faces through corner 0 lose their
    # elements and the other six become tetrahedra with apex 0
    om, xyz, _ = centred_cube([0.5, 0, 0, 0.5, 0, 0.5])
    st = om.coarsen()
    assert st["committed"] == 1 and om.sizes() == (8, 6)
    d = om.export()
    assert (d["tet"][:, 0] == 0).all()
    checker3.check_mesh(d, exact=True, rows=om.rows())


def test_collapse_threshold_is_strict():
    # diag(1, 1/2, 1/2): the centre edges have L^2 = 0.25 + 0.125 + 0.125 = 1/2 exactly
    om, _, _ = centred_cube([1.0, 0, 0, 0.5, 0, 0.5])
    assert om.coarsen()["committed"] == 0
    om, _, _ = centred_cube([1.0, 0, 0, 0.5, 0, 0.5 - 2 ** -20])
    assert om.coarsen()["committed"] == 1


def test_collapse_quality_bound_is_inclusive():
    # onto corner 0 the centre leaves six path tetrahedra from corner 0 to
    # corner 7 (S = 10 c, D = 1, det = c^3 with c = 1/2): q^3 = 432/1000 in
    # the root-free form, 54/125 rounded once; q_min = 0.7559526299369239 has
    # (q_min^2) q_min equal to it to the last bit, so the bound holds with
    # equality and the collapse is allowed; the next double up blocks it
    qm = 0.7559526299369239
    assert (qm * qm) * qm == (((432.0 * 0.125) * 1.0) * 1.0) / ((5.0 * 5.0) * 5.0)
    om, _, _ = centred_cube([0.5, 0, 0, 0.5, 0, 0.5])
    assert om.coarsen(q_min=qm)["committed"] == 1
    om, _, _ = centred_cube([0.5, 0, 0, 0.5, 0, 0.5])
    assert om.coarsen(q_min=float(np.nextafter(qm, 1.0)))["committed"] == 0


def test_one_long_edge_bisects_once():
    # only 0-1 is long under 2.5 I; the midpoint becomes vertex 4 at (1/2, 0, 0);
    # the child keeping vertex 0 keeps id 0: (0, 4, 2, 3) -> (0, 2, 3, 4); the
    # other (4, 1, 2, 3) -> (1, 4, 3, 2) -> (1, 2, 4, 3)
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0.5, 0.25, 0], [0.5, 0, 0.25]], float)
    om = one_tet(xyz, [2.5, 0, 0, 2.5, 0, 2.5])
    st = om.refine()
    assert (st["committed"], st["new_vertices"], st["new_elements"], st["rounds"]) == (1, 1, 1, 1)
    d = om.export()
    assert d["xyz"][4].tolist() == [0.5, 0.0, 0.0]
    assert d["tet"].tolist() == [[0, 2, 3, 4], [1, 2, 4, 3]]


def test_equal_long_edges_bisect_in_id_order():
    # opposite edges 0-1 and 2-3 are the only long ones, with L^2 = 2.5 both: the
    # tie goes to (0, 1) (mid 4) before (2, 3) (mid 5); depth first the leaves are
    # (0,4,5,2) (0,4,3,5) (4,1,5,2) (4,1,3,5), stored as below
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0.5, -0.5, 0.5], [0.5, 0.5, 0.5]], float)
    om = OracleMesh3(xyz, np.array([[0, 1, 3, 2]], np.int32), np.tile([2.5, 0, 0, 2.5, 0, 2.5], (4, 1)),
                     np.zeros(4, np.uint8))
    st = om.refine(max_passes=1)
    assert (st["new_vertices"], st["new_elements"]) == (2, 3)
    d = om.export()
    assert d["xyz"][4].tolist() == [0.5, 0.0, 0.0] and d["xyz"][5].tolist() == [0.5, 0.0, 0.5]
    assert d["tet"].tolist() == [[0, 2, 4, 5], [0, 3, 5, 4], [1, 2, 5, 4], [1, 3, 4, 5]]
    assert (checker3.vol6(d["xyz"], d["tet"]) > 0).all()


def test_longer_edges_bisect_first():
    # 0-1 (L^2 = 2.5 * 1) is longer than 2-3 (2.5 * 0.81): 0-1 first, so the
    # element splits into four with the same layout as the tie above
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0.5, -0.45, 0.5], [0.5, 0.45, 0.5]], float)
    om = OracleMesh3(xyz, np.array([[0, 1, 3, 2]], np.int32), np.tile([2.5, 0, 0, 2.5, 0, 2.5], (4, 1)),
                     np.zeros(4, np.uint8))
    om.refine(max_passes=1)
    assert om.export()["tet"].tolist() == [[0, 2, 4, 5], [0, 3, 5, 4], [1, 2, 5, 4], [1, 3, 4, 5]]
    # and with 2-3 the longer one, 2-3 goes first
    xyz2 = np.array([[0, 0, 0], [0.9, 0, 0], [0.45, -0.5, 0.5], [0.45, 0.5, 0.5]], float)
    om2 = OracleMesh3(xyz2, np.array([[0, 1, 3, 2]], np.int32), np.tile([2.5, 0, 0, 2.5, 0, 2.5], (4, 1)),
                      np.zeros(4, np.uint8))
    om2.refine(max_passes=1)
    assert om2.export()["tet"].tolist() != om.export()["tet"].tolist()


def test_a_shared_face_is_cut_the_same_way_from_both_sides():
    # two tetrahedra on the face (0, 1, 2); two of its edges are long with equal
    # L^2 (a tie broken by ids) and each apex edge is long too: both sides must
    # bisect the face's edges in one order, or the mesh would not conform
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0.25, 0.25, 0.75], [0.25, 0.25, -0.75]], float)
    tet = np.array([[0, 1, 2, 3], [0, 2, 1, 4]], np.int32)
    tags = np.zeros(5, np.uint8)
    om = OracleMesh3(xyz, tet, np.tile([3.0, 0, 0, 3.0, 0, 3.0], (5, 1)), tags)
    om.refine(max_passes=1)
    d = om.export()
    F = checker3.faces_of(d["tet"])
    key, cnt = np.unique(np.sort(F, axis=1), axis=0, return_counts=True)
    # the refined face (0, 1, 2) and every face inside one parent appear twice;
    # the rest are on the outer surface of the pair
    D = checker3.vol6(d["xyz"], d["tet"])
    assert (D > 0).all() and abs(D.sum() / 6 - 0.75 / 3) < 1e-15
    inner = [k for k, c in zip(key.tolist(), cnt.tolist()) if c == 2]
    on_face = [k for k in inner if all(d["xyz"][v][2] == 0.0 for v in k)]
    assert len(on_face) >= 2                    # the split face's triangles are shared
    assert cnt.max() == 2


@pytest.mark.parametrize("m6", [[64.0, 0, 0, 64.0, 0, 64.0], [16.0, 4.0, 0, 32.0, 0, 8.0]])
def test_constant_metric_grid_is_a_smoothing_fixed_point(m6):
    # the Kuhn grid's neighbourhoods are point-symmetric and dyadic: r = 0
    # exactly, every vertex moves onto itself and the equal minimum is accepted
    xyz, tet = inputs.cube_grid(5)
    om = OracleMesh3(xyz, tet, np.tile(m6, (len(xyz), 1)))
    st = om.smooth(0, 2)
    assert st["evaluated"] == 2 * 27 and st["committed"] == st["evaluated"]
    assert np.array_equal(om.export()["xyz"], xyz)


# ---- every class, re-derived ---------------------------------------------------------------

def on_classes(om, phase, check):
    snap = {}

    def hook(ph, rnd, cls, stage):
        if ph != phase:
            return
        if stage == 0:
            snap["d"] = om.export()
            snap["mem"] = om.class_members().copy()
            snap["whole"] = om.class_whole().copy()
        else:
            check(snap["d"], om.export(), snap["mem"], snap["whole"], rnd)

    om.set_hook(hook)


@pytest.mark.parametrize("n,seed,scale", [(7, 1, 0.3), (9, 2, 0.1)])
def test_every_collapse_class_is_the_independent_rule(n, seed, scale):
    mi = inputs.make_mesh3(n, jitter_seed=seed, scale=scale)
    om = OracleMesh3.from_input(mi, seed=seed)
    tally = dict(collapsed=0, kept=0, skipped=0, deferred=0)

    def check(before, after, mem, whole, rnd):
        P = ind.Patches3(before)
        ctx = ctx_of(0, PH_COARSEN, rnd)
        deferred = ind.deferred_set(P, whole, lambda v: (prio(seed, ctx, v), v))
        assert sorted(mem.tolist()) == sorted(set(whole.tolist()) - deferred)
        tally["deferred"] += len(deferred)
        ms = set(mem.tolist())
        for v in mem.tolist():
            assert not (set(P.nbrs[v]) & ms), "members adjacent"
            u, margin = ind.collapse_decision(P, v)
            if margin < MARGIN:
                tally["skipped"] += 1
                continue
            if u is None:
                assert after["valive"][v], f"vertex {v} collapsed but should not"
                tally["kept"] += 1
            else:
                assert not after["valive"][v], f"vertex {v} should collapse onto {u}"
                # its surviving elements now hold u
                for k in P.elems[v]:
                    t = P.tid[k]
                    if after["talive"][t]:
                        assert u in after["tet"][t], f"vertex {v}: element {t} not re-pointed to {u}"
                tally["collapsed"] += 1
        checker3.check_mesh(after, exact=True)

    on_classes(om, PH_COARSEN, check)
    st = om.coarsen()
    assert tally["collapsed"] > 100 and tally["deferred"] > 0, tally
    assert tally["deferred"] == st["deferred"]
    checker3.check_mesh(om.export(), exact=True, rows=om.rows())
    # fixpoint: no vertex has a short legal edge it may collapse along
    d = om.export()
    P = ind.Patches3(dict(d, talive=np.ones(len(d["tet"]), bool)))
    for v in range(om.sizes()[0]):
        u, margin = ind.collapse_decision(P, v)
        assert u is None or margin < MARGIN, f"vertex {v} could still collapse onto {u}"


@pytest.mark.parametrize("n,seed", [(9, 1)])
def test_every_smoothing_move_is_the_independent_rule(n, seed):
    # a tilted layer: every tensor entry is non-zero, so every term of the
    # 3x3 solve matters
    mi = inputs.make_mesh3(n, jitter_seed=seed, amp_y=0.1)
    om = OracleMesh3.from_input(mi, seed=seed)
    tally = dict(moved=0, kept=0, skipped=0)

    def check(before, after, mem, whole, rnd):
        P = ind.Patches3(before)
        for v in mem.tolist():
            ok, p, margin = ind.laplace_decision(P, v)
            if margin < MARGIN:
                tally["skipped"] += 1
                continue
            if ok:
                np.testing.assert_allclose(after["xyz"][v], p, rtol=0, atol=1e-13, err_msg=f"vertex {v}")
                tally["moved"] += 1
            else:
                assert np.array_equal(after["xyz"][v], before["xyz"][v]), f"vertex {v} moved"
                tally["kept"] += 1

    on_classes(om, PH_SMOOTH, check)
    st = om.smooth(0, 2)
    assert tally["moved"] > 50 and tally["kept"] > 0, tally
    assert tally["moved"] + tally["kept"] + tally["skipped"] == st["evaluated"]
    checker3.check_mesh(om.export(), rows=om.rows())


def test_refinement_converges_to_no_long_edge_and_conforms():
    mi = inputs.make_mesh3(5, jitter_seed=4, scale=0.05)
    om = OracleMesh3.from_input(mi, seed=0)
    st = om.refine()
    assert st["converged"] == 1 and st["new_vertices"] > 100
    d = om.export()
    checker3.check_mesh(d, exact=True, rows=om.rows())
    nn_off, nn, _, _ = om.rows()
    a = np.repeat(np.arange(len(nn_off) - 1), np.diff(nn_off))
    assert checker3.metric_len2(d["xyz"], d["metric"], a, nn).max() <= 2.0
    # new vertices are edge midpoints with the edge-mean metric
    V0 = mi.V
    assert d["xyz"].shape[0] == V0 + st["new_vertices"]


def test_sweeps_keep_every_invariant():
    mi = inputs.make_mesh3(7, jitter_seed=5)
    om = OracleMesh3.from_input(mi, seed=5)
    for s in range(2):
        om.sweep(s)
        checker3.check_mesh(om.export(), rows=om.rows())
