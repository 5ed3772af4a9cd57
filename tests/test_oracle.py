"""Pins of the CPU oracle against what the mathematics and the paper fix.

Nothing here compares the oracle with itself: each test checks a closed form,
a published reference value, an invariant, a hand-derived tiny case, or an
independent (differently computed) evaluation.
"""
import math
import os

import numpy as np
import pytest

from oracle.orc import OracleMesh, ctx_of, prio, splitmix, PH_COARSEN, PH_SWAP, PH_SMOOTH
from paper_1505_04694_amd import inputs
from tests import checker

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
EQ = np.array([[0.0, 0.0], [1.0, 0.0], [0.5, math.sqrt(3.0) / 2.0]])


def one_tri(xy, M, tri=(0, 1, 2)):
    met = np.tile(np.asarray(M, float), (len(xy), 1))
    return OracleMesh(np.asarray(xy, float), np.array([tri], np.int32), met, np.zeros(len(xy), np.uint8))


def quality_of(xy, M):
    return one_tri(xy, M).element_quality()[0]


# ---- priorities --------------------------------------------------------------

def test_splitmix_reference_vector():
    vals = [int(l) for l in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt")) if l.strip() and l[0] != "#"]
    assert [splitmix(1234567, i) for i in range(5)] == vals


def test_priority_bits_balanced():
    ids = range(20000)
    p = np.array([prio(7, ctx_of(1, PH_COARSEN, 3), i) for i in ids], np.uint64)
    bits = ((p[:, None] >> np.arange(32, dtype=np.uint64)[None, :]) & np.uint64(1)).mean(0)
    assert np.all(np.abs(bits - 0.5) < 0.02)
    q = np.array([prio(7, ctx_of(1, PH_COARSEN, 4), i) for i in ids], np.uint64)
    assert (p == q).mean() < 0.001


# ---- quality functional (Sec. 2.2) -------------------------------------------

def test_quality_equilateral_unit_metric():
    assert quality_of(EQ, [1.0, 0.0, 1.0]) == pytest.approx(1.0, abs=1e-15)


def test_quality_right_isosceles():
    q = quality_of([[0, 0], [1, 0], [0, 1]], [1.0, 0.0, 1.0])
    assert q == pytest.approx(math.sqrt(3.0) / 2.0, abs=1e-15)


@pytest.mark.parametrize("seed", range(5))
def test_quality_equilateral_in_metric_space(seed):
    rng = np.random.default_rng(seed)
    F = rng.normal(size=(2, 2))
    if np.linalg.det(F) < 0:
        F[:, 0] *= -1
    M = F.T @ F
    xy = (np.linalg.solve(F, EQ.T)).T          # F x is equilateral
    q = quality_of(xy, [M[0, 0], M[0, 1], M[1, 1]])
    assert q == pytest.approx(1.0, rel=1e-12)


@pytest.mark.parametrize("seed", range(5))
def test_quality_invariances_and_bound(seed):
    rng = np.random.default_rng(100 + seed)
    xy = rng.uniform(0, 1, (3, 2))
    if checker.doubled_areas(xy, np.array([[0, 1, 2]]))[0] < 0:
        xy = xy[[0, 2, 1]]
    F = rng.normal(size=(2, 2))
    M = F.T @ F + 0.1 * np.eye(2)
    m = [M[0, 0], M[0, 1], M[1, 1]]
    q = quality_of(xy, m)
    assert 0 < q <= 1.0 + 1e-15
    assert quality_of(xy, [7.0 * v for v in m]) == pytest.approx(q, rel=1e-13)      # q(cM) = q(M)
    assert quality_of(xy * 0.25 + 0.3, m) == pytest.approx(q, rel=1e-12)              # similarity in x
    # q(F^T F; x) = q(I; F x)
    L = np.linalg.cholesky(M).T                    # M = L^T L
    assert quality_of((L @ xy.T).T, [1.0, 0.0, 1.0]) == pytest.approx(q, rel=1e-12)


def test_quality_matches_matrix_form_on_config0():
    mi = inputs.config0()
    om = OracleMesh.from_input(mi)
    q = om.element_quality()
    d = om.export()
    ref = checker.mean_ratio(d["xy"], d["metric"], d["tri"])
    np.testing.assert_allclose(q, ref, rtol=1e-12)


# ---- generators ------------------------------------------------------------------

@pytest.mark.parametrize("n", [2, 3, 9, 33])
def test_generator_counts(n):
    xy, tri = inputs.grid(n)
    V, T = n * n, 2 * (n - 1) ** 2
    E = 3 * (n - 1) ** 2 + 2 * (n - 1)
    assert xy.shape == (V, 2) and tri.shape == (T, 3)
    mesh = dict(xy=xy, tri=tri, tags=inputs.unit_square_tags(xy))
    s = checker.check_mesh(mesh, exact=True)
    assert (s["V"], s["E"], s["F"]) == (V, E, T)
    if n >= 3:
        deg = np.bincount(np.unique(np.sort(checker.edges_of(tri), 1), axis=0).ravel(), minlength=V)
        inner = mesh["tags"] == 0
        h = np.bincount(deg[inner])
        assert set(np.nonzero(h)[0]) <= {4, 8}


def test_generator_metric_spd_and_layer_symmetry():
    mi = inputs.config2(65)
    m = mi.metric
    assert (m[:, 0] > 0).all() and (m[:, 0] * m[:, 2] - m[:, 1] ** 2 > 0).all()
    xy, _ = inputs.grid(33)
    a = inputs.layer_y(xy)
    b = inputs.layer_x(xy[:, ::-1])                # swap the roles of x and y
    np.testing.assert_allclose(a[:, [2, 1, 0]], b, rtol=1e-12, atol=1e-9)


def test_initial_euclidean_quality():
    xy, tri = inputs.grid(9)
    om = OracleMesh(xy, tri, np.tile([1.0, 0.0, 1.0], (len(xy), 1)))
    np.testing.assert_allclose(om.element_quality(), math.sqrt(3) / 2, rtol=1e-15)


# ---- colouring (Sec. 3.2) ------------------------------------------------------------

def jones_plassmann(nbrs, active, key):
    """Textbook JP iteration: in each step every uncoloured vertex that beats all
    its uncoloured active neighbours takes the smallest colour unused by its
    coloured active neighbours."""
    col = {v: -1 for v in active}
    left = set(active)
    while left:
        ready = [v for v in left if all(key[w] < key[v] for w in nbrs[v] if w in left)]
        for v in ready:
            used = {col[w] for w in nbrs[v] if w in col and col[w] >= 0}
            c = 0
            while c in used:
                c += 1
            col[v] = c
        left -= set(ready)
    return col


@pytest.mark.parametrize("seed,frac", [(0, 1.0), (3, 0.6), (11, 0.3)])
def test_colouring_equals_jones_plassmann(seed, frac):
    mi = inputs.make_mesh(17, layers=2, jitter_seed=seed)
    om = OracleMesh.from_input(mi, seed=seed)
    rng = np.random.default_rng(seed)
    active = (rng.uniform(size=mi.V) < frac).astype(np.uint8)
    ctx = ctx_of(2, PH_SWAP, 5)
    col, ncol = om.colour(active, ctx)
    nn_off, nn, _, _ = om.rows()
    nbrs = {v: set(nn[nn_off[v]:nn_off[v + 1]].tolist()) for v in range(mi.V)}
    act = [v for v in range(mi.V) if active[v]]
    key = {v: (prio(seed, ctx, v), v) for v in act}
    ref = jones_plassmann(nbrs, act, key)
    for v in range(mi.V):
        assert col[v] == (ref[v] if active[v] else -1)
    assert ncol == max(ref.values()) + 1
    # proper colouring, bounded by max degree + 1
    for v in act:
        for w in nbrs[v]:
            if active[w]:
                assert col[v] != col[w]
    assert ncol <= max(len(nbrs[v] & set(act)) for v in act) + 1


# ---- hand-derived tiny cases (Sec. 2.4) ----------------------------------------------

SQ = np.array([[0, 0], [1, 0], [1, 1], [0, 1], [0.5, 0.5]], float)
SQ_TRI = np.array([[0, 1, 4], [1, 2, 4], [2, 3, 4], [3, 0, 4]], np.int32)


def sq_mesh(c, centre=(0.5, 0.5)):
    xy = SQ.copy()
    xy[4] = centre
    return OracleMesh(xy, SQ_TRI, np.tile([c, 0.0, c], (5, 1)), seed=0)


def test_collapse_centre_onto_smallest_corner():
    # centre edges have L^2 = 0.5c; all four tie, so corner 0 is taken; the two
    # elements on edge (4,0) die and the other two are re-pointed to 0
    om = sq_mesh(0.99)
    st = om.coarsen()
    assert st["committed"] == 1
    d = om.export()
    assert d["tri"].tolist() == [[0, 1, 2], [0, 2, 3]]
    assert d["xy"].shape[0] == 4


def test_collapse_threshold_is_strict():
    om = sq_mesh(1.0)                      # L^2 = 0.5 exactly: not short
    st = om.coarsen()
    assert st["committed"] == 0 and om.sizes() == (5, 4)


def test_collapse_blocked_by_quality():
    om = sq_mesh(0.99)                     # re-pointed elements have q = sqrt(3)/2
    st = om.coarsen(q_min=0.87)
    assert st["committed"] == 0 and om.sizes() == (5, 4)
    om = sq_mesh(0.99)
    assert om.coarsen(q_min=0.86)["committed"] == 1


def test_collapse_nearest_candidate_first():
    om = sq_mesh(0.5, centre=(0.6, 0.4))   # corner 1 = (1, 0) is nearest
    om.coarsen()
    d = om.export()
    assert sorted(map(tuple, d["tri"].tolist())) == [(0, 1, 3), (1, 2, 3)]


def test_collapse_boundary_vertex_stays_on_its_side():
    # vertex 1 sits on x = 0; it may only collapse onto 0 or 2 (same side)
    xy = np.array([[0, 0], [0, 0.5], [0, 1], [1, 0], [1, 1]], float)
    tri = np.array([[0, 3, 1], [1, 3, 4], [1, 4, 2]], np.int32)
    om = OracleMesh(xy, tri, np.tile([0.3, 0.0, 0.3], (5, 1)))
    st = om.coarsen()
    assert st["committed"] == 1
    d = om.export()
    # 1 -> 0: (0,3,1) dies, (1,3,4) -> (0,3,4), (1,4,2) -> (0,4,2); then the
    # stable renumbering maps 2->1, 3->2, 4->3
    assert d["tri"].tolist() == [[0, 2, 3], [0, 3, 1]]
    assert d["xy"].tolist() == [[0, 0], [0, 1], [1, 0], [1, 1]]


RT = np.array([[0, 0], [1, 0], [0, 1]], float)


def test_refine_three_splits():
    # M = 3I: edge L^2 = 3, 3, 6 > 2. Mid-points get ids 3 (0-1), 4 (0-2), 5 (1-2);
    # children (0,3,4), (3,1,5), (4,5,2), (3,5,4), first keeps the parent id
    om = one_tri(RT, [3.0, 0.0, 3.0])
    st = om.refine()
    d = om.export()
    assert st["new_vertices"] == 3 and st["new_elements"] == 3 and st["rounds"] == 1
    assert d["xy"][3:].tolist() == [[0.5, 0], [0, 0.5], [0.5, 0.5]]
    assert d["tri"].tolist() == [[0, 3, 4], [1, 5, 3], [2, 4, 5], [3, 5, 4]]


def test_refine_one_split():
    # M = 1.5I: only the hypotenuse (L^2 = 3) splits
    om = one_tri(RT, [1.5, 0.0, 1.5])
    om.refine()
    d = om.export()
    assert d["tri"].tolist() == [[0, 1, 3], [0, 3, 2]]
    assert d["xy"][3].tolist() == [0.5, 0.5]


def test_refine_two_splits_shorter_diagonal():
    # M = diag(3, 1.5): edges 0-1 (L^2 3) and 1-2 (4.5) split, 0-2 (1.5) does not.
    # Corner child (3,1,4); the quad 2,0,3,4 is cut along 0-4 (L^2 1.125) rather
    # than 2-3 (2.25)
    om = one_tri(RT, [3.0, 0.0, 1.5])
    om.refine()
    d = om.export()
    assert d["tri"].tolist() == [[1, 4, 3], [0, 4, 2], [0, 3, 4]]


def test_swap_flat_quad():
    # flat quad: diagonal 0-2 gives two slivers; the flip to 1-3 improves the minimum
    xy = np.array([[0, 0], [0.5, -0.1], [1, 0], [0.5, 0.1]], float)
    om = OracleMesh(xy, np.array([[0, 1, 2], [0, 2, 3]], np.int32), np.tile([1.0, 0, 1.0], (4, 1)),
                    np.zeros(4, np.uint8))
    q0 = om.element_quality().min()
    st = om.swap()
    d = om.export()
    assert st["committed"] == 1 and st["converged"] == 1
    assert sorted(map(tuple, d["tri"].tolist())) == [(0, 1, 3), (1, 2, 3)]
    assert om.element_quality().min() > q0


def test_swap_keeps_good_diagonal():
    xy = np.array([[0, 0], [0.5, -0.1], [1, 0], [0.5, 0.1]], float)
    om = OracleMesh(xy, np.array([[0, 1, 3], [1, 2, 3]], np.int32), np.tile([1.0, 0, 1.0], (4, 1)),
                    np.zeros(4, np.uint8))
    assert om.swap()["committed"] == 0


def test_smooth_moves_to_metric_centroid():
    om = sq_mesh(1.0, centre=(0.3, 0.4))
    st = om.smooth(kind=0)
    assert st["committed"] == 1
    np.testing.assert_allclose(om.export()["xy"][4], [0.5, 0.5], atol=1e-15)


def test_smooth_constant_metric_grid_is_fixed_point():
    xy, tri = inputs.grid(17)
    om = OracleMesh(xy, tri, np.tile([40.0, 3.0, 90.0], (len(xy), 1)))
    om.smooth(kind=0, sweeps=2)
    assert np.array_equal(om.export()["xy"], xy)


def test_create_rejects_invalid():
    xy = np.array([[0, 0], [1, 0], [0, 1]], float)
    met = np.tile([1.0, 0, 1.0], (3, 1))
    with pytest.raises(ValueError):
        OracleMesh(xy, np.array([[0, 2, 1]], np.int32), met)        # clockwise
    with pytest.raises(ValueError):
        OracleMesh(xy, np.array([[0, 1, 3]], np.int32), met)        # id out of range
    with pytest.raises(ValueError):
        OracleMesh(xy, np.array([[0, 1, 2]], np.int32), np.tile([1.0, 2.0, 1.0], (3, 1)))  # not SPD
