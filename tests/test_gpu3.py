"""Parity of the tetrahedral HIP path (include/pm3.h, called through the C ABI)
with the CPU oracle: rows, colourings, and every phase's element arrays, live
flags and op counts exactly; coordinates bitwise (they come out equal when the
device rounds like the host); quality sum within 1e-12 and minimum within
1e-14 (the reported value takes a cube root)."""
import numpy as np
import pytest

from oracle.orc import OracleMesh3, ctx_of
from paper_1505_04694_amd import inputs
from paper_1505_04694_amd.pmesh3 import Mesh3
from tests import checker3

pytestmark = pytest.mark.gpu

CASES = [
    ("k5_j4", lambda: inputs.make_mesh3(5, jitter_seed=4, scale=0.05), 4),
    ("k7_j1", lambda: inputs.make_mesh3(7, jitter_seed=1, scale=0.3), 1),
    ("k9_j2", lambda: inputs.make_mesh3(9, jitter_seed=2, scale=0.1), 2),
    ("k9_layer", lambda: inputs.make_mesh3(9, jitter_seed=3), 3),
]
STAT_KEYS = ["rounds", "coloured", "evaluated", "deferred", "committed", "colours", "edges", "converged",
             "new_vertices", "new_elements"]


def both(mi, seed):
    return OracleMesh3.from_input(mi, seed=seed), Mesh3.from_input(mi, seed=seed)


def compare(om, gm, where):
    a, b = om.export(), gm.export()
    assert a["tet"].shape == b["tet"].shape and a["xyz"].shape == b["xyz"].shape, f"{where}: sizes"
    assert np.array_equal(a["valive"], b["valive"]) and np.array_equal(a["talive"], b["talive"]), where
    ta = a["talive"]
    assert np.array_equal(a["tet"][ta], b["tet"][ta]), f"{where}: elements differ"
    assert np.array_equal(a["tags"], b["tags"]) and np.array_equal(a["metric"], b["metric"]), where
    va = a["valive"]
    assert np.array_equal(a["xyz"][va], b["xyz"][va]), f"{where}: coordinates differ"
    ro, rg = om.rows(), gm.rows()
    for x, y in zip(ro, rg):
        assert np.array_equal(x, y), f"{where}: rows differ"


def compare_stats(so, sg, where):
    for k in STAT_KEYS:
        assert so[k] == sg[k], f"{where}: {k} {so[k]} vs {sg[k]}"


def compare_quality(om, gm, where):
    Qo, qo = om.quality()
    Qg, qg = gm.quality()
    assert abs(Qo - Qg) <= 1e-12 * abs(Qo), f"{where}: Q {Qo!r} vs {Qg!r}"
    assert abs(qo - qg) <= 1e-14 * abs(qo), f"{where}: qmin {qo!r} vs {qg!r}"


@pytest.mark.parametrize("name,make,seed", CASES)
def test_create_rows_and_colouring(name, make, seed):
    mi = make()
    om, gm = both(mi, seed)
    compare(om, gm, "create")
    rng = np.random.default_rng(seed)
    for ctx, frac in ((0, None), (ctx_of(2, 1, 5), 0.5)):
        act = None if frac is None else (rng.uniform(size=mi.V) < frac).astype(np.uint8)
        co, no = om.colour(act, ctx)
        cg, ng = gm.colour(act, ctx)
        assert no == ng and np.array_equal(co, cg), f"colouring ctx={ctx}"
    compare_quality(om, gm, "create")


@pytest.mark.parametrize("name,make,seed", CASES)
def test_phases_match_the_oracle(name, make, seed):
    mi = make()
    om, gm = both(mi, seed)
    for s in range(2):
        for ph, fo, fg in (("coarsen", lambda: om.coarsen(s), lambda: gm.coarsen(s)),
                           ("refine", lambda: om.refine(), lambda: gm.refine()),
                           ("smooth", lambda: om.smooth(s, 2), lambda: gm.smooth(s, 2))):
            where = f"sweep {s} {ph}"
            compare_stats(fo(), fg(), where)
            compare(om, gm, where)
    checker3.check_mesh(gm.export(), rows=gm.rows())
    compare_quality(om, gm, "end")


def test_round_cap_leaves_a_valid_mesh():
    mi = inputs.make_mesh3(9, jitter_seed=2, scale=0.1)
    om, gm = both(mi, 2)
    so, sg = om.coarsen(max_rounds=1), gm.coarsen(max_rounds=1)
    compare_stats(so, sg, "one round")
    assert sg["status"] == "PM_W_NOT_CONVERGED"
    compare(om, gm, "one round")
    checker3.check_mesh(gm.export(), exact=True, rows=gm.rows())


def test_device_arrays_and_invalid_meshes():
    import torch
    mi = inputs.make_mesh3(5, jitter_seed=4, scale=0.05)
    dev = torch.device("cuda:0")
    gm = Mesh3(torch.from_numpy(mi.xyz).to(dev), torch.from_numpy(mi.tet).to(dev),
               torch.from_numpy(mi.metric).to(dev), torch.from_numpy(mi.tags).to(dev), seed=4)
    om = OracleMesh3.from_input(mi, seed=4)
    compare(om, gm, "create from device arrays")
    from paper_1505_04694_amd.pmesh import PMError
    bad = mi.tet.copy()
    bad[0, [1, 2]] = bad[0, [2, 1]]                 # negative volume
    with pytest.raises(PMError):
        Mesh3(mi.xyz, bad, mi.metric, mi.tags)


@pytest.mark.parametrize("n,target", [(11, 8000.0), (17, 40000.0)])
def test_psi_benchmark_adaptation_matches_the_oracle(n, target):
    """The 3D benchmark's procedure at reduced size: psi extruded along z,
    two iterations of coarsen then refine, then a smoothing sweep; every phase
    compared with the oracle."""
    mi = inputs.psi_start3(n, target=target)
    om, gm = both(mi, 0)
    for it in range(2):
        compare_stats(om.coarsen(it), gm.coarsen(it), f"iteration {it} coarsen")
        compare(om, gm, f"iteration {it} coarsen")
        compare_stats(om.refine(), gm.refine(), f"iteration {it} refine")
        compare(om, gm, f"iteration {it} refine")
    compare_stats(om.smooth(0, 1), gm.smooth(0, 1), "smooth")
    compare(om, gm, "smooth")
    compare_quality(om, gm, "end")
    checker3.check_mesh(gm.export(), rows=gm.rows())


def test_psi_benchmark_full_size_matches_the_oracle_result():
    """The 3D benchmark procedure at its full size (29^3 Kuhn grid, about 50^3
    tetrahedra, adapted to 1.4 M) against the oracle's stored result
    (tests/golden/make_psi3.py): every phase's op counts and the final
    topology, tags, metric and coordinates."""
    import json
    import os
    import torch
    from tests.golden.make_psi3 import ITERATIONS, N, SEED, TARGET, summary
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "psi3_29.json")))
    mi = inputs.psi_start3(N, target=TARGET)
    assert mi.digest() == gold["input"]
    dev = torch.device("cuda")
    gm = Mesh3(*(torch.from_numpy(a).to(dev) for a in (mi.xyz, mi.tet, mi.metric, mi.tags)), seed=SEED)
    for it in range(ITERATIONS):
        g = gold["phases"][it]
        compare_stats(g["coarsen"], gm.coarsen(it), f"iteration {it} coarsen")
        compare_stats(g["refine"], gm.refine(), f"iteration {it} refine")
    compare_stats(gold["smooth"], gm.smooth(0, 1), "smooth")
    got, want = summary(gm.export()), gold["final"]
    for k in ("V", "T", "tet", "tags", "metric"):
        assert got[k] == want[k], k
    if got["xyz"] != want["xyz"]:
        assert abs(got["xyz_sum"] - want["xyz_sum"]) <= 1e-12 * abs(want["xyz_sum"])
    Q, qmin = gm.quality()
    assert abs(Q - gold["quality"][0]) <= 1e-12 * abs(Q) and abs(qmin - gold["quality"][1]) <= 1e-14 * qmin


def test_commit_out_of_room_rebuilds_and_matches_the_oracle():
    """Pools with the least headroom: row commits of the coarsening run out of
    room, the host rebuilds every row from the elements and runs the round's
    later classes again. Every phase still equals the oracle's."""
    mi = inputs.psi_start3(17, target=40000.0)
    om = OracleMesh3.from_input(mi, seed=0)
    gm = Mesh3.from_input(mi, seed=0, pool_headroom=1.0)
    rebuilt = 0
    for it in range(2):
        sg = gm.coarsen(it)
        compare_stats(om.coarsen(it), sg, f"iteration {it} coarsen")
        compare(om, gm, f"iteration {it} coarsen")
        rebuilt += sg["room_rebuilds"]
        compare_stats(om.refine(), gm.refine(), f"iteration {it} refine")
        compare(om, gm, f"iteration {it} refine")
    assert rebuilt > 0
    checker3.check_mesh(gm.export(), rows=gm.rows())


def _star(levels=3):
    """Tetrahedra joining the centre of the unit cube to the faces of an
    icosphere (the icosahedron, each face cut into four `levels` times, points
    pushed onto the sphere of radius 0.45): the centre is in every element."""
    t = (1 + 5 ** 0.5) / 2
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6),
         (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10),
         (8, 6, 7), (9, 8, 1)]
    v = [np.array(p, float) / np.linalg.norm(p) for p in v]
    for _ in range(levels):
        mid = {}

        def m(a, b):
            k = (min(a, b), max(a, b))
            if k not in mid:
                p = v[a] + v[b]
                v.append(p / np.linalg.norm(p))
                mid[k] = len(v) - 1
            return mid[k]
        nf = []
        for a, b, c in f:
            ab, bc, ca = m(a, b), m(b, c), m(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = nf
    xyz = np.vstack([[0.5, 0.5, 0.5], 0.5 + 0.45 * np.array(v)])
    tet = np.hstack([np.zeros((len(f), 1), int), np.array(f) + 1]).astype(np.int32)
    return xyz, tet


def test_a_vertex_in_every_element():
    """A centre vertex in all 1280 elements (642 neighbours): its sorted row
    takes the serial form, and a coarsening class that changes it has rows
    past the wavefront row commit, so the round falls back to a full row
    rebuild. Rows, colourings and every phase equal the oracle's."""
    xyz, tet = _star(3)
    met = np.tile([25.0, 0, 0, 25.0, 0, 25.0], (len(xyz), 1))
    tags = np.zeros(len(xyz), np.uint8)
    om, gm = OracleMesh3(xyz, tet, met, tags, seed=5), Mesh3(xyz, tet, met, tags, seed=5)
    compare(om, gm, "create")
    assert np.diff(gm.rows()[2])[0] == len(tet)
    co, no = om.colour(None, 0)
    cg, ng = gm.colour(None, 0)
    assert no == ng and np.array_equal(co, cg)
    sg = gm.coarsen(0)
    compare_stats(om.coarsen(0), sg, "coarsen")
    compare(om, gm, "coarsen")
    assert sg["room_rebuilds"] > 0
    for ph, fo, fg in (("refine", lambda: om.refine(), lambda: gm.refine()),
                       ("smooth", lambda: om.smooth(0, 1), lambda: gm.smooth(0, 1))):
        compare_stats(fo(), fg(), ph)
        compare(om, gm, ph)
    compare_quality(om, gm, "end")


def test_single_element_and_nothing_to_do():
    # one tetrahedron: nothing to collapse (every vertex a cube corner), one
    # refinement pass of its long edges, smoothing of no interior vertex
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    tet = np.array([[0, 1, 2, 3]], np.int32)
    met = np.tile([3.0, 0, 0, 3.0, 0, 3.0], (4, 1))
    om = OracleMesh3(xyz, tet, met, np.zeros(4, np.uint8))
    gm = Mesh3(xyz, tet, met, np.zeros(4, np.uint8))
    for ph, fo, fg in (("coarsen", lambda: om.coarsen(), lambda: gm.coarsen()),
                       ("refine", lambda: om.refine(max_passes=1), lambda: gm.refine(max_passes=1)),
                       ("smooth", lambda: om.smooth(0, 1), lambda: gm.smooth(0, 1))):
        compare_stats(fo(), fg(), ph)
        compare(om, gm, ph)
    compare_quality(om, gm, "end")
    # no short edge (every L^2 >= 1 under 4 I on the 3^3 grid): nothing to do,
    # the phase converges at once and the mesh is unchanged
    mi = inputs.make_mesh3(3)
    gm2 = Mesh3(mi.xyz, mi.tet, np.tile([4.0, 0, 0, 4.0, 0, 4.0], (mi.V, 1)), mi.tags)
    st = gm2.coarsen()
    assert st["committed"] == 0 and st["converged"] == 1 and gm2.sizes() == (mi.V, mi.T)
    assert np.array_equal(gm2.export()["xyz"], mi.xyz)
