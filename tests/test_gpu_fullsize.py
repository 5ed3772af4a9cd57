"""Parity at the workloads' full sizes, in the launch configuration bench.py
times: the 1025 x 1025 one-layer mesh over three adaptation sweeps, and the
benchmark step on the 2049 x 2049 jittered two-layer mesh with a comparison
after every phase (including the adjoint at all 4.2M vertices)."""
import numpy as np
import pytest

from paper_1505_04694_amd import inputs
from tests import checker, fdcheck
from tests.parity import both, compare_mesh, compare_quality, compare_stats, run_sweeps

pytestmark = pytest.mark.gpu


def test_config1_three_sweeps():
    om, gm = both(inputs.config1(), 0)
    compare_mesh(om, gm, "create", rows=True)
    run_sweeps(om, gm, 3, smooth_kinds=(0,))
    checker.check_mesh(gm.export(), exact=True, rows=gm.rows())
    compare_quality(om, gm, "end")


def test_config2_benchmark_step():
    mi = inputs.config2()
    om, gm = both(mi, 1)
    compare_quality(om, gm, "initial")
    # the adjoint against central differences at the 64 protocol vertices
    _, _, gx, gmet = gm.quality(grad=True)
    gx, gmet = gx.cpu().numpy(), gmet.cpu().numpy()
    for v in fdcheck.protocol_vertices(mi.V):
        v = int(v)
        fx, fm, Qv, hx, hm = fdcheck.central_differences(om, v, mi.xy[v], mi.metric[v])
        fdcheck.check_entries(fx, gx[v], Qv, hx, f"dQ/dx at {v}")
        fdcheck.check_entries(fm, gmet[v], Qv, hm, f"dQ/dM at {v}")
    del gx, gmet
    for name, fo, fg in (
            ("smooth plain", lambda: om.smooth(0, 0, 1), lambda: gm.smooth(0, 0, 1)),
            ("smooth gradient", lambda: om.smooth(0, 1, 1), lambda: gm.smooth(0, 1, 1)),
            ("coarsen", lambda: om.coarsen(0), lambda: gm.coarsen(0)),
            ("refine", lambda: om.refine(), lambda: gm.refine()),
            ("swap", lambda: om.swap(0), lambda: gm.swap(0)),
            ("smooth", lambda: om.smooth(0, 0, 1), lambda: gm.smooth(0, 0, 1))):
        compare_stats(fo(), fg(), name)
        compare_mesh(om, gm, name, rows=name not in ("smooth plain", "smooth gradient"))
    compare_quality(om, gm, "end")
    checker.check_mesh(gm.export(), exact=False, rows=gm.rows())


def test_config4_two_sweeps_match_the_oracle_result():
    """The 4097 x 4097 workload (two sweeps, gradient smoothing) against the
    oracle's stored result (tests/golden/make_config4.py): every phase's op
    counts, and the final topology, tags, metric and coordinates."""
    import json
    import os
    import torch
    from paper_1505_04694_amd import pmesh
    from tests.golden.make_config4 import N, SEED, SWEEPS, summary
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "config4_4097.json")))
    mi = inputs.config4(N)
    assert mi.digest() == gold["input"]
    dev = torch.device("cuda")
    gm = pmesh.Mesh(*(torch.from_numpy(a).to(dev) for a in (mi.xy, mi.tri, mi.metric, mi.tags)), seed=SEED)
    for s in range(SWEEPS):
        g = gold["phases"][s]
        for name, fg in (("coarsen", lambda: gm.coarsen(s)), ("refine", lambda: gm.refine()),
                         ("swap", lambda: gm.swap(s)), ("smooth", lambda: gm.smooth(s, 1, 1))):
            compare_stats(g[name], fg(), f"sweep {s} {name}")
    got = summary(gm.export())
    want = gold["final"]
    for k in ("V", "T", "tri", "tags", "metric"):
        assert got[k] == want[k], k
    if got["xy"] != want["xy"]:
        assert abs(got["xy_sum"] - want["xy_sum"]) <= 1e-12 * abs(want["xy_sum"])
    Q, qmin = gm.quality()
    assert abs(Q - gold["quality"][0]) <= 1e-12 * abs(Q) and qmin == gold["quality"][1]


def test_full_batch_matches_the_oracle_golden():
    """The whole batched workload (256 meshes of n log-uniform in [17, 513],
    two sweeps, plain smoothing) through one batched handle, as the benchmark
    runs it, against the oracle's run of every mesh alone
    (tests/golden/make_batch256.py): the summed op counts, and each mesh's
    final topology, tags and coordinates."""
    import json
    import os
    from paper_1505_04694_amd import pmesh
    from tests.golden.make_batch256 import COUNT, SEED, SWEEPS, summary
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "batch256.json")))
    mis = inputs.config3(COUNT, SEED)
    assert [mi.n for mi in mis] == [m["n"] for m in gold["meshes"]]
    gb = pmesh.Batch.from_inputs(mis, seed=SEED)
    ops = 0
    for s in range(SWEEPS):
        tr = gb.sweep(s)
        ops += sum(st["coloured"] + st["evaluated"] + st["edges"] for st in tr.values())
    assert ops == sum(m["ops"] for m in gold["meshes"])
    for i, m in enumerate(gold["meshes"]):
        got, want = summary(gb.export_mesh(i)), m["final"]
        for k in ("V", "T", "tri", "tags"):
            assert got[k] == want[k], f"mesh {i} (n = {m['n']}): {k}"
        if got["xy"] != want["xy"]:
            assert abs(got["xy_sum"] - want["xy_sum"]) <= 1e-12 * abs(want["xy_sum"]), f"mesh {i}: coordinates"
    gb.close()
