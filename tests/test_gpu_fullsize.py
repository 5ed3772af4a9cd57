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
