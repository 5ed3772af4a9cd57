"""Batched meshes: every mesh of a batch adapted by shared kernel launches
must equal the oracle's run of that mesh alone (exact topology, coordinates
to 1e-12), and the additive op counts must be the sums over the meshes."""
import numpy as np
import pytest

from oracle.orc import OracleMesh
from paper_1505_04694_amd import inputs, pmesh
from tests import checker

pytestmark = pytest.mark.gpu

ADDITIVE = ["coloured", "evaluated", "deferred", "committed", "edges", "new_vertices", "new_elements"]


def small_batch(count, seed=2, nmax=65):
    ps = inputs.batch_params(count, seed)
    return [inputs.make_mesh(min(p["n"], nmax), amp=p["amp"], width=p["width"], ht=p["ht"]) for p in ps]


def compare_one(o, g, where):
    ta = o["talive"]
    assert o["xy"].shape == g["xy"].shape, f"{where}: V {o['xy'].shape} vs {g['xy'].shape}"
    assert o["tri"].shape == g["tri"].shape, f"{where}: T {o['tri'].shape} vs {g['tri'].shape}"
    assert np.array_equal(o["valive"], g["valive"]) and np.array_equal(ta, g["talive"]), where
    assert np.array_equal(o["tri"][ta], g["tri"][ta]), f"{where}: elements differ"
    assert np.array_equal(o["tags"], g["tags"]) and np.array_equal(o["metric"], g["metric"]), where
    va = o["valive"]
    err = np.abs(o["xy"][va] - g["xy"][va]).max() / max(1.0, np.abs(o["xy"][va]).max())
    assert err <= 1e-12, f"{where}: coordinates {err:.2e}"


@pytest.mark.parametrize("count,nmax", [(6, 33), (24, 65)])
def test_batch_equals_solo_oracle_runs(count, nmax):
    mis = small_batch(count, nmax=nmax)
    gb = pmesh.Batch.from_inputs(mis, seed=2)
    oms = [OracleMesh.from_input(mi, seed=2) for mi in mis]
    for s in range(2):
        kind = s % 2
        for name, fo, fg in (
                ("coarsen", lambda om: om.coarsen(s), lambda: gb.coarsen(s)),
                ("refine", lambda om: om.refine(), lambda: gb.refine()),
                ("swap", lambda om: om.swap(s), lambda: gb.swap(s)),
                ("smooth", lambda om: om.smooth(s, kind), lambda: gb.smooth(s, kind))):
            so = [fo(om) for om in oms]
            sg = fg()
            for k in ADDITIVE:
                assert sum(x[k] for x in so) == sg[k], f"sweep {s} {name}: {k}"
            assert max(x["rounds"] for x in so) == sg["rounds"], f"sweep {s} {name}: rounds"
            for i, om in enumerate(oms):
                compare_one(om.export(), gb.export_mesh(i), f"sweep {s} {name} mesh {i}")
    Qg, qg = gb.quality_per_mesh()
    for i, om in enumerate(oms):
        Q, q = om.quality()
        assert abs(Q - Qg[i]) <= 1e-12 * abs(Q) and q == qg[i]
        checker.check_mesh(gb.export_mesh(i), exact=True)


def test_vasilevskii_batch_equals_solo_oracle_runs():
    mis = small_batch(6, nmax=33)
    vas = pmesh.PM_QUALITY_VASILEVSKII
    gb = pmesh.Batch.from_inputs(mis, seed=2, quality=vas)
    oms = [OracleMesh.from_input(mi, seed=2, quality=vas) for mi in mis]
    for s in range(2):
        so = [om.sweep(s, smooth_kind=2 - s) for om in oms]
        sg = gb.sweep(s, smooth_kind=2 - s)
        for ph in ("coarsen", "refine", "swap", "smooth"):
            assert sum(x[ph]["committed"] for x in so) == sg[ph]["committed"], f"sweep {s} {ph}"
        for i, om in enumerate(oms):
            compare_one(om.export(), gb.export_mesh(i), f"sweep {s} mesh {i}")
    Qg, qg = gb.quality_per_mesh()
    for i, om in enumerate(oms):
        Q, q = om.quality()
        assert abs(Q - Qg[i]) <= 1e-12 * abs(Q) and q == qg[i]


def test_batch_equals_plain_gpu_runs_on_uneven_sizes():
    mis = [inputs.make_mesh(n, amp=0.15, width=0.04, ht=0.08) for n in (17, 90, 33, 129, 20)]
    gb = pmesh.Batch.from_inputs(mis, seed=2)
    gms = [pmesh.Mesh.from_input(mi, seed=2) for mi in mis]
    for s in range(2):
        gb.sweep(s)
        for gm in gms:
            gm.sweep(s)
        for i, gm in enumerate(gms):
            compare_one(gm.export(), gb.export_mesh(i), f"sweep {s} mesh {i}")


def test_batch_of_many_small_meshes():
    # more meshes than fit the pinned staging of the batch ranges (the
    # uploads then take the synchronous path); sampled meshes against plain runs
    mis = [inputs.make_mesh(5 + 2 * (i % 3), amp=0.15, width=0.04, ht=0.08) for i in range(2100)]
    gb = pmesh.Batch.from_inputs(mis, seed=2)
    sample = list(range(0, 2100, 150)) + [2099]
    gms = {i: pmesh.Mesh.from_input(mis[i], seed=2) for i in sample}
    for s in range(2):
        gb.sweep(s)
        for gm in gms.values():
            gm.sweep(s)
        for i, gm in gms.items():
            compare_one(gm.export(), gb.export_mesh(i), f"sweep {s} mesh {i}")
