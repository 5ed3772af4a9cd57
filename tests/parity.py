"""Helpers that run the same phase sequence on the CPU oracle and on the HIP
path (through the C ABI) and compare the results element by element."""
import numpy as np

from oracle.orc import OracleMesh
from paper_1505_04694_amd import pmesh

STAT_KEYS = ["rounds", "coloured", "evaluated", "deferred", "committed", "colours", "edges", "converged",
             "new_vertices", "new_elements"]
XY_RTOL = 1e-12


def compare_stats(so, sg, where):
    for k in STAT_KEYS:
        assert so[k] == sg[k], f"{where}: stat {k}: oracle {so[k]} gpu {sg[k]}"


def compare_mesh(om, gm, where, rows=True):
    o = om.export()
    g = gm.export()
    assert o["xy"].shape == g["xy"].shape, f"{where}: V oracle {o['xy'].shape} gpu {g['xy'].shape}"
    assert o["tri"].shape == g["tri"].shape, f"{where}: T oracle {o['tri'].shape} gpu {g['tri'].shape}"
    assert np.array_equal(o["valive"], g["valive"]), f"{where}: live vertices differ"
    assert np.array_equal(o["talive"], g["talive"]), f"{where}: live elements differ"
    ta = o["talive"]
    bad = np.nonzero((o["tri"][ta] != g["tri"][ta]).any(1))[0]
    assert bad.size == 0, f"{where}: {bad.size} elements differ, first {np.nonzero(ta)[0][bad[0]]}"
    assert np.array_equal(o["tags"], g["tags"]), f"{where}: tags differ"
    assert np.array_equal(o["metric"], g["metric"]), f"{where}: metric differs"
    va = o["valive"]
    scale = max(1.0, float(np.abs(o["xy"][va]).max()))
    err = float(np.abs(o["xy"][va] - g["xy"][va]).max()) / scale
    assert err <= XY_RTOL, f"{where}: coordinates differ by {err:.3e} relative"
    if rows:
        ro = om.rows()
        rg = gm.rows()
        for a, b, nm in zip(ro, rg, ("nn_off", "nn", "ne_off", "ne")):
            assert np.array_equal(a, b), f"{where}: row array {nm} differs"
    return dict(V=int(va.sum()), T=int(ta.sum()), xy_bitwise=bool(np.array_equal(o["xy"], g["xy"])))


def compare_quality(om, gm, where, grad=True):
    """Q within 1e-12 relative, qmin exactly; the adjoint entry by entry within
    1e-12 relative, with a floor of 1e-12 times the vertex's largest entry of
    the same gradient (both sides sum the same terms in the same order, so in
    practice they are bitwise equal)."""
    Qo, qmo, gxo, gmo = om.quality(grad=True)
    Qg, qmg, gxg, gmg = gm.quality(grad=True)
    assert abs(Qo - Qg) <= 1e-12 * abs(Qo), f"{where}: Q {Qo!r} vs {Qg!r}"
    assert qmo == qmg, f"{where}: qmin {qmo!r} vs {qmg!r}"
    if grad:
        gxg = gxg.cpu().numpy(); gmg = gmg.cpu().numpy()
        for nm, o, g in (("dQ/dx", gxo, gxg), ("dQ/dM", gmo, gmg)):
            floor = 1e-12 * np.abs(o).max(axis=1, keepdims=True)
            bad = np.abs(o - g) > 1e-12 * np.abs(o) + floor
            assert not bad.any(), f"{where}: {nm} differs at {int(bad.sum())} entries, first vertex " \
                                  f"{int(np.nonzero(bad.any(1))[0][0])}"
    return Qo, qmo


def both(mi, seed, quality=0, **kw):
    return (OracleMesh.from_input(mi, seed=seed, quality=quality),
            pmesh.Mesh.from_input(mi, seed=seed, quality=quality, **kw))


def run_sweeps(om, gm, sweeps, smooth_kinds=(0,), rows=True, log=None):
    """Full coarsen -> refine -> swap -> smooth sweeps with a comparison after each phase."""
    for s in range(sweeps):
        kind = smooth_kinds[s % len(smooth_kinds)]
        for name, fo, fg in (
                ("coarsen", lambda: om.coarsen(s), lambda: gm.coarsen(s)),
                ("refine", lambda: om.refine(), lambda: gm.refine()),
                ("swap", lambda: om.swap(s), lambda: gm.swap(s)),
                ("smooth", lambda: om.smooth(s, kind), lambda: gm.smooth(s, kind))):
            so = fo()
            sg = fg()
            where = f"sweep {s} {name}"
            compare_stats(so, sg, where)
            info = compare_mesh(om, gm, where, rows=rows)
            if log is not None:
                log.append((where, so, info))
