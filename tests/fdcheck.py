"""Central-difference protocol for the adjoint of the quality functional.

Vertices: the 64 largest keys (priority, id) of the uint32 priorities drawn
with seed 1 in context 0 over all vertices (SplitMix64, Steele, Lea & Flood
2014, written here with numpy's wrapping uint64 arithmetic; the oracle's
generator is pinned to the published reference vector separately).

Steps: coordinates move by an absolute 1e-7 and the functional evaluated is
the patch-local Q_v (the elements around v), whose derivative in x_v and M_v
equals that of the global Q; metric entries move by 1e-7 times the tensor's
largest diagonal entry (the stored off-diagonal entry may be near zero).

Bound, per entry: |fd - analytic| <= 1e-6 |analytic| + the difference's own
rounding noise, taken as 1e-13 Q_v / step (about a thousand units in the last
place of Q_v, divided by the step). Entries that are not small against that
noise are therefore held to 1e-6 relative.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)
X_STEP = 1e-7
M_REL_STEP = 1e-7
REL = 1e-6
NOISE = 1e-13


def _mix(z):
    z = (z ^ (z >> np.uint64(30))) * M1
    z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def priorities(seed: int, ctx: int, n: int) -> np.ndarray:
    with np.errstate(over="ignore"):
        s = np.uint64(seed) ^ (np.uint64(ctx) << np.uint64(32))
        stream = _mix(s + GAMMA)
        ids = np.arange(n, dtype=np.uint64)
        return (_mix(stream + (ids + np.uint64(1)) * GAMMA) >> np.uint64(32)).astype(np.uint32)


def protocol_vertices(V: int, count: int = 64, seed: int = 1, ctx: int = 0) -> np.ndarray:
    p = priorities(seed, ctx, V).astype(np.int64)
    key = p * (1 << 32) + np.arange(V, dtype=np.int64)
    return np.sort(np.argsort(key)[-count:])


def central_differences(om, v: int, xy0, met0):
    """(dQ_v/dx_v (2), dQ_v/dM_v (3), Q_v, step_x, step_m) by central differences
    of the oracle's patch-local functional; restores the vertex afterwards."""
    x0, y0 = float(xy0[0]), float(xy0[1])
    h = X_STEP
    fx = []
    for dx, dy in ((h, 0.0), (0.0, h)):
        om.set_xy(v, x0 + dx, y0 + dy)
        qp = om.patch_quality(v)
        om.set_xy(v, x0 - dx, y0 - dy)
        qm = om.patch_quality(v)
        fx.append((qp - qm) / (2 * h))
    om.set_xy(v, x0, y0)
    m0 = np.array(met0, float)
    hm = M_REL_STEP * max(abs(m0[0]), abs(m0[2]))
    fm = []
    for k in range(3):
        mp = m0.copy(); mp[k] += hm
        om.set_metric(v, *mp)
        qp = om.patch_quality(v)
        mm = m0.copy(); mm[k] -= hm
        om.set_metric(v, *mm)
        qm = om.patch_quality(v)
        fm.append((qp - qm) / (2 * hm))
    om.set_metric(v, *m0)
    return np.array(fx), np.array(fm), om.patch_quality(v), h, hm


def check_entries(fd, ana, Qv, step, where):
    """Per-entry bound; returns the worst relative gap among entries above the noise."""
    noise = NOISE * abs(Qv) / step
    gap = np.abs(fd - ana)
    bad = gap > REL * np.abs(ana) + noise
    assert not bad.any(), f"{where}: fd {fd} analytic {ana} (noise {noise:.2e})"
    big = np.abs(ana) > noise / REL
    return float((gap[big] / np.abs(ana[big])).max()) if big.any() else 0.0
