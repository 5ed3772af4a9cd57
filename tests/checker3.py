"""Independent checks of tetrahedral meshes (numpy and exact rationals; shares
no code with the oracle or the HIP library)."""
from __future__ import annotations

from fractions import Fraction

import numpy as np

EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def live(mesh: dict):
    tet = mesh["tet"]
    if mesh.get("talive") is not None:
        tet = tet[np.asarray(mesh["talive"], bool)]
    va = mesh.get("valive")
    va = np.ones(mesh["xyz"].shape[0], bool) if va is None else np.asarray(va, bool)
    return mesh["xyz"], tet, mesh["tags"], va


def vol6(xyz, tet):
    p = xyz[tet]
    a, b, c = p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]
    return np.einsum("ni,ni->n", a, np.cross(b, c))


def exact_volume(xyz, tet) -> Fraction:
    """Sum of the signed volumes in exact rational arithmetic."""
    s = Fraction(0)
    F = [[Fraction(float(v)) for v in row] for row in xyz]
    for t in tet.tolist():
        p0, p1, p2, p3 = (F[i] for i in t)
        a = [p1[k] - p0[k] for k in range(3)]
        b = [p2[k] - p0[k] for k in range(3)]
        c = [p3[k] - p0[k] for k in range(3)]
        s += (a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0])
              + a[2] * (b[0] * c[1] - b[1] * c[0]))
    return s / 6


def mat(m6):
    m6 = np.asarray(m6, float)
    return np.stack([np.stack([m6[..., 0], m6[..., 1], m6[..., 2]], -1),
                     np.stack([m6[..., 1], m6[..., 3], m6[..., 4]], -1),
                     np.stack([m6[..., 2], m6[..., 4], m6[..., 5]], -1)], -2)


def mean_ratio(xyz, met, tet):
    """12 (3 sqrt(det M) |K|)^(2/3) / sum_e e^T M e, M the mean of the four
    vertex tensors (matrix form: determinant and quadratic forms by numpy)."""
    M = mat(met[tet].mean(axis=1))
    p = xyz[tet]
    S = np.zeros(len(tet))
    for i, j in EDGES:
        e = p[:, j] - p[:, i]
        S += np.einsum("ni,nij,nj->n", e, M, e)
    vol = vol6(xyz, tet) / 6.0
    vm = np.sqrt(np.linalg.det(M)) * vol
    return 12.0 * np.cbrt((3.0 * vm) ** 2) / S


def metric_len2(xyz, met, a, b):
    M = mat(0.5 * (met[a] + met[b]))
    e = xyz[b] - xyz[a]
    return np.einsum("ni,nij,nj->n", e, M, e)


def faces_of(tet):
    """Oriented boundary faces of each tetrahedron (outward for positive ones)."""
    t = np.asarray(tet)
    return np.concatenate([t[:, [1, 2, 3]], t[:, [0, 3, 2]], t[:, [0, 1, 3]], t[:, [0, 2, 1]]])


def check_mesh(mesh: dict, *, exact: bool = False, rows=None) -> dict:
    """Raise AssertionError on the first violated invariant; return a summary."""
    xyz, tet, tags, vmask = live(mesh)
    V = int(vmask.sum())
    T = tet.shape[0]
    assert T > 0, "no live elements"
    assert tet.min() >= 0 and tet.max() < xyz.shape[0], "element id out of range"
    assert vmask[tet].all(), "live element uses a dead vertex"
    srt = np.sort(tet, axis=1)
    assert (np.diff(srt, axis=1) > 0).all(), "repeated vertex in an element"
    used = np.zeros(xyz.shape[0], bool)
    used[tet.ravel()] = True
    assert (used == vmask).all(), "live vertex without elements (or dead vertex in use)"
    D = vol6(xyz, tet)
    assert (D > 0).all(), f"non-positive volume in {int((D <= 0).sum())} elements"
    # every face in at most two elements, with opposite orientations
    F = faces_of(tet)
    key = np.sort(F, axis=1).astype(np.int64)
    nv = xyz.shape[0] + 1
    k = (key[:, 0] * nv + key[:, 1]) * nv + key[:, 2]
    uniq, inv, cnt = np.unique(k, return_inverse=True, return_counts=True)
    assert cnt.max() <= 2, "face in more than two elements"
    # a face seen twice is seen once per orientation: the cyclic orders differ
    first = np.argmin(F, axis=1)
    canon = np.stack([F[np.arange(len(F)), (first + s) % 3] for s in range(3)], axis=1)
    ck = (canon[:, 0].astype(np.int64) * nv + canon[:, 1]) * nv + canon[:, 2]
    assert np.unique(ck).size == ck.size, "oriented face repeated (orientation or manifoldness)"
    # boundary faces lie on a side of the cube
    bf = F[cnt[inv] == 1]
    common = tags[bf[:, 0]] & tags[bf[:, 1]] & tags[bf[:, 2]]
    assert (common != 0).all(), "boundary face not on the cube's boundary"
    for ax in range(3):
        for bit, val in ((1 << (2 * ax), 0.0), (2 << (2 * ax), 1.0)):
            sel = (common & bit) != 0
            assert (xyz[bf[sel]][..., ax] == val).all(), "tagged vertex off its side"
    E = np.unique(np.sort(np.concatenate([tet[:, [i, j]] for i, j in EDGES]), axis=1), axis=0).shape[0]
    Fn = uniq.size
    assert V - E + Fn - T == 1, f"Euler characteristic {V - E + Fn - T} != 1"
    vol = float(D.sum()) / 6.0
    assert abs(vol - 1.0) < 1e-12, f"total volume {vol!r}"
    if exact:
        assert exact_volume(xyz, tet) == 1, "exact total volume != 1"
    if rows is not None:
        check_rows(mesh, rows)
    return dict(V=V, E=E, F=Fn, T=T, volume=vol)


def rebuild_rows(mesh: dict):
    xyz, tet, _, _ = live(mesh)
    tid = np.arange(mesh["tet"].shape[0])
    if mesh.get("talive") is not None:
        tid = tid[np.asarray(mesh["talive"], bool)]
    nv = xyz.shape[0]
    NE = [[] for _ in range(nv)]
    NN = [set() for _ in range(nv)]
    for t, row in zip(tid.tolist(), tet.tolist()):
        for v in row:
            NE[v].append(t)
            NN[v].update(w for w in row if w != v)
    return [sorted(s) for s in NN], [sorted(s) for s in NE]


def check_rows(mesh: dict, rows):
    nn_off, nn, ne_off, ne = rows
    NN, NE = rebuild_rows(mesh)
    for v in range(len(NN)):
        assert nn[nn_off[v]:nn_off[v + 1]].tolist() == NN[v], f"NN({v})"
        assert ne[ne_off[v]:ne_off[v + 1]].tolist() == NE[v], f"NE({v})"
