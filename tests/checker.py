"""Independent mesh invariant checker (numpy; shares no code with the oracle or
the HIP library).

Checks that a triangle mesh of the unit square is a valid, conforming,
consistently oriented triangulation, and that adjacency rows equal a rebuild
from the elements. Exact area uses rational arithmetic on the binary64
coordinates, so "total area 1" is tested without rounding.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

X0, X1, Y0, Y1 = 1, 2, 4, 8


def live(mesh: dict):
    """Return (xy, tri, tags, vmask) restricted to live elements; ids unchanged."""
    tri = mesh["tri"]
    ta = mesh.get("talive")
    if ta is not None:
        tri = tri[np.asarray(ta, bool)]
    va = mesh.get("valive")
    vmask = np.ones(mesh["xy"].shape[0], bool) if va is None else np.asarray(va, bool)
    return mesh["xy"], tri, mesh["tags"], vmask


def doubled_areas(xy, tri):
    p0, p1, p2 = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    return (p1[:, 0] - p0[:, 0]) * (p2[:, 1] - p0[:, 1]) - (p2[:, 0] - p0[:, 0]) * (p1[:, 1] - p0[:, 1])


def exact_area(xy, tri) -> Fraction:
    """Sum of triangle areas in exact rational arithmetic."""
    fx = [Fraction(float(v)) for v in xy[:, 0]]
    fy = [Fraction(float(v)) for v in xy[:, 1]]
    tot = Fraction(0)
    for a, b, c in tri.tolist():
        tot += (fx[b] - fx[a]) * (fy[c] - fy[a]) - (fx[c] - fx[a]) * (fy[b] - fy[a])
    return tot / 2


def edges_of(tri):
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    return e


def check_mesh(mesh: dict, *, exact: bool = False, rows=None) -> dict:
    """Raise AssertionError on the first violated invariant; return a summary."""
    xy, tri, tags, vmask = live(mesh)
    V = int(vmask.sum())
    F = tri.shape[0]
    assert F > 0, "no live elements"
    assert tri.min() >= 0 and tri.max() < xy.shape[0], "element id out of range"
    assert vmask[tri].all(), "live element uses a dead vertex"
    assert (tri[:, 0] != tri[:, 1]).all() and (tri[:, 1] != tri[:, 2]).all() and (tri[:, 0] != tri[:, 2]).all()
    used = np.zeros(xy.shape[0], bool)
    used[tri.ravel()] = True
    assert (used == vmask).all(), "live vertex without elements (or dead vertex in use)"
    D = doubled_areas(xy, tri)
    assert (D > 0).all(), f"non-positive area in {int((D <= 0).sum())} elements"
    # directed edges unique => consistent orientation and at most two elements per edge
    de = edges_of(tri).astype(np.int64)
    key = de[:, 0] * (xy.shape[0] + 1) + de[:, 1]
    assert np.unique(key).size == key.size, "directed edge repeated (orientation or manifoldness)"
    ue = np.sort(de, axis=1)
    ukey = ue[:, 0] * (xy.shape[0] + 1) + ue[:, 1]
    uniq, cnt = np.unique(ukey, return_counts=True)
    assert cnt.max() <= 2, "edge in more than two elements"
    E = uniq.size
    # boundary edges must lie on one side of the unit square
    bkeys = uniq[cnt == 1]
    ba = bkeys // (xy.shape[0] + 1)
    bb = bkeys % (xy.shape[0] + 1)
    common = tags[ba] & tags[bb]
    assert (common != 0).all(), "boundary edge not on the square's boundary"
    for bit, col, val in ((X0, 0, 0.0), (X1, 0, 1.0), (Y0, 1, 0.0), (Y1, 1, 1.0)):
        sel = (common & bit) != 0
        assert (xy[ba[sel], col] == val).all() and (xy[bb[sel], col] == val).all(), "tagged vertex off its side"
    assert V - E + F == 1, f"Euler characteristic {V - E + F} != 1"
    area = float(D.sum()) * 0.5
    assert abs(area - 1.0) < 1e-12, f"total area {area!r}"
    if exact:
        assert exact_area(xy, tri) == 1, "exact total area != 1"
    if rows is not None:
        check_rows(mesh, rows)
    return dict(V=V, E=E, F=F, area=area)


def rebuild_rows(mesh: dict):
    xy, tri, _, vmask = live(mesh)
    tid = np.arange(mesh["tri"].shape[0])
    if mesh.get("talive") is not None:
        tid = tid[np.asarray(mesh["talive"], bool)]
    nv = xy.shape[0]
    NE = [[] for _ in range(nv)]
    NN = [set() for _ in range(nv)]
    for t, (a, b, c) in zip(tid.tolist(), tri.tolist()):
        for v, o1, o2 in ((a, b, c), (b, c, a), (c, a, b)):
            NE[v].append(t)
            NN[v].add(o1)
            NN[v].add(o2)
    return [sorted(s) for s in NN], [sorted(s) for s in NE]


def check_rows(mesh: dict, rows):
    """rows = (nn_off, nn, ne_off, ne) CSR over all vertex slots."""
    nn_off, nn, ne_off, ne = rows
    NN, NE = rebuild_rows(mesh)
    for v in range(len(NN)):
        got_nn = nn[nn_off[v]:nn_off[v + 1]].tolist()
        got_ne = ne[ne_off[v]:ne_off[v + 1]].tolist()
        assert got_nn == NN[v], f"NN row of {v}: {got_nn} != {NN[v]}"
        assert got_ne == NE[v], f"NE row of {v}: {got_ne} != {NE[v]}"


def adjacency_pairs(tri) -> set:
    s = set()
    for a, b, c in tri.tolist():
        for p, q in ((a, b), (b, c), (c, a)):
            s.add((min(p, q), max(p, q)))
    return s


def assert_independent(members, tri):
    """Brute force: no two members share an edge."""
    mem = sorted(int(v) for v in members)
    ms = set(mem)
    pairs = adjacency_pairs(tri)
    for i, a in enumerate(mem):
        for b in mem[i + 1:]:
            assert (a, b) not in pairs, f"class members {a} and {b} are adjacent"
    return len(ms)


def canonical_tri(tri):
    """Rotate each row so the smallest id comes first (orientation kept)."""
    t = np.asarray(tri)
    k = np.argmin(t, axis=1)
    idx = (k[:, None] + np.arange(3)[None, :]) % 3
    return np.take_along_axis(t, idx, axis=1)


# ---- metric quantities computed independently in matrix form ----------------

def metric_len2(xy, met, a, b):
    """Edge length^2 in the mean metric of the end points: e^T M e."""
    M = 0.5 * (met[a] + met[b])
    e = xy[b] - xy[a]
    return M[:, 0] * e[:, 0] ** 2 + 2 * M[:, 1] * e[:, 0] * e[:, 1] + M[:, 2] * e[:, 1] ** 2


def size_factor(x):
    """(m (2 - m))^3 with m = min(x, 1/x): 1 at x = 1, below 1 elsewhere."""
    m = np.minimum(x, 1.0 / x)
    return (m * (2.0 - m)) ** 3


def vasilevskii(xy, met, tri):
    """Vasilevskii's functional 12 sqrt(3) |K|_M / P^2 * F(P / 3), computed
    from the three metric edge lengths alone: |K|_M by Heron's formula, P
    their sum (M the element's mean tensor, constant over the element)."""
    M = (met[tri[:, 0]] + met[tri[:, 1]] + met[tri[:, 2]]) / 3.0
    Mm = np.stack([np.stack([M[:, 0], M[:, 1]], -1), np.stack([M[:, 1], M[:, 2]], -1)], -2)
    P = xy[tri]
    L = []
    for i, j in ((0, 1), (1, 2), (2, 0)):
        e = P[:, j] - P[:, i]
        L.append(np.sqrt(np.einsum("ni,nij,nj->n", e, Mm, e)))
    a, b, c = L
    per = a + b + c
    area = 0.25 * np.sqrt(np.maximum(per * (b + c - a) * (a - b + c) * (a + b - c), 0.0))
    return 12.0 * np.sqrt(3.0) * area / per ** 2 * size_factor(per / 3.0)


def quality(xy, met, tri, kind=0):
    """The element functional: 0 the mean ratio, 1 Vasilevskii's."""
    return vasilevskii(xy, met, tri) if kind == 1 else mean_ratio(xy, met, tri)


def mean_ratio(xy, met, tri):
    """4 sqrt(3) sqrt(det M) A / sum_e e^T M e with M the element's mean tensor."""
    M = (met[tri[:, 0]] + met[tri[:, 1]] + met[tri[:, 2]]) / 3.0
    Mm = np.stack([np.stack([M[:, 0], M[:, 1]], -1), np.stack([M[:, 1], M[:, 2]], -1)], -2)
    P = xy[tri]
    A = 0.5 * doubled_areas(xy, tri)
    S = np.zeros(len(tri))
    for i, j in ((0, 1), (1, 2), (2, 0)):
        e = P[:, j] - P[:, i]
        S += np.einsum("ni,nij,nj->n", e, Mm, e)
    return 4.0 * np.sqrt(3.0) * np.sqrt(np.linalg.det(Mm)) * A / S
