"""Independent re-derivation of the tetrahedral path's per-member decisions
(numpy matrix forms; shares no code with the oracle or the HIP library).

  - collapse (Sec. 2.4.1): candidates u in NN(v) on every boundary face v is
    on, with L^2 < L_low^2, in ascending (L^2, u); the first whose re-pointed
    elements all keep a positive volume and quality >= q_min is taken;
  - smoothing (Sec. 2.4.4): the Laplacian in the metric, a 3x3 solve with
    edge-mean tensors, kept when every element keeps a positive volume and
    the patch minimum quality does not drop.
Each returns a margin: the smallest relative gap between two quantities whose
comparison decided it; callers skip members whose margin is below rounding.
"""
from __future__ import annotations

import numpy as np

from tests import checker3


class Patches3:
    def __init__(self, d):
        self.d = d
        ta = np.asarray(d["talive"], bool)
        self.tid = np.nonzero(ta)[0]
        self.tet = d["tet"][ta]
        V = d["xyz"].shape[0]
        self.elems = [[] for _ in range(V)]
        for k, row in enumerate(self.tet.tolist()):
            for v in row:
                self.elems[v].append(k)
        self.nbrs = [sorted({w for k in self.elems[v] for w in self.tet[k].tolist() if w != v}) for v in range(V)]


def _rel(a, b):
    return abs(a - b) / max(abs(a), abs(b), 1e-300)


def collapse_decision(P: Patches3, v, L_low2=0.5, q_min=0.1):
    """(target or None, margin)."""
    d = P.d
    xyz, met, tags = d["xyz"], d["metric"], d["tags"]
    nb = np.array(P.nbrs[v], np.int64)
    if nb.size == 0:
        return None, 1.0
    L2 = checker3.metric_len2(xyz, met, np.full(nb.size, v), nb)
    ok_tag = (tags[v] & ~tags[nb]) == 0
    margin = 1.0
    for L, u in sorted(zip(L2.tolist(), nb.tolist())):
        margin = min(margin, _rel(L, L_low2))
        if L >= L_low2 or not ok_tag[nb.tolist().index(u)]:
            continue
        rows = [P.tet[k].copy() for k in P.elems[v] if u not in P.tet[k]]
        if not rows:
            return u, margin
        rows = np.array(rows)
        rows[rows == v] = u
        D = checker3.vol6(xyz, rows)
        q = checker3.mean_ratio(xyz, met, rows) if (D > 0).all() else None
        margin = min(margin, float(np.abs(D).min() / max(np.abs(D).max(), 1e-300)))
        if q is not None:
            margin = min(margin, _rel(float(q.min()), q_min))
        if (D > 0).all() and (q >= q_min).all():
            return u, margin
    return None, margin


def laplace_target(P: Patches3, v):
    xyz, met = P.d["xyz"], P.d["metric"]
    G = np.zeros((3, 3))
    r = np.zeros(3)
    for j in P.nbrs[v]:
        M = checker3.mat(0.5 * (met[v] + met[j]))
        G += M
        r += M @ (xyz[j] - xyz[v])
    return xyz[v] + np.linalg.solve(G, r)


def laplace_decision(P: Patches3, v):
    """(moves, new position, margin)."""
    xyz, met = P.d["xyz"], P.d["metric"]
    rows = P.tet[P.elems[v]]
    p = laplace_target(P, v)
    old = float(checker3.mean_ratio(xyz, met, rows).min())
    xyz2 = xyz.copy()
    xyz2[v] = p
    D = checker3.vol6(xyz2, rows)
    margin = float(np.abs(D).min() / max(np.abs(D).max(), 1e-300))
    if not (D > 0).all():
        return False, p, margin
    new = float(checker3.mean_ratio(xyz2, met, rows).min())
    margin = min(margin, _rel(new, old))
    return new >= old, p, margin


def deferred_set(P: Patches3, whole, key):
    cls = set(int(v) for v in whole)
    return {v for v in cls if any(w in cls and key(w) > key(v) for w in P.nbrs[v])}
