"""Independent re-derivation of each per-member decision of the adaptation
kernels, used to pin the oracle's rules (numpy matrix forms, and torch CPU
autograd in float64 for the gradient; shares no code with the oracle or the
HIP library).

Each function takes a snapshot of a mesh (the dict that ``export()`` returns)
and a vertex, and says what the rule as read from the paper does to it:
  - smoothing (Sec. 2.4.4): Laplacian in the metric, solved as a 2x2 linear
    system; gradient ascent of the patch's quality sum with a halving step;
    a move is kept when every area stays positive and the patch minimum does
    not drop (the gradient form also needs the patch sum to rise);
  - swapping (Sec. 2.4.3): the flip of an interior edge at v with the largest
    new minimum quality, ties to the smaller far vertex, kept only if that
    minimum beats the old one strictly;
  - re-validation (Sec. 3.2): a class member adjacent to a same-class member
    of larger key waits for the next round.
Each decision also returns a margin: the smallest relative gap between two
quantities whose comparison decided it. Where the margin is below a rounding
tolerance the decision may legitimately differ in the last bit, and the
callers skip that member.
"""
from __future__ import annotations

import numpy as np
import torch

from tests import checker


def live_tri(d):
    return d["tri"][d["talive"]], np.nonzero(d["talive"])[0]


class Patches:
    """Elements and neighbours around each vertex of a snapshot (rebuilt with
    numpy from the live element list)."""

    def __init__(self, d, kind=0):
        self.d = d
        self.kind = kind  # element functional: 0 mean ratio, 1 Vasilevskii
        tri, tid = live_tri(d)
        self.tri = tri
        self.tid = tid
        V = d["xy"].shape[0]
        self.elems = [[] for _ in range(V)]
        for k, row in enumerate(tri.tolist()):
            for v in row:
                self.elems[v].append(k)
        self.nbrs = [sorted({w for k in self.elems[v] for w in tri[k].tolist() if w != v}) for v in range(V)]

    def rows_of(self, v):
        return self.tri[self.elems[v]]


def _min_q(xy, met, rows, kind=0):
    D = checker.doubled_areas(xy, rows)
    return bool((D > 0).all()), float(checker.quality(xy, met, rows, kind).min())


def _torch_q(pts, Mm, kind):
    """The element functional in torch float64 from its corner points and
    mean tensor: the mean ratio in matrix form, or Vasilevskii's from the
    metric edge lengths with Heron's formula."""
    M = torch.stack([torch.stack([Mm[0], Mm[1]]), torch.stack([Mm[1], Mm[2]])])
    e = [pts[1] - pts[0], pts[2] - pts[1], pts[0] - pts[2]]
    if kind == 1:
        a, b, c = (torch.sqrt(ei @ M @ ei) for ei in e)
        per = a + b + c
        area = 0.25 * torch.sqrt(per * (b + c - a) * (a - b + c) * (a + b - c))
        x = per / 3.0
        m = torch.minimum(x, 1.0 / x)
        return 12.0 * np.sqrt(3.0) * area / per ** 2 * (m * (2.0 - m)) ** 3
    S = sum(ei @ M @ ei for ei in e)
    A = 0.5 * ((pts[1][0] - pts[0][0]) * (pts[2][1] - pts[0][1]) - (pts[2][0] - pts[0][0]) * (pts[1][1] - pts[0][1]))
    return 4.0 * np.sqrt(3.0) * torch.sqrt(torch.det(M)) * A / S


def _rel(a, b):
    s = max(abs(a), abs(b), 1e-300)
    return abs(a - b) / s


# ---- smoothing -------------------------------------------------------------------

def laplace_target(P: Patches, v):
    """p = x_v + G^-1 r, G = sum of edge-mean tensors, r = sum M_vj (x_j - x_v)."""
    xy, met = P.d["xy"], P.d["metric"]
    G = np.zeros((2, 2))
    r = np.zeros(2)
    for j in P.nbrs[v]:
        m = 0.5 * (met[v] + met[j])
        Mj = np.array([[m[0], m[1]], [m[1], m[2]]])
        G += Mj
        r += Mj @ (xy[j] - xy[v])
    return xy[v] + np.linalg.solve(G, r)


def laplace_decision(P: Patches, v):
    """(moves, new position, margin)."""
    xy, met = P.d["xy"], P.d["metric"]
    rows = P.rows_of(v)
    p = laplace_target(P, v)
    _, old = _min_q(xy, met, rows, P.kind)
    xy2 = xy.copy()
    xy2[v] = p
    D = checker.doubled_areas(xy2, rows)
    new = float(checker.quality(xy2, met, rows, P.kind).min())
    margin = min(_rel(new, old), float(np.abs(D).min() / max(np.abs(D).max(), 1e-300)))
    ok = bool((D > 0).all()) and new >= old
    return ok, p, margin


def _torch_patch_q(xy, met, rows, v, kind=0):
    """Q_v as a function of x_v (torch float64)."""
    X = torch.tensor(xy, dtype=torch.float64)
    xv = X[v].clone().requires_grad_(True)
    Mt = torch.tensor(met, dtype=torch.float64)
    total = torch.zeros((), dtype=torch.float64)
    for row in rows.tolist():
        pts = [xv if w == v else X[w] for w in row]
        Mm = (Mt[row[0]] + Mt[row[1]] + Mt[row[2]]) / 3.0
        total = total + _torch_q(pts, Mm, kind)
    return total, xv


def patch_gradient(P: Patches, v):
    total, xv = _torch_patch_q(P.d["xy"], P.d["metric"], P.rows_of(v), v, P.kind)
    total.backward()
    return xv.grad.numpy().copy(), float(total.detach())


def gradient_decision(P: Patches, v, steps=4):
    """Direction g / max(|g_x|, |g_y|); trial steps h/2, h/4, ..., h/2^steps with
    h the smallest max-norm distance to a neighbour; the first trial that keeps
    the areas positive, does not lower the patch minimum and raises Q_v wins.
    Returns (moves, new position, margin, k)."""
    xy, met = P.d["xy"], P.d["metric"]
    rows = P.rows_of(v)
    g, Q0 = patch_gradient(P, v)
    if g[0] == 0.0 and g[1] == 0.0:
        return False, xy[v].copy(), 1.0, 0
    dvec = g / np.abs(g).max()
    h = min(float(np.abs(xy[j] - xy[v]).max()) for j in P.nbrs[v])
    _, old = _min_q(xy, met, rows, P.kind)
    margin = 1.0
    t = h
    for k in range(1, steps + 1):
        t = t * 0.5
        p = xy[v] + t * dvec
        xy2 = xy.copy()
        xy2[v] = p
        D = checker.doubled_areas(xy2, rows)
        new = float(checker.quality(xy2, met, rows, P.kind).min())
        Qp = float(checker.quality(xy2, met, rows, P.kind).sum())
        margin = min(margin, _rel(new, old), _rel(Qp, Q0),
                     float(np.abs(D).min() / max(np.abs(D).max(), 1e-300)))
        if (D > 0).all() and new >= old and Qp > Q0:
            return True, p, margin, k
    return False, xy[v].copy(), margin, 0


def _torch_elem_grad(xy, met, row, v, kind=0):
    """q of one element and its gradient in x_v (torch float64)."""
    X = torch.tensor(xy, dtype=torch.float64)
    xv = X[v].clone().requires_grad_(True)
    Mt = torch.tensor(met, dtype=torch.float64)
    pts = [xv if w == v else X[w] for w in row]
    Mm = (Mt[row[0]] + Mt[row[1]] + Mt[row[2]]) / 3.0
    q = _torch_q(pts, Mm, kind)
    q.backward()
    return float(q.detach()), xv.grad.numpy().copy()


def minmax_decision(P: Patches, v, steps=4):
    """Ascent on the patch minimum: the gradient of the worst element's q
    (ties to the first in ascending element order), or, when the second worst
    is within 1%, the point nearest the origin on the segment between the two
    gradients; max-norm normalised; steps h/2 .. h/2^steps; the first step
    keeping the areas positive and raising the patch minimum strictly wins.
    Returns (moves, new position, margin)."""
    xy, met = P.d["xy"], P.d["metric"]
    rows = P.rows_of(v)
    qs = checker.quality(xy, met, rows, P.kind)
    order = sorted(range(len(rows)), key=lambda i: (qs[i], P.tid[P.elems[v][i]]))
    i1 = order[0]
    margin = 1.0
    if len(order) > 1:
        margin = min(margin, _rel(qs[order[1]], qs[i1]))
    _, g1 = _torch_elem_grad(xy, met, rows[i1].tolist(), v, P.kind)
    g = g1
    if len(order) > 1:
        i2 = order[1]
        margin = min(margin, abs(qs[i2] - 1.01 * qs[i1]) / qs[i1])
        if qs[i2] <= 1.01 * qs[i1]:
            _, g2 = _torch_elem_grad(xy, met, rows[i2].tolist(), v, P.kind)
            e = g2 - g1
            den = float(e @ e)
            if den > 0:
                lam = min(max(-float(g1 @ e) / den, 0.0), 1.0)
                g = g1 + lam * e
    if g[0] == 0.0 and g[1] == 0.0:
        return False, xy[v].copy(), margin
    dvec = g / np.abs(g).max()
    h = min(float(np.abs(xy[j] - xy[v]).max()) for j in P.nbrs[v])
    _, old = _min_q(xy, met, rows, P.kind)
    t = h
    for k in range(1, steps + 1):
        t = t * 0.5
        p = xy[v] + t * dvec
        xy2 = xy.copy()
        xy2[v] = p
        D = checker.doubled_areas(xy2, rows)
        new = float(checker.quality(xy2, met, rows, P.kind).min())
        margin = min(margin, _rel(new, old), float(np.abs(D).min() / max(np.abs(D).max(), 1e-300)))
        if (D > 0).all() and new > old:
            return True, p, margin
    return False, xy[v].copy(), margin


# ---- swapping ---------------------------------------------------------------------

def flip_decision(P: Patches, v):
    """(w, a, b, t1, t2, newmin) of the chosen flip at v, or None; and a margin.
    t1 holds the directed edge v->w, t2 the edge w->v (slot indices of the live
    element list)."""
    xy, met = P.d["xy"], P.d["metric"]
    tri = P.tri
    q = checker.quality(xy, met, tri[P.elems[v]], P.kind) if P.elems[v] else []
    qd = dict(zip(P.elems[v], q))
    cands = []
    margin = 1.0
    for w in P.nbrs[v]:
        t1 = t2 = None
        for k in P.elems[v]:
            row = tri[k].tolist()
            i = row.index(v)
            if row[(i + 1) % 3] == w:
                t1 = k
            elif row[(i + 2) % 3] == w:
                t2 = k
        if t1 is None or t2 is None:
            continue
        r1, r2 = tri[t1].tolist(), tri[t2].tolist()
        a = r1[(r1.index(v) + 2) % 3]
        b = r2[(r2.index(v) + 1) % 3]
        new = np.array([[v, b, a], [w, a, b]])
        D = checker.doubled_areas(xy, new)
        margin = min(margin, float(np.abs(D).min() / max(np.abs(D).max(), 1e-300)))
        if not (D > 0).all():
            continue
        nmin = float(checker.quality(xy, met, new, P.kind).min())
        omin = min(qd[t1], qd[t2])
        margin = min(margin, _rel(nmin, omin))
        if nmin > omin:
            cands.append((nmin, w, a, b, t1, t2))
    if not cands:
        return None, margin
    cands.sort(key=lambda c: (-c[0], c[1]))
    if len(cands) > 1:
        margin = min(margin, _rel(cands[0][0], cands[1][0]))
    nmin, w, a, b, t1, t2 = cands[0]
    return (w, a, b, t1, t2, nmin), margin


# ---- re-validation -----------------------------------------------------------------

def deferred_set(P: Patches, whole, key):
    """Members of the class `whole` adjacent to a member with a larger key."""
    cls = set(int(v) for v in whole)
    out = set()
    for v in cls:
        if any(w in cls and key(w) > key(v) for w in P.nbrs[v]):
            out.add(v)
    return out
