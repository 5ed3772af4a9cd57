"""Seeded synthetic inputs: structured unit-square grids and analytic metric fields.

This module is the only code shared between the HIP path and the CPU oracle. It
builds input arrays and holds none of the adaptation arithmetic (no edge length,
no quality, no colouring). The paper's own workloads (Section 4: viscous
fingering, structural compliance, the synthetic psi benchmark) need solvers or a
Hessian-to-metric rule that the paper does not give, so analytic anisotropic
metric fields of the same character stand in for them: a boundary layer along a
sinusoidal curve, resolved at 0.01 across and 0.1 along it.

Numbering (all configurations):
  vertex id  = j*n + i,  x = i/(n-1), y = j/(n-1)
  cell (i,j) is split along '/' = (i,j)-(i+1,j+1) when (i+j) is even, else along
  '\\' = (i,j+1)-(i+1,j); the lower triangle comes first, element id =
  2*(j*(n-1)+i) + k, every triangle counter-clockwise.
Metric entries are stored per vertex as (m00, m01, m11) of the symmetric 2x2
tensor [[m00, m01], [m01, m11]].
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

# boundary tag bits, derived from exact coordinates of the unit square
TAG_X0, TAG_X1, TAG_Y0, TAG_Y1 = 1, 2, 4, 8


@dataclass
class MeshInput:
    xy: np.ndarray          # (V, 2) float64
    tri: np.ndarray         # (T, 3) int32, counter-clockwise
    metric: np.ndarray      # (V, 3) float64: m00, m01, m11
    tags: np.ndarray        # (V,) uint8
    n: int = 0
    info: dict = field(default_factory=dict)

    @property
    def V(self) -> int:
        return int(self.xy.shape[0])

    @property
    def T(self) -> int:
        return int(self.tri.shape[0])

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.xy, self.tri, self.metric, self.tags):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()[:16]


def grid(n: int) -> tuple[np.ndarray, np.ndarray]:
    """Criss-cross triangulation of the unit square on an n x n vertex grid."""
    if n < 2:
        raise ValueError("grid needs n >= 2")
    i = np.arange(n, dtype=np.float64)
    xs = i / (n - 1)
    X, Y = np.meshgrid(xs, xs, indexing="xy")          # X[j, i] = x_i
    xy = np.stack([X.ravel(), Y.ravel()], axis=1).copy()
    ci, cj = np.meshgrid(np.arange(n - 1), np.arange(n - 1), indexing="xy")
    ci = ci.ravel().astype(np.int64)
    cj = cj.ravel().astype(np.int64)
    v00 = cj * n + ci
    v10 = v00 + 1
    v01 = v00 + n
    v11 = v01 + 1
    slash = ((ci + cj) % 2) == 0
    lower = np.where(slash[:, None],
                     np.stack([v00, v10, v11], 1),
                     np.stack([v00, v10, v01], 1))
    upper = np.where(slash[:, None],
                     np.stack([v00, v11, v01], 1),
                     np.stack([v10, v11, v01], 1))
    tri = np.empty((2 * (n - 1) ** 2, 3), dtype=np.int32)
    tri[0::2] = lower
    tri[1::2] = upper
    return xy, tri


def unit_square_tags(xy: np.ndarray) -> np.ndarray:
    x, y = xy[:, 0], xy[:, 1]
    t = np.zeros(xy.shape[0], dtype=np.uint8)
    t |= np.where(x == 0.0, TAG_X0, 0).astype(np.uint8)
    t |= np.where(x == 1.0, TAG_X1, 0).astype(np.uint8)
    t |= np.where(y == 0.0, TAG_Y0, 0).astype(np.uint8)
    t |= np.where(y == 1.0, TAG_Y1, 0).astype(np.uint8)
    return t


def _tensor(theta: np.ndarray, ht: np.ndarray | float, hn: np.ndarray) -> np.ndarray:
    """R(theta) diag(1/ht^2, 1/hn^2) R(theta)^T as (m00, m01, m11)."""
    c, s = np.cos(theta), np.sin(theta)
    lt = 1.0 / (np.asarray(ht) ** 2)
    ln = 1.0 / (hn ** 2)
    return np.stack([c * c * lt + s * s * ln, c * s * (lt - ln), s * s * lt + c * c * ln], axis=1)


def layer_y(xy: np.ndarray, amp: float = 0.1, width: float = 0.05, ht: float = 0.1) -> np.ndarray:
    """Boundary layer along y = 0.5 + amp*sin(2 pi x): h_n across, h_t along the curve."""
    x, y = xy[:, 0], xy[:, 1]
    d = y - 0.5 - amp * np.sin(2 * math.pi * x)
    hn = 0.01 + 0.2 * (1.0 - np.exp(-np.abs(d) / width))
    theta = np.arctan(2 * math.pi * amp * np.cos(2 * math.pi * x))
    return _tensor(theta, ht, hn)


def layer_x(xy: np.ndarray, amp: float = 0.1, width: float = 0.05, ht: float = 0.1) -> np.ndarray:
    """The same layer along the curve x = 0.5 + amp*sin(2 pi y)."""
    x, y = xy[:, 0], xy[:, 1]
    d = x - 0.5 - amp * np.sin(2 * math.pi * y)
    hn = 0.01 + 0.2 * (1.0 - np.exp(-np.abs(d) / width))
    theta = np.arctan2(np.ones_like(y), 2 * math.pi * amp * np.cos(2 * math.pi * y))
    return _tensor(theta, ht, hn)


def jitter(xy: np.ndarray, tags: np.ndarray, n: int, seed: int, frac: float = 0.2) -> np.ndarray:
    """Move interior vertices uniformly by up to frac*h per coordinate (h = 1/(n-1))."""
    rng = np.random.default_rng(seed)
    h = 1.0 / (n - 1)
    d = rng.uniform(-frac * h, frac * h, size=xy.shape)
    out = xy.copy()
    inner = tags == 0
    out[inner] += d[inner]
    return out


def make_mesh(n: int, *, layers: int = 1, jitter_seed: int | None = None,
              amp: float = 0.1, width: float = 0.05, ht: float = 0.1) -> MeshInput:
    xy, tri = grid(n)
    tags = unit_square_tags(xy)
    if jitter_seed is not None:
        xy = jitter(xy, tags, n, jitter_seed)
    met = layer_y(xy, amp, width, ht)
    if layers == 2:
        met = met + layer_x(xy, amp, width, ht)
    return MeshInput(xy=xy, tri=tri, metric=np.ascontiguousarray(met), tags=tags, n=n,
                     info=dict(n=n, layers=layers, jitter_seed=jitter_seed,
                               amp=amp, width=width, ht=ht))


def fan(k: int = 48, radius: float = 0.25, n_outer: int = 17, layers: int = 2, scale: float = 1.0,
        hubs: int = 1) -> MeshInput:
    """A high-degree start: one hub at (0.5, 0.5), or two at (0.45, 0.5) and
    (0.55, 0.5), joined to a ring of k vertices at the given radius around
    the centre, the rest of the unit square triangulated from an
    n_outer x n_outer grid (Delaunay of the point set, every triangle turned
    counter-clockwise). Each hub's adjacency rows hold about k / hubs entries.
    Metric: the layer field (layers 1 or 2) times scale; layers 0: scale times
    the identity; layers -1: a graded isotropic field c(r) I, r the distance
    to the centre, c = scale * min(4 + 4000 (r / radius)^4, 4004): coarse at
    the hubs (their joining edge is the only short one), fine at the ring."""
    from scipy.spatial import Delaunay
    g, _ = grid(n_outer)
    far = np.hypot(g[:, 0] - 0.5, g[:, 1] - 0.5) > radius * 1.3
    ang = 2 * math.pi * (np.arange(k) + 0.5) / k
    ring = np.stack([0.5 + radius * np.cos(ang), 0.5 + radius * np.sin(ang)], 1)
    centre = [[0.5, 0.5]] if hubs == 1 else [[0.45, 0.5], [0.55, 0.5]]
    xy = np.vstack([centre, ring, g[far]])
    tri = Delaunay(xy).simplices.astype(np.int32)
    p0, p1, p2 = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    D = (p1[:, 0] - p0[:, 0]) * (p2[:, 1] - p0[:, 1]) - (p2[:, 0] - p0[:, 0]) * (p1[:, 1] - p0[:, 1])
    tri = tri[D > 1e-14]
    D = D[D > 1e-14]
    tri[D < 0] = tri[D < 0][:, [0, 2, 1]]
    tags = unit_square_tags(xy)
    if layers == 0:
        met = np.tile([1.0, 0.0, 1.0], (xy.shape[0], 1))
    elif layers == -1:
        r = np.hypot(xy[:, 0] - 0.5, xy[:, 1] - 0.5)
        c = np.minimum(4.0 + 4000.0 * (r / radius) ** 4, 4004.0)
        met = np.stack([c, np.zeros_like(c), c], 1)
    else:
        met = layer_y(xy)
        if layers == 2:
            met = met + layer_x(xy)
    return MeshInput(xy=xy, tri=np.ascontiguousarray(tri, np.int32), metric=np.ascontiguousarray(met * scale),
                     tags=tags, n=n_outer,
                     info=dict(k=k, radius=radius, n_outer=n_outer, layers=layers, scale=scale, hubs=hubs))


# ---- named workloads -------------------------------------------------------

def refine_start(n: int = 17, scale: float = 200.0, jitter_seed: int = 7) -> MeshInput:
    """A coarse jittered grid under the two-layer field times scale: almost
    every edge is long, and refinement grows 512 triangles (n = 17) to about
    1.1e5 over seven passes."""
    mi = make_mesh(n, layers=2, jitter_seed=jitter_seed)
    mi.metric = np.ascontiguousarray(mi.metric * scale)
    mi.info["scale"] = scale
    return mi


# ---- the paper's synthetic benchmark (a time-varying solution psi) ---------------

def psi_hessian(xy: np.ndarray, phase: float) -> np.ndarray:
    """Analytic Hessian (h_xx, h_xy, h_yy) of
    psi(x, y) = 0.1 sin(50x + phase) + arctan(-0.1 / (2x - sin(5y + phase))),
    phase = 2 pi t / T. With u = 2x - sin(5y + phase) and f(u) = arctan(-0.1/u):
    f' = 0.1 / (u^2 + 0.01) and f'' = -0.2 u / (u^2 + 0.01)^2, smooth at u = 0
    (psi jumps by pi there, its derivatives do not)."""
    x, y = xy[:, 0], xy[:, 1]
    a = 50.0 * x + phase
    b = 5.0 * y + phase
    u = 2.0 * x - np.sin(b)
    den = u * u + 0.01
    f1 = 0.1 / den
    f2 = -0.2 * u / (den * den)
    ux, uy, uyy = 2.0, -5.0 * np.cos(b), 25.0 * np.sin(b)
    hxx = -250.0 * np.sin(a) + f2 * ux * ux
    hxy = f2 * ux * uy
    hyy = f2 * uy * uy + f1 * uyy
    return np.stack([hxx, hxy, hyy], axis=1)


def psi_metric(xy: np.ndarray, phase: float, eps: float, hmin: float = 1e-3, hmax: float = 0.2) -> np.ndarray:
    """Metric from the Hessian: R diag(lam~) R^T with lam~ = clamp(|lam| / eps,
    1/hmax^2, 1/hmin^2), H = R diag(lam) R^T (the usual Hessian-based reading;
    the paper does not give the rule). The 2x2 eigen-decomposition is written
    in closed form (elementwise, so the same on every host): lam = (a + c)/2
    +- sqrt(((a - c)/2)^2 + b^2), the first eigenvector at angle
    0.5 atan2(2b, a - c)."""
    h = psi_hessian(xy, phase)
    a, b, c = h[:, 0], h[:, 1], h[:, 2]
    mean = 0.5 * (a + c)
    rad = np.sqrt((0.5 * (a - c)) ** 2 + b * b)
    lo, hi = 1.0 / hmax ** 2, 1.0 / hmin ** 2
    l1 = np.clip(np.abs(mean + rad) / eps, lo, hi)
    l2 = np.clip(np.abs(mean - rad) / eps, lo, hi)
    th = 0.5 * np.arctan2(2.0 * b, a - c)
    cs, sn = np.cos(th), np.sin(th)
    return np.ascontiguousarray(np.stack([l1 * cs * cs + l2 * sn * sn, (l1 - l2) * cs * sn,
                                          l1 * sn * sn + l2 * cs * cs], axis=1))


def ideal_elements(xy: np.ndarray, tri: np.ndarray, metric: np.ndarray) -> float:
    """Elements of an ideal mesh for the metric: the metric-space area over the
    area of a unit equilateral triangle, sqrt(3)/4 (element metric = vertex mean)."""
    p0, p1, p2 = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    A = 0.5 * np.abs((p1[:, 0] - p0[:, 0]) * (p2[:, 1] - p0[:, 1]) - (p2[:, 0] - p0[:, 0]) * (p1[:, 1] - p0[:, 1]))
    m = (metric[tri[:, 0]] + metric[tri[:, 1]] + metric[tri[:, 2]]) / 3.0
    det = np.maximum(m[:, 0] * m[:, 2] - m[:, 1] ** 2, 0.0)
    return float((np.sqrt(det) * A).sum() / (math.sqrt(3.0) / 4.0))


def psi_eps(xy: np.ndarray, tri: np.ndarray, target: float, phase: float = 0.0, **kw) -> float:
    """The eps of psi_metric whose ideal element count on (xy, tri) is target (bisection in log eps)."""
    lo, hi = -12.0, 6.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        n = ideal_elements(xy, tri, psi_metric(xy, phase, 10.0 ** mid, **kw))
        if n > target:
            lo = mid
        else:
            hi = mid
    return 10.0 ** (0.5 * (lo + hi))


def psi_start(n: int = 201, target: float = 550e3, steps: int = 50) -> MeshInput:
    """The benchmark's start: an isotropic n x n grid of the unit square (about
    2(n-1)^2 triangles: 80,000 for n = 201) and the metric of psi at t = 0 with
    eps set for about `target` elements; the time step advances the phase by
    2 pi / steps (info: eps, steps)."""
    xy, tri = grid(n)
    eps = psi_eps(xy, tri, target)
    return MeshInput(xy=xy, tri=tri, metric=psi_metric(xy, 0.0, eps), tags=unit_square_tags(xy), n=n,
                     info=dict(eps=eps, steps=steps, target=target))


def config0() -> MeshInput:
    """33 x 33 grid, one-layer field; priority seed 0."""
    return make_mesh(33)


def config1() -> MeshInput:
    """1025 x 1025 grid, one-layer field; priority seed 0."""
    return make_mesh(1025)


def config2(n: int = 2049) -> MeshInput:
    """2049 x 2049 grid, interior jitter 0.2h from seed 1, two-layer field."""
    return make_mesh(n, layers=2, jitter_seed=1)


def config4(n: int = 4097) -> MeshInput:
    """4097 x 4097 grid, two-layer field, jitter from seed 3."""
    return make_mesh(n, layers=2, jitter_seed=3)


def batch_params(count: int = 256, seed: int = 2) -> list[dict]:
    """Per-mesh draw for the batched workload: n log-uniform in [17, 513] and
    the one-layer field's amplitude, layer width and tangential size."""
    rng = np.random.default_rng(seed)
    out = []
    lo, hi = math.log(17.0), math.log(513.0)
    for _ in range(count):
        n = int(round(math.exp(rng.uniform(lo, hi))))
        amp = float(rng.uniform(0.05, 0.2))
        width = float(rng.uniform(0.02, 0.1))
        ht = float(rng.uniform(0.05, 0.2))
        out.append(dict(n=n, amp=amp, width=width, ht=ht))
    return out


def config3(count: int = 256, seed: int = 2) -> list[MeshInput]:
    return [make_mesh(p["n"], amp=p["amp"], width=p["width"], ht=p["ht"])
            for p in batch_params(count, seed)]


PRIORITY_SEED = {0: 0, 1: 0, 2: 1, 3: 2, 4: 3}


# ---- tetrahedral meshes of the unit cube ------------------------------------------------

@dataclass
class MeshInput3:
    xyz: np.ndarray         # (V, 3) float64
    tet: np.ndarray         # (T, 4) int32, positively oriented
    metric: np.ndarray      # (V, 6) float64: m00, m01, m02, m11, m12, m22
    tags: np.ndarray        # (V,) uint8: x=0, x=1, y=0, y=1, z=0, z=1 bits
    n: int = 0
    info: dict = field(default_factory=dict)

    @property
    def V(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def T(self) -> int:
        return int(self.tet.shape[0])

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.xyz, self.tet, self.metric, self.tags):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()[:16]


def cube_grid(n: int) -> tuple[np.ndarray, np.ndarray]:
    """Kuhn (Freudenthal) triangulation of the unit cube on an n x n x n vertex
    grid: vertex id = (k n + j) n + i, every cube split into the six
    tetrahedra along its main diagonal (one per order of the three axes,
    ascending order of the axis permutations), positively oriented. The same
    split in every cube makes the mesh conforming."""
    if n < 2:
        raise ValueError("cube_grid needs n >= 2")
    s = np.arange(n, dtype=np.float64) / (n - 1)
    K, J, I = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    xyz = np.stack([s[I.ravel()], s[J.ravel()], s[K.ravel()]], axis=1)
    c = np.arange(n - 1)
    k, j, i = [a.ravel() for a in np.meshgrid(c, c, c, indexing="ij")]

    def vid(di, dj, dk):
        return ((k + dk) * n + (j + dj)) * n + (i + di)

    tets = []
    for perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        p = [0, 0, 0]
        path = [vid(0, 0, 0)]
        for ax in perm:
            p[ax] = 1
            path.append(vid(*p))
        # the path's volume has the sign of the permutation
        inversions = sum(1 for a in range(3) for b in range(a + 1, 3) if perm[a] > perm[b])
        if inversions % 2:
            path[2], path[3] = path[3], path[2]
        tets.append(np.stack(path, axis=1))
    tet = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    return xyz, tet


def unit_cube_tags(xyz: np.ndarray) -> np.ndarray:
    t = np.zeros(xyz.shape[0], dtype=np.uint8)
    for ax in range(3):
        t |= np.where(xyz[:, ax] == 0.0, 1 << (2 * ax), 0).astype(np.uint8)
        t |= np.where(xyz[:, ax] == 1.0, 2 << (2 * ax), 0).astype(np.uint8)
    return t


def _met6(M: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.stack([M[:, 0, 0], 0.5 * (M[:, 0, 1] + M[:, 1, 0]), 0.5 * (M[:, 0, 2] + M[:, 2, 0]),
                                          M[:, 1, 1], 0.5 * (M[:, 1, 2] + M[:, 2, 1]), M[:, 2, 2]], axis=1))


def layer_z(xyz: np.ndarray, amp: float = 0.1, width: float = 0.05, ht: float = 0.1, scale: float = 1.0,
            amp_y: float = 0.0) -> np.ndarray:
    """Boundary layer along the surface z = 0.5 + amp sin(2 pi x) + amp_y
    sin(2 pi y): h_n across it (0.01 at the surface, growing to 0.21 away from
    it over `width`), h_t along it; times `scale`. With amp_y != 0 the normal
    has all three components, so every tensor entry is non-zero."""
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    d = z - 0.5 - amp * np.sin(2 * math.pi * x) - amp_y * np.sin(2 * math.pi * y)
    hn = 0.01 + 0.2 * (1.0 - np.exp(-np.abs(d) / width))
    nrm = np.stack([-2 * math.pi * amp * np.cos(2 * math.pi * x), -2 * math.pi * amp_y * np.cos(2 * math.pi * y),
                    np.ones_like(x)], axis=1)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    P = np.einsum("ni,nj->nij", nrm, nrm)
    M = P / hn[:, None, None] ** 2 + (np.eye(3)[None] - P) / ht ** 2
    return _met6(M * scale)


def jitter3(xyz: np.ndarray, tags: np.ndarray, n: int, seed: int, frac: float = 0.1) -> np.ndarray:
    """Interior vertices moved uniformly by up to frac * h per coordinate
    (h = 1/(n-1); 0.1 h keeps every Kuhn tetrahedron positive, whose smallest
    height is h / sqrt(2))."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(-frac, frac, xyz.shape) / (n - 1)
    out = xyz.copy()
    inner = tags == 0
    out[inner] += d[inner]
    return out


def make_mesh3(n: int, *, jitter_seed: int | None = None, scale: float = 1.0, amp: float = 0.1,
               width: float = 0.05, ht: float = 0.1, amp_y: float = 0.0) -> MeshInput3:
    xyz, tet = cube_grid(n)
    tags = unit_cube_tags(xyz)
    if jitter_seed is not None:
        xyz = jitter3(xyz, tags, n, jitter_seed)
    return MeshInput3(xyz=xyz, tet=tet, metric=layer_z(xyz, amp, width, ht, scale, amp_y), tags=tags, n=n,
                      info=dict(jitter_seed=jitter_seed, scale=scale, amp_y=amp_y))


def psi_metric3(xyz: np.ndarray, phase: float, eps: float, hmin: float = 1e-3, hmax: float = 0.2) -> np.ndarray:
    """psi extruded along z: its Hessian has no z row, so the metric is the 2D
    rule in (x, y) and 1/hmax^2 along z. The 2x2 eigen-decomposition is
    written in closed form (elementwise, so the same on every host):
    lam = (a + c)/2 +- sqrt(((a - c)/2)^2 + b^2), the first eigenvector at
    angle 0.5 atan2(2b, a - c)."""
    h = psi_hessian(np.ascontiguousarray(xyz[:, :2]), phase)
    a, b, c = h[:, 0], h[:, 1], h[:, 2]
    mean = 0.5 * (a + c)
    rad = np.sqrt((0.5 * (a - c)) ** 2 + b * b)
    lo, hi = 1.0 / hmax ** 2, 1.0 / hmin ** 2
    l1 = np.clip(np.abs(mean + rad) / eps, lo, hi)
    l2 = np.clip(np.abs(mean - rad) / eps, lo, hi)
    th = 0.5 * np.arctan2(2.0 * b, a - c)
    cs, sn = np.cos(th), np.sin(th)
    m00 = l1 * cs * cs + l2 * sn * sn
    m01 = (l1 - l2) * cs * sn
    m11 = l1 * sn * sn + l2 * cs * cs
    z = np.zeros_like(a)
    return np.ascontiguousarray(np.stack([m00, m01, z, m11, z, np.full_like(a, lo)], axis=1))


def ideal_elements3(xyz: np.ndarray, tet: np.ndarray, metric: np.ndarray) -> float:
    """Elements of an ideal mesh for the metric: the metric-space volume over
    the volume of the regular tetrahedron with unit edges, sqrt(2)/12
    (determinants in closed form, elementwise)."""
    p = xyz[tet]
    a, b, c = p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]
    vol = np.abs(a[:, 0] * (b[:, 1] * c[:, 2] - b[:, 2] * c[:, 1]) - a[:, 1] * (b[:, 0] * c[:, 2] - b[:, 2] * c[:, 0])
                 + a[:, 2] * (b[:, 0] * c[:, 1] - b[:, 1] * c[:, 0])) / 6.0
    m = metric[tet].mean(axis=1)
    det = (m[:, 0] * (m[:, 3] * m[:, 5] - m[:, 4] * m[:, 4]) - m[:, 1] * (m[:, 1] * m[:, 5] - m[:, 4] * m[:, 2])
           + m[:, 2] * (m[:, 1] * m[:, 4] - m[:, 3] * m[:, 2]))
    return float((np.sqrt(np.maximum(det, 0.0)) * vol).sum() / (math.sqrt(2.0) / 12.0))


def psi_start3(n: int = 29, target: float = 210e3, steps: int = 50) -> MeshInput3:
    """The 3D benchmark's start: a Kuhn grid of the unit cube (n = 29: 131,712
    tetrahedra, about 50^3) and psi's metric at t = 0 with eps set for about
    `target` elements."""
    xyz, tet = cube_grid(n)
    lo, hi = -12.0, 6.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if ideal_elements3(xyz, tet, psi_metric3(xyz, 0.0, 10.0 ** mid)) > target:
            lo = mid
        else:
            hi = mid
    eps = 10.0 ** (0.5 * (lo + hi))
    return MeshInput3(xyz=xyz, tet=tet, metric=psi_metric3(xyz, 0.0, eps), tags=unit_cube_tags(xyz), n=n,
                      info=dict(eps=eps, steps=steps, target=target))
