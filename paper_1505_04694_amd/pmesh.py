"""Python binding of libpmesh.so (ctypes; argument marshalling only).

Every function carries the name of the C entry point it calls (include/pm.h).
Device memory and streams come from PyTorch: device-side inputs and gradient
outputs are torch tensors on the current GPU, and work is issued on
torch.cuda.current_stream(). The HIP library is required: if it is missing
or fails to load, every call raises, there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpmesh.so")

PM_OK, PM_E_ARG, PM_E_MESH, PM_E_NOMEM, PM_E_DEVICE, PM_W_NOT_CONVERGED, PM_W_PAUSED = range(7)
PM_MEM_HOST, PM_MEM_DEVICE = 0, 1
PM_SMOOTH_LAPLACE, PM_SMOOTH_GRADIENT, PM_SMOOTH_MINMAX = 0, 1, 2
PM_QUALITY_MEAN_RATIO, PM_QUALITY_VASILEVSKII = 0, 1
PM_PHASE_COARSEN, PM_PHASE_SWAP, PM_PHASE_REFINE, PM_PHASE_SMOOTH, PM_PHASE_DONE = 1, 2, 3, 4, 5
STATUS = {0: "PM_OK", 1: "PM_E_ARG", 2: "PM_E_MESH", 3: "PM_E_NOMEM", 4: "PM_E_DEVICE", 5: "PM_W_NOT_CONVERGED",
          6: "PM_W_PAUSED"}
STAT_NAMES = ["rounds", "coloured", "evaluated", "deferred", "committed", "colours", "edges", "converged",
              "new_vertices", "new_elements", "records", "relocated", "jp_iterations", "room_rebuilds"]

EXPORTS = ["pm_default_options", "pm_mesh_create", "pm_mesh_destroy", "pm_mesh_sizes", "pm_mesh_memory", "pm_mesh_export",
           "pm_mesh_rows", "pm_colour", "pm_coarsen", "pm_refine", "pm_swap", "pm_smooth", "pm_quality",
           "pm_adapt", "pm_get_context", "pm_set_context", "pm_mesh_update", "pm_quality_noalloc",
           "pm_last_error", "pm_version", "pm_fp64_selfcheck", "pm_profile", "pm_profile_read",
           "pm_batch_create", "pm_batch_count", "pm_batch_sizes", "pm_batch_export", "pm_batch_quality"]
KERNELS = ["jp", "collapse", "flip", "smooth", "commit", "adjoint", "quality", "select"]
# ids pm_profile_read takes: the kernels, and the commit counted in committed operations
PROFILE_READS = KERNELS + ["commit_ops"]


class PMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Tuning(C.Structure):
    _fields_ = [("op_lanes", C.c_int32), ("smooth_lanes", C.c_int32), ("commit_chunk", C.c_int32),
                ("small_work", C.c_int32), ("class_colours", C.c_int32), ("commit_order", C.c_int32),
                ("host_rounds", C.c_int32), ("reserved", C.c_int32)]
    KEYS = ["op_lanes", "smooth_lanes", "commit_chunk", "small_work", "class_colours", "commit_order", "host_rounds"]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k in self.KEYS}

    @classmethod
    def of(cls, d=None):
        t = cls()
        for k, v in (d or {}).items():
            setattr(t, k, v)
        return t


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("release", RELEASE_FN), ("user", C.c_void_p)]


def torch_allocator():
    """A pm_allocator whose blocks come from torch's caching allocator on the
    handle's stream (so torch's memory statistics and limits cover the
    handle). Keep the returned object alive as long as the handle."""
    import torch

    def alloc(nbytes, stream, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        except Exception:  # noqa: BLE001 - the library turns NULL into PM_E_NOMEM
            return None

    def release(ptr, nbytes, stream, user):
        torch.cuda.caching_allocator_delete(int(ptr))

    a = Allocator(ALLOC_FN(alloc), RELEASE_FN(release), None)
    return a


def _allocator_of(allocator):
    if allocator is None or isinstance(allocator, Allocator):
        return allocator
    if allocator == "torch":
        return torch_allocator()
    raise ValueError(f"unknown allocator {allocator!r}")


class Options(C.Structure):
    _fields_ = [("L_low2", C.c_double), ("L_up2", C.c_double), ("q_min", C.c_double), ("seed", C.c_uint64),
                ("sweep", C.c_int32), ("coarsen_rounds", C.c_int32), ("swap_rounds", C.c_int32),
                ("refine_passes", C.c_int32), ("smooth_kind", C.c_int32), ("smooth_sweeps", C.c_int32),
                ("slack", C.c_double), ("pool_headroom", C.c_double), ("max_iterations", C.c_int32),
                ("max_phases", C.c_int32), ("tune", Tuning), ("quality", C.c_int32), ("reserved", C.c_int32),
                ("allocator", C.POINTER(Allocator))]


class Context(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("iteration", C.c_int32), ("phase", C.c_int32), ("changed", C.c_int32),
                ("reserved", C.c_int32)]

    def as_dict(self):
        return dict(seed=int(self.seed), iteration=int(self.iteration), phase=int(self.phase),
                    changed=int(self.changed))


class Stats(C.Structure):
    _fields_ = [("v", C.c_int64 * 16)]

    def as_dict(self):
        return {k: int(self.v[i]) for i, k in enumerate(STAT_NAMES)}


class MeshDesc(C.Structure):
    _fields_ = [("xy", C.c_void_p), ("tri", C.c_void_p), ("metric", C.c_void_p), ("tags", C.c_void_p),
                ("V", C.c_int64), ("T", C.c_int64), ("mem_kind", C.c_int32)]


_lib = None


def lib():
    """Load libpmesh.so; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1505_04694_amd/build.py")
        # torch first: its HIP runtime (soname libamdhip64.so.7) is then the one
        # this library binds to, so torch and the library share one runtime
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        P, S = C.c_void_p, C.c_int
        L.pm_default_options.restype = S
        L.pm_default_options.argtypes = [C.POINTER(Options)]
        L.pm_mesh_create.restype = S
        L.pm_mesh_create.argtypes = [C.POINTER(MeshDesc), C.POINTER(Options), P, C.POINTER(P)]
        L.pm_mesh_destroy.restype = S
        L.pm_mesh_destroy.argtypes = [P]
        L.pm_mesh_sizes.restype = S
        L.pm_mesh_sizes.argtypes = [P, P, P]
        L.pm_mesh_memory.restype = S
        L.pm_mesh_memory.argtypes = [P, P, P]
        L.pm_mesh_export.restype = S
        L.pm_mesh_export.argtypes = [P, P, P, P, P, P, P, C.c_int32]
        L.pm_mesh_rows.restype = S
        L.pm_mesh_rows.argtypes = [P, P, P, P, P, P, P]
        L.pm_colour.restype = S
        L.pm_colour.argtypes = [P, P, C.c_uint32, P, P, C.c_int32]
        for f in ("pm_coarsen", "pm_refine", "pm_swap", "pm_smooth", "pm_adapt"):
            getattr(L, f).restype = S
            getattr(L, f).argtypes = [P, C.POINTER(Options), C.POINTER(Stats)]
        L.pm_quality.restype = S
        L.pm_quality.argtypes = [P, P, P, P, P]
        L.pm_quality_noalloc.restype = S
        L.pm_quality_noalloc.argtypes = [P, P, P, P, P]
        L.pm_get_context.restype = S
        L.pm_get_context.argtypes = [P, C.POINTER(Context)]
        L.pm_set_context.restype = S
        L.pm_set_context.argtypes = [P, C.POINTER(Context)]
        L.pm_mesh_update.restype = S
        L.pm_mesh_update.argtypes = [P, P, P, C.c_int32]
        L.pm_last_error.restype = C.c_char_p
        L.pm_last_error.argtypes = [P]
        L.pm_version.restype = C.c_char_p
        L.pm_version.argtypes = []
        L.pm_profile.restype = S
        L.pm_profile.argtypes = [P, C.c_uint32]
        L.pm_profile_read.restype = S
        L.pm_profile_read.argtypes = [P, C.c_int32, P, P, P]
        L.pm_batch_create.restype = S
        L.pm_batch_create.argtypes = [P, C.c_int32, C.POINTER(Options), P, C.POINTER(P)]
        L.pm_batch_count.restype = S
        L.pm_batch_count.argtypes = [P, P]
        L.pm_batch_sizes.restype = S
        L.pm_batch_sizes.argtypes = [P, C.c_int32, P, P]
        L.pm_batch_export.restype = S
        L.pm_batch_export.argtypes = [P, C.c_int32, P, P, P, P, P, P]
        L.pm_batch_quality.restype = S
        L.pm_batch_quality.argtypes = [P, P, P]
        L.pm_fp64_selfcheck.restype = S
        L.pm_fp64_selfcheck.argtypes = [P, P, C.c_int64, P, P]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


def _check(h, status, allow_warn=True):
    if status == PM_OK or (allow_warn and status in (PM_W_NOT_CONVERGED, PM_W_PAUSED)):
        return status
    msg = lib().pm_last_error(h).decode() if h else ""
    raise PMError(status, msg)


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def pm_default_options(**kw) -> Options:
    """Defaults, with any field set by keyword; tune takes a dict of Tuning fields."""
    o = Options()
    _check(None, lib().pm_default_options(C.byref(o)))
    for k, v in kw.items():
        if k == "tune":
            v = Tuning.of(v) if not isinstance(v, Tuning) else v
        setattr(o, k, v)
    return o


def pm_fp64_selfcheck(a, b):
    a = np.ascontiguousarray(a, np.float64); b = np.ascontiguousarray(b, np.float64)
    q = np.empty_like(a); r = np.empty_like(a)
    _check(None, lib().pm_fp64_selfcheck(_p(a), _p(b), a.size, _p(q), _p(r)))
    return q, r


def pm_profile(h, mask: int):
    _check(h, lib().pm_profile(h, mask))


def pm_profile_read(h, kid: int):
    ms, n, u = C.c_double(), C.c_int64(), C.c_int64()
    _check(h, lib().pm_profile_read(h, kid, C.byref(ms), C.byref(n), C.byref(u)))
    return dict(ms=ms.value, launches=n.value, units=u.value)


def pm_version() -> str:
    return lib().pm_version().decode()


def pm_mesh_create(xy, tri, metric, tags=None, options: Options | None = None, stream=None):
    """Create a handle from host numpy arrays or device torch tensors."""
    on_dev = hasattr(xy, "is_cuda") and xy.is_cuda
    if on_dev:
        import torch
        xy = xy.to(torch.float64).contiguous()
        tri = tri.to(torch.int32).contiguous()
        metric = metric.to(torch.float64).contiguous()
        tags = None if tags is None else tags.to(torch.uint8).contiguous()
        V, T = xy.shape[0], tri.shape[0]
    else:
        xy = np.ascontiguousarray(xy, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        metric = np.ascontiguousarray(metric, dtype=np.float64)
        tags = None if tags is None else np.ascontiguousarray(tags, dtype=np.uint8)
        V, T = xy.shape[0], tri.shape[0]
    d = MeshDesc()
    d.V, d.T = V, T
    d.mem_kind = PM_MEM_DEVICE if on_dev else PM_MEM_HOST
    d.xy = _p(xy).value
    d.tri = _p(tri).value
    d.metric = _p(metric).value
    d.tags = _p(tags).value if tags is not None else None
    h = C.c_void_p()
    o = options if options is not None else pm_default_options()
    st = lib().pm_mesh_create(C.byref(d), C.byref(o), stream if stream is not None else _stream(), C.byref(h))
    if st != PM_OK:
        raise PMError(st, "pm_mesh_create: " + lib().pm_last_error(None).decode())
    return h


def pm_mesh_destroy(h):
    _check(h, lib().pm_mesh_destroy(h))


def pm_mesh_sizes(h):
    V, T = C.c_int64(), C.c_int64()
    _check(h, lib().pm_mesh_sizes(h, C.byref(V), C.byref(T)))
    return V.value, T.value


def pm_mesh_memory(h):
    """(current, peak) device bytes held by the handle."""
    cur, peak = C.c_int64(), C.c_int64()
    _check(h, lib().pm_mesh_memory(h, C.byref(cur), C.byref(peak)))
    return cur.value, peak.value


def pm_mesh_export(h):
    V, T = pm_mesh_sizes(h)
    xy = np.empty((V, 2)); met = np.empty((V, 3)); tri = np.empty((T, 3), np.int32)
    tags = np.empty(V, np.uint8); va = np.empty(V, np.uint8); ta = np.empty(max(T, 1), np.uint8)
    _check(h, lib().pm_mesh_export(h, _p(xy), _p(tri), _p(met), _p(tags), _p(va), _p(ta), PM_MEM_HOST))
    return dict(xy=xy, tri=tri, metric=met, tags=tags, valive=va.astype(bool), talive=ta[:T].astype(bool))


def pm_mesh_rows(h):
    a, b = C.c_int64(), C.c_int64()
    _check(h, lib().pm_mesh_rows(h, C.byref(a), C.byref(b), None, None, None, None))
    V, _ = pm_mesh_sizes(h)
    nn_off = np.empty(V + 1, np.int64); ne_off = np.empty(V + 1, np.int64)
    nn = np.empty(max(a.value, 1), np.int32); ne = np.empty(max(b.value, 1), np.int32)
    _check(h, lib().pm_mesh_rows(h, C.byref(a), C.byref(b), _p(nn_off), _p(nn), _p(ne_off), _p(ne)))
    return nn_off, nn[:a.value], ne_off, ne[:b.value]


def pm_colour(h, active=None, ctx: int = 0):
    V, _ = pm_mesh_sizes(h)
    out = np.empty(V, np.int32)
    n = C.c_int32()
    act = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
    _check(h, lib().pm_colour(h, _p(act), ctx, _p(out), C.byref(n), PM_MEM_HOST))
    return out, n.value


def _phase(fn, h, options):
    st = Stats()
    o = options if options is not None else pm_default_options()
    status = _check(h, getattr(lib(), fn)(h, C.byref(o), C.byref(st)))
    d = st.as_dict()
    d["status"] = STATUS[status]
    return d


def pm_coarsen(h, options: Options | None = None):
    return _phase("pm_coarsen", h, options)


def pm_refine(h, options: Options | None = None):
    return _phase("pm_refine", h, options)


def pm_swap(h, options: Options | None = None):
    return _phase("pm_swap", h, options)


def pm_smooth(h, options: Options | None = None):
    return _phase("pm_smooth", h, options)


def pm_adapt(h, options: Options | None = None):
    return _phase("pm_adapt", h, options)


def pm_get_context(h) -> dict:
    c = Context()
    _check(h, lib().pm_get_context(h, C.byref(c)))
    return c.as_dict()


def pm_set_context(h, ctx: dict):
    c = Context()
    c.seed, c.iteration, c.phase, c.changed = ctx["seed"], ctx["iteration"], ctx["phase"], ctx["changed"]
    _check(h, lib().pm_set_context(h, C.byref(c)))


def pm_mesh_update(h, xy=None, metric=None):
    """New coordinates and/or metric: host numpy arrays or device torch tensors (float64)."""
    on_dev = any(a is not None and hasattr(a, "is_cuda") and a.is_cuda for a in (xy, metric))
    conv = []
    for a, w in ((xy, 2), (metric, 3)):
        if a is None:
            conv.append(None)
        elif on_dev:
            import torch
            conv.append(a.detach().to(torch.float64).contiguous())
        else:
            conv.append(np.ascontiguousarray(a, dtype=np.float64))
    _check(h, lib().pm_mesh_update(h, _p(conv[0]), _p(conv[1]), PM_MEM_DEVICE if on_dev else PM_MEM_HOST))


def pm_quality(h, grad: bool = False):
    """Q and qmin; with grad, also dQ/dx (V x 2) and dQ/dM (V x 3) as torch tensors on the GPU."""
    Q, qmin = C.c_double(), C.c_double()
    if not grad:
        _check(h, lib().pm_quality(h, C.byref(Q), C.byref(qmin), None, None))
        return Q.value, qmin.value
    import torch
    V, _ = pm_mesh_sizes(h)
    gx = torch.empty((V, 2), dtype=torch.float64, device="cuda")
    gm = torch.empty((V, 3), dtype=torch.float64, device="cuda")
    _check(h, lib().pm_quality(h, C.byref(Q), C.byref(qmin), _p(gx), _p(gm)))
    return Q.value, qmin.value, gx, gm


def pm_quality_noalloc(h, dQdx=None, dQdM=None):
    """Q and qmin with no device allocation in the library; gradients are
    written into caller-provided float64 device tensors (V x 2, V x 3) when given."""
    Q, qmin = C.c_double(), C.c_double()
    _check(h, lib().pm_quality_noalloc(h, C.byref(Q), C.byref(qmin), _p(dQdx), _p(dQdM)))
    return Q.value, qmin.value


def pm_batch_create(meshes, options: Options | None = None, stream=None):
    """meshes: list of (xy, tri, metric, tags-or-None) host arrays."""
    n = len(meshes)
    descs = (MeshDesc * n)()
    keep = []
    for i, (xy, tri, metric, tags) in enumerate(meshes):
        xy = np.ascontiguousarray(xy, np.float64); tri = np.ascontiguousarray(tri, np.int32)
        metric = np.ascontiguousarray(metric, np.float64)
        tags = None if tags is None else np.ascontiguousarray(tags, np.uint8)
        keep += [xy, tri, metric, tags]
        descs[i].xy = _p(xy).value
        descs[i].tri = _p(tri).value
        descs[i].metric = _p(metric).value
        descs[i].tags = _p(tags).value if tags is not None else None
        descs[i].V, descs[i].T = xy.shape[0], tri.shape[0]
        descs[i].mem_kind = PM_MEM_HOST
    h = C.c_void_p()
    o = options if options is not None else pm_default_options()
    st = lib().pm_batch_create(descs, n, C.byref(o), stream if stream is not None else _stream(), C.byref(h))
    if st != PM_OK:
        raise PMError(st, "pm_batch_create: " + lib().pm_last_error(None).decode())
    return h


def pm_batch_count(h) -> int:
    n = C.c_int32()
    _check(h, lib().pm_batch_count(h, C.byref(n)))
    return n.value


def pm_batch_sizes(h, i: int):
    V, T = C.c_int64(), C.c_int64()
    _check(h, lib().pm_batch_sizes(h, i, C.byref(V), C.byref(T)))
    return V.value, T.value


def pm_batch_export(h, i: int):
    V, T = pm_batch_sizes(h, i)
    xy = np.empty((V, 2)); met = np.empty((V, 3)); tri = np.empty((max(T, 1), 3), np.int32)
    tags = np.empty(V, np.uint8); va = np.empty(V, np.uint8); ta = np.empty(max(T, 1), np.uint8)
    _check(h, lib().pm_batch_export(h, i, _p(xy), _p(tri), _p(met), _p(tags), _p(va), _p(ta)))
    return dict(xy=xy, tri=tri[:T], metric=met, tags=tags, valive=va.astype(bool), talive=ta[:T].astype(bool))


def pm_batch_quality(h):
    n = pm_batch_count(h)
    Q = np.empty(n); qm = np.empty(n)
    _check(h, lib().pm_batch_quality(h, _p(Q), _p(qm)))
    return Q, qm


class Mesh:
    """Owning wrapper around a pm_mesh handle."""

    def __init__(self, xy, tri, metric, tags=None, seed: int = 0, slack: float = 2.0, stream=None, tune=None,
                 pool_headroom: float = 3.0, quality: int = PM_QUALITY_MEAN_RATIO, allocator=None):
        """allocator: None (the library's block cache), "torch" (torch's
        caching allocator) or an Allocator, kept alive with the handle."""
        self.tune = dict(tune or {})
        o = pm_default_options(seed=seed, slack=slack, pool_headroom=pool_headroom, quality=quality)
        self._allocator = _allocator_of(allocator)
        if self._allocator is not None:
            o.allocator = C.pointer(self._allocator)
        self.h = pm_mesh_create(xy, tri, metric, tags, o, stream)

    @classmethod
    def from_input(cls, mi, seed: int = 0, **kw):
        return cls(mi.xy, mi.tri, mi.metric, mi.tags, seed=seed, **kw)

    def close(self):
        if getattr(self, "h", None):
            pm_mesh_destroy(self.h)
            self.h = None

    __del__ = close

    def sizes(self):
        return pm_mesh_sizes(self.h)

    def memory(self):
        return pm_mesh_memory(self.h)

    def export(self):
        return pm_mesh_export(self.h)

    def rows(self):
        return pm_mesh_rows(self.h)

    def colour(self, active=None, ctx: int = 0):
        return pm_colour(self.h, active, ctx)

    def coarsen(self, sweep=0, L_low2=0.5, q_min=0.1, max_rounds=200):
        return pm_coarsen(self.h, pm_default_options(sweep=sweep, L_low2=L_low2, q_min=q_min,
                                                     coarsen_rounds=max_rounds, tune=self.tune))

    def refine(self, L_up2=2.0, max_passes=32):
        return pm_refine(self.h, pm_default_options(L_up2=L_up2, refine_passes=max_passes, tune=self.tune))

    def swap(self, sweep=0, max_rounds=100):
        return pm_swap(self.h, pm_default_options(sweep=sweep, swap_rounds=max_rounds, tune=self.tune))

    def smooth(self, sweep=0, kind=0, sweeps=1):
        return pm_smooth(self.h, pm_default_options(sweep=sweep, smooth_kind=kind, smooth_sweeps=sweeps,
                                                    tune=self.tune))

    def adapt(self, max_iterations=8, max_phases=0, smooth_kind=0, smooth_sweeps=1):
        """Algorithm 1 from the handle's loop state; returns (stats, finished)."""
        st = pm_adapt(self.h, pm_default_options(max_iterations=max_iterations, max_phases=max_phases,
                                                 smooth_kind=smooth_kind, smooth_sweeps=smooth_sweeps,
                                                 tune=self.tune))
        return st, st["status"] == "PM_OK"

    def get_context(self):
        return pm_get_context(self.h)

    def set_context(self, ctx):
        pm_set_context(self.h, ctx)

    def update(self, xy=None, metric=None):
        pm_mesh_update(self.h, xy, metric)

    def quality(self, grad: bool = False):
        return pm_quality(self.h, grad)

    def profile(self, mask: int):
        pm_profile(self.h, mask)

    def profile_read(self, names=None):
        """Timing per kernel group; names: the groups to read (default all)."""
        names = PROFILE_READS if names is None else names
        return {k: pm_profile_read(self.h, PROFILE_READS.index(k)) for k in names}

    def sweep(self, sweep: int, smooth_kind: int = 0, smooth_sweeps: int = 1):
        return dict(coarsen=self.coarsen(sweep), refine=self.refine(), swap=self.swap(sweep),
                    smooth=self.smooth(sweep, smooth_kind, smooth_sweeps))


class Batch(Mesh):
    """A batch of independent meshes adapted by the same kernel launches."""

    def __init__(self, meshes, seed: int = 0, slack: float = 2.0, stream=None, tune=None,
                 pool_headroom: float = 3.0, quality: int = PM_QUALITY_MEAN_RATIO, allocator=None):
        self.tune = dict(tune or {})
        o = pm_default_options(seed=seed, slack=slack, pool_headroom=pool_headroom, quality=quality)
        self._allocator = _allocator_of(allocator)
        if self._allocator is not None:
            o.allocator = C.pointer(self._allocator)
        self.h = pm_batch_create(meshes, o, stream)

    @classmethod
    def from_inputs(cls, mis, seed: int = 0, **kw):
        return cls([(mi.xy, mi.tri, mi.metric, mi.tags) for mi in mis], seed=seed, **kw)

    def count(self):
        return pm_batch_count(self.h)

    def export_mesh(self, i: int):
        return pm_batch_export(self.h, i)

    def quality_per_mesh(self):
        return pm_batch_quality(self.h)


def _autograd_function():
    import torch

    class QualityFn(torch.autograd.Function):
        """Q(xy, metric) = the sum of the mean-ratio qualities of a mesh's
        elements (Sec. 2.2), as a differentiable function of its vertex
        coordinates (V x 2) and metric (V x 3 stored entries m00, m01, m11).
        forward writes xy and metric into the handle (pm_mesh_update) and runs
        pm_quality with the adjoint; backward scales the library's dQ/dx and
        dQ/dM by the incoming gradient. Usage: Q = QualityFn.apply(xy, metric, mesh)."""

        @staticmethod
        def forward(ctx, xy, metric, mesh):
            pm_mesh_update(mesh.h, xy, metric)
            Q, _, gx, gm = pm_quality(mesh.h, grad=True)
            ctx.save_for_backward(gx, gm)
            return torch.tensor(Q, dtype=torch.float64, device=xy.device)

        @staticmethod
        def backward(ctx, gQ):
            gx, gm = ctx.saved_tensors
            return gQ * gx, gQ * gm, None

    return QualityFn


def __getattr__(name):
    # QualityFn needs torch; built on first use so that the module imports without it
    if name == "QualityFn":
        fn = _autograd_function()
        globals()["QualityFn"] = fn
        return fn
    raise AttributeError(name)
