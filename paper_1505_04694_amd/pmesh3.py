"""ctypes binding of the tetrahedral path (include/pm3.h): argument marshalling
only; every step runs in the HIP library, which must be built (no fallback)."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import pmesh
from .pmesh import PM_MEM_DEVICE, PM_MEM_HOST, Options, PMError, STATUS, Stats, pm_default_options

EXPORTS3 = ["pm3_mesh_create", "pm3_mesh_destroy", "pm3_mesh_sizes", "pm3_mesh_export", "pm3_mesh_rows",
            "pm3_colour", "pm3_coarsen", "pm3_refine", "pm3_smooth", "pm3_quality", "pm3_last_error"]


class MeshDesc3(C.Structure):
    _fields_ = [("xyz", C.c_void_p), ("tet", C.c_void_p), ("metric", C.c_void_p), ("tags", C.c_void_p),
                ("V", C.c_int64), ("T", C.c_int64), ("mem_kind", C.c_int32)]


_ready = False


def lib():
    global _ready
    L = pmesh.lib()
    if not _ready:
        P = C.c_void_p
        S = C.c_int
        L.pm3_mesh_create.restype = S
        L.pm3_mesh_create.argtypes = [C.POINTER(MeshDesc3), C.POINTER(Options), P, C.POINTER(P)]
        L.pm3_mesh_destroy.restype = S
        L.pm3_mesh_destroy.argtypes = [P]
        L.pm3_mesh_sizes.restype = S
        L.pm3_mesh_sizes.argtypes = [P, P, P]
        L.pm3_mesh_export.restype = S
        L.pm3_mesh_export.argtypes = [P, P, P, P, P, P, P, C.c_int32]
        L.pm3_mesh_rows.restype = S
        L.pm3_mesh_rows.argtypes = [P, P, P, P, P, P, P]
        L.pm3_colour.restype = S
        L.pm3_colour.argtypes = [P, P, C.c_uint32, P, P]
        for f in ("pm3_coarsen", "pm3_refine", "pm3_smooth"):
            getattr(L, f).restype = S
            getattr(L, f).argtypes = [P, C.POINTER(Options), C.POINTER(Stats)]
        L.pm3_quality.restype = S
        L.pm3_quality.argtypes = [P, P, P]
        L.pm3_last_error.restype = C.c_char_p
        L.pm3_last_error.argtypes = [P]
        _ready = True
    return L


def _p(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


def _check(h, status):
    if status in (pmesh.PM_OK, pmesh.PM_W_NOT_CONVERGED):
        return status
    msg = lib().pm3_last_error(h).decode()
    raise PMError(status, msg)


class Mesh3:
    """Owning wrapper around a pm3_mesh handle (host or torch-device arrays)."""

    def __init__(self, xyz, tet, metric, tags=None, seed: int = 0, stream=None, pool_headroom: float = 0.0):
        on_dev = hasattr(xyz, "data_ptr")
        if on_dev:
            keep = [xyz.contiguous(), tet.contiguous().int(), metric.contiguous(),
                    None if tags is None else tags.contiguous()]
        else:
            keep = [np.ascontiguousarray(xyz, np.float64), np.ascontiguousarray(tet, np.int32),
                    np.ascontiguousarray(metric, np.float64),
                    None if tags is None else np.ascontiguousarray(tags, np.uint8)]
        d = MeshDesc3(_p(keep[0]), _p(keep[1]), _p(keep[2]), _p(keep[3]), keep[0].shape[0], keep[1].shape[0],
                      PM_MEM_DEVICE if on_dev else PM_MEM_HOST)
        o = pm_default_options(seed=seed)
        if pool_headroom:
            o.pool_headroom = pool_headroom
        h = C.c_void_p()
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        st = lib().pm3_mesh_create(C.byref(d), C.byref(o), C.c_void_p(stream), C.byref(h))
        if st != pmesh.PM_OK:
            raise PMError(st, lib().pm3_last_error(None).decode())
        self.h = h

    @classmethod
    def from_input(cls, mi, seed: int = 0, **kw):
        return cls(mi.xyz, mi.tet, mi.metric, mi.tags, seed=seed, **kw)

    def close(self):
        if getattr(self, "h", None):
            lib().pm3_mesh_destroy(self.h)
            self.h = None

    __del__ = close

    def sizes(self):
        V, T = C.c_int64(), C.c_int64()
        _check(self.h, lib().pm3_mesh_sizes(self.h, C.byref(V), C.byref(T)))
        return V.value, T.value

    def export(self):
        V, T = self.sizes()
        xyz = np.empty((V, 3)); met = np.empty((V, 6)); tet = np.empty((T, 4), np.int32)
        tags = np.empty(V, np.uint8); va = np.empty(V, np.uint8); ta = np.empty(max(T, 1), np.uint8)
        _check(self.h, lib().pm3_mesh_export(self.h, _p(xyz), _p(tet), _p(met), _p(tags), _p(va), _p(ta),
                                             PM_MEM_HOST))
        return dict(xyz=xyz, tet=tet, metric=met, tags=tags, valive=va.astype(bool), talive=ta[:T].astype(bool))

    def rows(self):
        a, b = C.c_int64(), C.c_int64()
        _check(self.h, lib().pm3_mesh_rows(self.h, C.byref(a), C.byref(b), None, None, None, None))
        V, _ = self.sizes()
        nn_off = np.empty(V + 1, np.int64); ne_off = np.empty(V + 1, np.int64)
        nn = np.empty(max(a.value, 1), np.int32); ne = np.empty(max(b.value, 1), np.int32)
        _check(self.h, lib().pm3_mesh_rows(self.h, C.byref(a), C.byref(b), _p(nn_off), _p(nn), _p(ne_off),
                                           _p(ne)))
        return nn_off, nn[:a.value], ne_off, ne[:b.value]

    def colour(self, active=None, ctx: int = 0):
        V, _ = self.sizes()
        out = np.empty(V, np.int32)
        n = C.c_int32()
        act = None if active is None else np.ascontiguousarray(active, np.uint8)
        _check(self.h, lib().pm3_colour(self.h, _p(act), ctx, _p(out), C.byref(n)))
        return out, n.value

    def _phase(self, fn, o):
        st = Stats()
        status = _check(self.h, getattr(lib(), fn)(self.h, C.byref(o), C.byref(st)))
        d = st.as_dict()
        d["status"] = STATUS[status]
        return d

    def coarsen(self, sweep=0, L_low2=0.5, q_min=0.1, max_rounds=200):
        return self._phase("pm3_coarsen", pm_default_options(sweep=sweep, L_low2=L_low2, q_min=q_min,
                                                             coarsen_rounds=max_rounds))

    def refine(self, L_up2=2.0, max_passes=32):
        return self._phase("pm3_refine", pm_default_options(L_up2=L_up2, refine_passes=max_passes))

    def smooth(self, sweep=0, sweeps=1):
        return self._phase("pm3_smooth", pm_default_options(sweep=sweep, smooth_sweeps=sweeps))

    def quality(self):
        Q, q = C.c_double(), C.c_double()
        _check(self.h, lib().pm3_quality(self.h, C.byref(Q), C.byref(q)))
        return Q.value, q.value

    def sweep(self, sweep: int, smooth_sweeps: int = 1):
        """One outer sweep: coarsen -> refine -> smooth (no swaps in 3D)."""
        return dict(coarsen=self.coarsen(sweep), refine=self.refine(), smooth=self.smooth(sweep, smooth_sweeps))
