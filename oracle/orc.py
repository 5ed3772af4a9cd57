"""ctypes front end of the CPU oracle (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg use this
module. It loads oracle/liboracle.so, which shares no code with the HIP
library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

NSTATS = 16
STAT_NAMES = ["rounds", "coloured", "evaluated", "deferred", "committed", "colours",
              "edges", "converged", "new_vertices", "new_elements"]
PH_COARSEN, PH_SWAP, PH_SMOOTH = 1, 2, 3
PHASE_COARSEN, PHASE_SWAP, PHASE_REFINE, PHASE_SMOOTH, PHASE_DONE = 1, 2, 3, 4, 5
QUALITY_MEAN_RATIO, QUALITY_VASILEVSKII = 0, 1

_lib = None

HOOK = C.CFUNCTYPE(None, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.c_int64, C.c_int64, P, P, P, P, C.c_uint64]
        L.orc_destroy.argtypes = [P]
        L.orc_sizes.argtypes = [P, P, P]
        L.orc_export.argtypes = [P, P, P, P, P, P, P]
        L.orc_row_totals.argtypes = [P, P, P]
        L.orc_export_rows.argtypes = [P, P, P, P, P]
        L.orc_set_xy.argtypes = [P, C.c_int32, C.c_double, C.c_double]
        L.orc_set_metric.argtypes = [P, C.c_int32, C.c_double, C.c_double, C.c_double]
        L.orc_splitmix.restype = C.c_uint64
        L.orc_splitmix.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_prio.restype = C.c_uint32
        L.orc_prio.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32]
        L.orc_colour.restype = C.c_int32
        L.orc_colour.argtypes = [P, P, C.c_uint32, P]
        L.orc_set_hook.argtypes = [P, HOOK, P]
        L.orc_set_order_seed.argtypes = [P, C.c_uint64]
        L.orc_set_quality.restype = C.c_int32
        L.orc_set_quality.argtypes = [P, C.c_int32]
        L.orc_class_members.restype = C.c_int64
        L.orc_class_members.argtypes = [P, P, C.c_int64]
        L.orc_class_whole.restype = C.c_int64
        L.orc_class_whole.argtypes = [P, P, C.c_int64]
        L.orc_coarsen.restype = C.c_int32
        L.orc_coarsen.argtypes = [P, C.c_int32, C.c_double, C.c_double, C.c_int32, P]
        L.orc_refine.restype = C.c_int32
        L.orc_refine.argtypes = [P, C.c_double, C.c_int32, P]
        L.orc_swap.restype = C.c_int32
        L.orc_swap.argtypes = [P, C.c_int32, C.c_int32, P]
        L.orc_smooth.restype = C.c_int32
        L.orc_smooth.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, P]
        L.orc_compact.argtypes = [P]
        L.orc_adapt.restype = C.c_int32
        L.orc_adapt.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                C.c_double, C.c_int32, C.c_int32, C.c_int32, P]
        L.orc_get_context.argtypes = [P, P, P, P]
        L.orc_set_context.argtypes = [P, C.c_int32, C.c_int32, C.c_int32]
        L.orc_quality.argtypes = [P, P, P, P, P]
        L.orc_element_quality.argtypes = [P, P]
        L.orc_patch_quality.restype = C.c_double
        L.orc_patch_quality.argtypes = [P, C.c_int32]
        L.orc3_create.restype = P
        L.orc3_create.argtypes = [C.c_int64, C.c_int64, P, P, P, P, C.c_uint64]
        L.orc3_destroy.argtypes = [P]
        L.orc3_sizes.argtypes = [P, P, P]
        L.orc3_export.argtypes = [P, P, P, P, P, P, P]
        L.orc3_row_totals.argtypes = [P, P, P]
        L.orc3_export_rows.argtypes = [P, P, P, P, P]
        L.orc3_set_xyz.argtypes = [P, C.c_int32, C.c_double, C.c_double, C.c_double]
        L.orc3_set_hook.argtypes = [P, HOOK, P]
        L.orc3_class_members.restype = C.c_int64
        L.orc3_class_members.argtypes = [P, P, C.c_int64]
        L.orc3_class_whole.restype = C.c_int64
        L.orc3_class_whole.argtypes = [P, P, C.c_int64]
        L.orc3_colour.restype = C.c_int32
        L.orc3_colour.argtypes = [P, P, C.c_uint32, P]
        L.orc3_coarsen.restype = C.c_int32
        L.orc3_coarsen.argtypes = [P, C.c_int32, C.c_double, C.c_double, C.c_int32, P]
        L.orc3_refine.restype = C.c_int32
        L.orc3_refine.argtypes = [P, C.c_double, C.c_int32, P]
        L.orc3_smooth.restype = C.c_int32
        L.orc3_smooth.argtypes = [P, C.c_int32, C.c_int32, P]
        L.orc3_quality.argtypes = [P, P, P]
        L.orc3_element_quality.argtypes = [P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def splitmix(s: int, i: int) -> int:
    return int(lib().orc_splitmix(s, i))


def prio(seed: int, ctx: int, ident: int) -> int:
    return int(lib().orc_prio(seed, ctx, ident))


def ctx_of(sweep: int, phase: int, rnd: int) -> int:
    return (sweep << 20) | (phase << 16) | rnd


class OracleMesh:
    """One mesh held by the oracle."""

    def __init__(self, xy, tri, metric, tags=None, seed: int = 0, quality: int = QUALITY_MEAN_RATIO):
        xy = np.ascontiguousarray(xy, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        metric = np.ascontiguousarray(metric, dtype=np.float64)
        tg = None if tags is None else np.ascontiguousarray(tags, dtype=np.uint8)
        self.h = lib().orc_create(xy.shape[0], tri.shape[0], _p(xy), _p(tri), _p(metric), _p(tg), seed)
        if not self.h:
            raise ValueError("oracle rejected the mesh")
        self._hook_ref = None
        self._hook_exc = None
        if lib().orc_set_quality(self.h, quality) != 0:
            raise ValueError(f"unknown quality functional {quality}")

    @classmethod
    def from_input(cls, mi, seed: int = 0, quality: int = QUALITY_MEAN_RATIO):
        return cls(mi.xy, mi.tri, mi.metric, mi.tags, seed, quality)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_destroy(h)
            self.h = None

    def sizes(self):
        V = C.c_int64()
        T = C.c_int64()
        lib().orc_sizes(self.h, C.byref(V), C.byref(T))
        return V.value, T.value

    def export(self, live_only: bool = False):
        V, T = self.sizes()
        xy = np.empty((V, 2)); met = np.empty((V, 3))
        tri = np.empty((T, 3), np.int32)
        tags = np.empty(V, np.uint8); va = np.empty(V, np.uint8); ta = np.empty(T, np.uint8)
        lib().orc_export(self.h, _p(xy), _p(tri), _p(met), _p(tags), _p(va), _p(ta))
        d = dict(xy=xy, tri=tri, metric=met, tags=tags, valive=va.astype(bool), talive=ta.astype(bool))
        return d

    def rows(self):
        V, _ = self.sizes()
        a = C.c_int64(); b = C.c_int64()
        lib().orc_row_totals(self.h, C.byref(a), C.byref(b))
        nn_off = np.empty(V + 1, np.int64); ne_off = np.empty(V + 1, np.int64)
        nn = np.empty(max(a.value, 1), np.int32); ne = np.empty(max(b.value, 1), np.int32)
        lib().orc_export_rows(self.h, _p(nn_off), _p(nn), _p(ne_off), _p(ne))
        return nn_off, nn[:a.value], ne_off, ne[:b.value]

    def set_xy(self, v, x, y):
        lib().orc_set_xy(self.h, v, x, y)

    def set_metric(self, v, a, b, c):
        lib().orc_set_metric(self.h, v, a, b, c)

    def set_hook(self, fn):
        """fn(phase, round, cls, stage) called before (stage 0) and after
        (stage 1) every class; None removes it."""
        if fn is None:
            self._hook_ref = None
            lib().orc_set_hook(self.h, HOOK(0), None)
            return
        # an exception cannot cross the C frames: the first one is kept, later
        # calls are skipped, and the phase call raises it when it returns
        self._hook_exc = None

        def call(user, ph, r, c, st):
            if self._hook_exc is not None:
                return
            try:
                fn(ph, r, c, st)
            except BaseException as e:  # noqa: BLE001 - re-raised by _raise_hook
                self._hook_exc = e

        cb = HOOK(call)
        self._hook_ref = cb
        lib().orc_set_hook(self.h, cb, None)

    def _raise_hook(self):
        e = getattr(self, "_hook_exc", None)
        if e is not None:
            self._hook_exc = None
            raise e

    def class_members(self):
        n = lib().orc_class_members(self.h, None, 0)
        out = np.empty(max(n, 1), np.int32)
        lib().orc_class_members(self.h, _p(out), n)
        return out[:n]

    def class_whole(self):
        """The class the hook is called for, before re-validation."""
        n = lib().orc_class_whole(self.h, None, 0)
        out = np.empty(max(n, 1), np.int32)
        lib().orc_class_whole(self.h, _p(out), n)
        return out[:n]

    def set_order_seed(self, s: int):
        lib().orc_set_order_seed(self.h, s)

    def colour(self, active=None, ctx: int = 0):
        V, _ = self.sizes()
        out = np.empty(V, np.int32)
        act = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
        n = lib().orc_colour(self.h, _p(act), ctx, _p(out))
        return out, int(n)

    @staticmethod
    def _stats(st):
        return {k: int(st[i]) for i, k in enumerate(STAT_NAMES)}

    def coarsen(self, sweep=0, L_low2=0.5, q_min=0.1, max_rounds=200):
        st = np.zeros(NSTATS, np.int64)
        rc = lib().orc_coarsen(self.h, sweep, L_low2, q_min, max_rounds, _p(st))
        self._raise_hook()
        if rc < 0:
            raise RuntimeError(f"oracle coarsen failed: {rc}")
        return self._stats(st)

    def refine(self, L_up2=2.0, max_passes=32):
        st = np.zeros(NSTATS, np.int64)
        rc = lib().orc_refine(self.h, L_up2, max_passes, _p(st))
        self._raise_hook()
        if rc < 0:
            raise RuntimeError(f"oracle refine failed: {rc}")
        return self._stats(st)

    def swap(self, sweep=0, max_rounds=100):
        st = np.zeros(NSTATS, np.int64)
        rc = lib().orc_swap(self.h, sweep, max_rounds, _p(st))
        self._raise_hook()
        if rc < 0:
            raise RuntimeError(f"oracle swap failed: {rc}")
        return self._stats(st)

    def smooth(self, sweep=0, kind=0, sweeps=1):
        st = np.zeros(NSTATS, np.int64)
        rc = lib().orc_smooth(self.h, sweep, kind, sweeps, _p(st))
        self._raise_hook()
        if rc < 0:
            raise RuntimeError(f"oracle smooth failed: {rc}")
        return self._stats(st)

    def compact(self):
        lib().orc_compact(self.h)

    def quality(self, grad: bool = False):
        V, _ = self.sizes()
        Q = C.c_double(); qmin = C.c_double()
        gx = np.empty((V, 2)) if grad else None
        gm = np.empty((V, 3)) if grad else None
        lib().orc_quality(self.h, C.byref(Q), C.byref(qmin), _p(gx), _p(gm))
        if grad:
            return Q.value, qmin.value, gx, gm
        return Q.value, qmin.value

    def element_quality(self):
        _, T = self.sizes()
        q = np.empty(T)
        lib().orc_element_quality(self.h, _p(q))
        return q

    def patch_quality(self, v: int) -> float:
        return float(lib().orc_patch_quality(self.h, v))

    def adapt(self, max_iterations=8, max_phases=0, smooth_kind=0, smooth_sweeps=1, L_low2=0.5, L_up2=2.0,
              q_min=0.1, coarsen_rounds=200, swap_rounds=100, refine_passes=32):
        """Algorithm 1 from the mesh's loop state; returns (stats, finished)."""
        st = np.zeros(NSTATS, np.int64)
        rc = lib().orc_adapt(self.h, max_iterations, max_phases, smooth_kind, smooth_sweeps, L_low2, L_up2, q_min,
                             coarsen_rounds, swap_rounds, refine_passes, _p(st))
        self._raise_hook()
        if rc < 0:
            raise RuntimeError(f"oracle adapt failed: {rc}")
        return self._stats(st), rc == 0

    def get_context(self):
        it, ph, ch = C.c_int32(), C.c_int32(), C.c_int32()
        lib().orc_get_context(self.h, C.byref(it), C.byref(ph), C.byref(ch))
        return dict(iteration=it.value, phase=ph.value, changed=ch.value)

    def set_context(self, iteration, phase, changed):
        lib().orc_set_context(self.h, iteration, phase, changed)

    def sweep(self, sweep: int, smooth_kind: int = 0, smooth_sweeps: int = 1,
              L_low2=0.5, L_up2=2.0, q_min=0.1, coarsen_rounds=200, refine_passes=32, swap_rounds=100):
        """One outer sweep: coarsen -> refine -> swap -> smooth."""
        return dict(coarsen=self.coarsen(sweep, L_low2, q_min, coarsen_rounds),
                    refine=self.refine(L_up2, refine_passes),
                    swap=self.swap(sweep, swap_rounds),
                    smooth=self.smooth(sweep, smooth_kind, smooth_sweeps))


class OracleMesh3:
    """One tetrahedral mesh held by the oracle (coarsen, refine, smooth)."""

    def __init__(self, xyz, tet, metric, tags=None, seed: int = 0):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tet = np.ascontiguousarray(tet, dtype=np.int32)
        metric = np.ascontiguousarray(metric, dtype=np.float64)
        tg = None if tags is None else np.ascontiguousarray(tags, dtype=np.uint8)
        self.h = lib().orc3_create(xyz.shape[0], tet.shape[0], _p(xyz), _p(tet), _p(metric), _p(tg), seed)
        if not self.h:
            raise ValueError("oracle rejected the mesh")
        self._hook_ref = None
        self._hook_exc = None

    @classmethod
    def from_input(cls, mi, seed: int = 0):
        return cls(mi.xyz, mi.tet, mi.metric, mi.tags, seed)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc3_destroy(h)
            self.h = None

    def sizes(self):
        V = C.c_int64(); T = C.c_int64()
        lib().orc3_sizes(self.h, C.byref(V), C.byref(T))
        return V.value, T.value

    def export(self):
        V, T = self.sizes()
        xyz = np.empty((V, 3)); met = np.empty((V, 6))
        tet = np.empty((T, 4), np.int32)
        tags = np.empty(V, np.uint8); va = np.empty(V, np.uint8); ta = np.empty(T, np.uint8)
        lib().orc3_export(self.h, _p(xyz), _p(tet), _p(met), _p(tags), _p(va), _p(ta))
        return dict(xyz=xyz, tet=tet, metric=met, tags=tags, valive=va.astype(bool), talive=ta.astype(bool))

    def rows(self):
        V, _ = self.sizes()
        a = C.c_int64(); b = C.c_int64()
        lib().orc3_row_totals(self.h, C.byref(a), C.byref(b))
        nn_off = np.empty(V + 1, np.int64); ne_off = np.empty(V + 1, np.int64)
        nn = np.empty(max(a.value, 1), np.int32); ne = np.empty(max(b.value, 1), np.int32)
        lib().orc3_export_rows(self.h, _p(nn_off), _p(nn), _p(ne_off), _p(ne))
        return nn_off, nn[:a.value], ne_off, ne[:b.value]

    def set_xyz(self, v, x, y, z):
        lib().orc3_set_xyz(self.h, v, x, y, z)

    def set_hook(self, fn):
        """fn(phase, round, cls, stage) before (stage 0) and after (stage 1)
        every class; an exception in fn fails the phase call."""
        if fn is None:
            self._hook_ref = None
            lib().orc3_set_hook(self.h, HOOK(0), None)
            return
        self._hook_exc = None

        def call(user, ph, r, c, st):
            if self._hook_exc is not None:
                return
            try:
                fn(ph, r, c, st)
            except BaseException as e:  # noqa: BLE001 - re-raised by _raise_hook
                self._hook_exc = e

        cb = HOOK(call)
        self._hook_ref = cb
        lib().orc3_set_hook(self.h, cb, None)

    def _raise_hook(self):
        e = self._hook_exc
        if e is not None:
            self._hook_exc = None
            raise e

    def class_members(self):
        n = lib().orc3_class_members(self.h, None, 0)
        out = np.empty(max(n, 1), np.int32)
        lib().orc3_class_members(self.h, _p(out), n)
        return out[:n]

    def class_whole(self):
        n = lib().orc3_class_whole(self.h, None, 0)
        out = np.empty(max(n, 1), np.int32)
        lib().orc3_class_whole(self.h, _p(out), n)
        return out[:n]

    def colour(self, active=None, ctx: int = 0):
        V, _ = self.sizes()
        out = np.empty(V, np.int32)
        act = None if active is None else np.ascontiguousarray(active, np.uint8)
        n = lib().orc3_colour(self.h, _p(act), ctx, _p(out))
        return out, n

    def coarsen(self, sweep=0, L_low2=0.5, q_min=0.1, max_rounds=200):
        st = np.zeros(NSTATS, np.int64)
        rc = lib().orc3_coarsen(self.h, sweep, L_low2, q_min, max_rounds, _p(st))
        self._raise_hook()
        if rc < 0:
            raise RuntimeError(f"oracle coarsen failed: {rc}")
        return OracleMesh._stats(st)

    def refine(self, L_up2=2.0, max_passes=32):
        st = np.zeros(NSTATS, np.int64)
        rc = lib().orc3_refine(self.h, L_up2, max_passes, _p(st))
        self._raise_hook()
        if rc < 0:
            raise RuntimeError(f"oracle refine failed: {rc}")
        return OracleMesh._stats(st)

    def smooth(self, sweep=0, sweeps=1):
        st = np.zeros(NSTATS, np.int64)
        rc = lib().orc3_smooth(self.h, sweep, sweeps, _p(st))
        self._raise_hook()
        if rc < 0:
            raise RuntimeError(f"oracle smooth failed: {rc}")
        return OracleMesh._stats(st)

    def quality(self):
        Q = C.c_double(); qmin = C.c_double()
        lib().orc3_quality(self.h, C.byref(Q), C.byref(qmin))
        return Q.value, qmin.value

    def element_quality(self):
        _, T = self.sizes()
        q = np.empty(T)
        lib().orc3_element_quality(self.h, _p(q))
        return q

    def sweep(self, sweep: int, smooth_sweeps: int = 1, L_low2=0.5, L_up2=2.0, q_min=0.1):
        """One outer sweep: coarsen -> refine -> smooth (no swaps in 3D)."""
        return dict(coarsen=self.coarsen(sweep, L_low2, q_min), refine=self.refine(L_up2),
                    smooth=self.smooth(sweep, smooth_sweeps))
