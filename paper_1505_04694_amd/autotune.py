"""Autotuner of the kernel shapes (pm_tuning) for a given mesh or batch.

Every pm_tuning choice gives bit-identical meshes; the choices trade lanes per
class member, members per commit work-group, one-block kernels for small
lists and the size of the first class-list table against each other, and the
best one depends on the mesh sizes. The tuner runs one adaptation sweep
(coarsen, refine, swap, smooth) on fresh copies of the caller's meshes for
each candidate, times it on the device, checks that the copies come out
identical, and keeps the fastest choice, one knob at a time (coordinate
descent from the defaults). Results are cached in a JSON file keyed by the
device name and the mesh sizes rounded to a power of two.
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import time

from . import pmesh

# candidate values per knob, the default first
SPACE = {
    "op_lanes": [16, 8, 1],
    "commit_chunk": [0, 32, 64, 128],
    "smooth_lanes": [8, 1],
    "small_work": [0, 1],
    "class_colours": [32, 256],
    "commit_order": [0, 1, 2],
    "host_rounds": [0, 1, 2],
}
CACHE_ENV = "PMESH_TUNE_CACHE"


def cache_path() -> str:
    return os.environ.get(CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache", "pmesh", "tune.json")


def _bucket(x: int) -> int:
    return 1 << max(0, int(math.ceil(math.log2(max(x, 1)))))


def cache_key(meshes) -> str:
    import torch
    V = sum(int(m[0].shape[0]) for m in meshes)
    T = sum(int(m[1].shape[0]) for m in meshes)
    return f"{torch.cuda.get_device_name()}|B{len(meshes)}|V{_bucket(V)}|T{_bucket(T)}"


def _digest(handle) -> str:
    """Hash of a handle's meshes (every mesh of a batch)."""
    h = hashlib.sha256()
    if isinstance(handle, pmesh.Batch):
        for i in range(handle.count()):
            e = handle.export_mesh(i)
            for k in ("xy", "tri", "tags"):
                h.update(e[k].tobytes())
    else:
        e = handle.export()
        for k in ("xy", "tri", "tags"):
            h.update(e[k].tobytes())
    return h.hexdigest()


def _run(meshes, seed, tune, repeats):
    """Best time of `repeats` sweeps, each on a fresh copy; the result's digest."""
    import torch
    best, dig = float("inf"), None
    for _ in range(repeats):
        if len(meshes) == 1:
            h = pmesh.Mesh(*meshes[0], seed=seed, tune=tune)
        else:
            h = pmesh.Batch(meshes, seed=seed, tune=tune)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.sweep(0)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
        d = _digest(h)
        h.close()
        if dig is not None and d != dig:
            raise RuntimeError("a sweep gave different meshes on two runs")
        dig = d
    return best, dig


def autotune(meshes, seed: int = 0, repeats: int = 2, use_cache: bool = True, log=None):
    """meshes: list of (xy, tri, metric, tags) host arrays (one: a single
    mesh; more: a batch). Returns (tuning dict, report) where report lists
    every candidate's time and the digest all of them produced."""
    key = cache_key(meshes)
    path = cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return dict(cache[key]["tune"]), dict(cached=True, key=key)
    best = {k: v[0] for k, v in SPACE.items()}
    t_best, digest = _run(meshes, seed, best, repeats)
    tried = [dict(tune=dict(best), seconds=t_best)]
    for knob, values in SPACE.items():
        for v in values[1:]:
            cand = dict(best)
            cand[knob] = v
            t, d = _run(meshes, seed, cand, repeats)
            tried.append(dict(tune=dict(cand), seconds=t))
            if d != digest:
                raise RuntimeError(f"tuning {cand} changed the result")
            if log:
                log(f"{cand}: {t * 1e3:.2f} ms")
            if t < t_best:
                best, t_best = cand, t
    report = dict(key=key, best=best, seconds=t_best, digest=digest, tried=tried, cached=False)
    if use_cache:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        cache[key] = dict(tune=best, seconds=t_best)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, path)
    return dict(best), report
