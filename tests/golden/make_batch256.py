"""Writes batch256.json: the oracle's result for every mesh of the batched
workload (256 unit-square meshes, n log-uniform in [17, 513] from seed 2,
per-mesh layer parameters; priority seed 2; two sweeps of coarsen -> refine
-> swap -> plain smoothing), each mesh run alone. Calls only the oracle and
the input generator; the GPU test runs the whole batch through one batched
handle and compares every mesh with the file.

Usage: python tests/golden/make_batch256.py   (a few seconds on 8 cores)
"""
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

COUNT, SWEEPS, SEED = 256, 2, 2


def digest(a) -> str:
    return hashlib.sha256(a.tobytes()).hexdigest()[:32]


def summary(d) -> dict:
    """Hashes of the live mesh in slot order (topology, tags, coordinates),
    and the coordinate sum for a tolerance check."""
    tri = d["tri"][d["talive"]]
    va = d["valive"]
    return dict(V=int(va.sum()), T=int(tri.shape[0]), tri=digest(tri), tags=digest(d["tags"][va]),
                xy=digest(d["xy"][va]), xy_sum=float(d["xy"][va].sum()))


def one_mesh(args):
    i, p = args
    sys.path.insert(0, ROOT)
    from oracle.orc import OracleMesh
    from paper_1505_04694_amd import inputs
    mi = inputs.make_mesh(p["n"], amp=p["amp"], width=p["width"], ht=p["ht"])
    om = OracleMesh.from_input(mi, seed=SEED)
    ops = 0
    for s in range(SWEEPS):
        tr = om.sweep(s)
        ops += sum(st["coloured"] + st["evaluated"] + st["edges"] for st in tr.values())
    return i, dict(n=p["n"], ops=ops, final=summary(om.export()))


def main():
    from paper_1505_04694_amd import inputs
    t0 = time.time()
    params = inputs.batch_params(COUNT, SEED)
    order = sorted(enumerate(params), key=lambda ip: -ip[1]["n"])  # largest first
    with mp.get_context("spawn").Pool(min(8, len(os.sched_getaffinity(0)))) as pool:
        res = dict(pool.map(one_mesh, order, chunksize=1))
    out = dict(workload=f"{COUNT} meshes (n log-uniform in [17, 513], seed {SEED}), priority seed {SEED}; "
                        f"{SWEEPS} sweeps coarsen -> refine -> swap -> plain smoothing, each mesh alone",
               meshes=[res[i] for i in range(COUNT)])
    with open(os.path.join(HERE, "batch256.json"), "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote batch256.json in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
