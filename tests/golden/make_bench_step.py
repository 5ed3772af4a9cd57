"""Writes bench_step_<n>.json: the oracle's result for bench.py's step on the
n x n jittered two-layer workload (default 2049; priority seed 1): op count
(vertices coloured + members evaluated + edges tested), the final topology
hash in bench.py's form, and the final quality. Calls only the oracle, the
input generator and bench.py's phase sequence.

Usage: python tests/golden/make_bench_step.py [n]   (about 20 s for 2049)
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from bench import PRIO_SEED, op_count, run_step, topo_hash  # noqa: E402
from oracle.orc import OracleMesh  # noqa: E402
from paper_1505_04694_amd import inputs  # noqa: E402


def main(n=2049):
    mi = inputs.config2(n)
    om = OracleMesh.from_input(mi, seed=PRIO_SEED)
    tr = run_step(om)
    out = dict(workload=f"{n}x{n} benchmark step, priority seed {PRIO_SEED}", input=mi.digest(), ops=op_count(tr),
               topology_hash=topo_hash(om.export()), final_quality=list(tr[-1][1]),
               phases={name: st for name, st in tr if isinstance(st, dict)})
    with open(os.path.join(HERE, f"bench_step_{n}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote bench_step_{n}.json", flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 2049)
