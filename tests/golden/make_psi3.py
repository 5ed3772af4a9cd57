"""Writes psi3_29.json: the oracle's result for the 3D psi benchmark procedure
(the 29^3 Kuhn grid of the unit cube, psi extruded along z with eps for about
210k elements, priority seed 0; two iterations of coarsen then refine, then
one smoothing sweep). Calls only the oracle and the input generator; the GPU
test compares its own run with the file.

Usage: python tests/golden/make_psi3.py   (a few minutes on one core)
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.orc import OracleMesh3  # noqa: E402
from paper_1505_04694_amd import inputs  # noqa: E402

N, TARGET, ITERATIONS, SEED = 29, 210e3, 2, 0


def digest(a) -> str:
    return hashlib.sha256(a.tobytes()).hexdigest()[:32]


def summary(d) -> dict:
    """Hashes of the live mesh in slot order and the coordinate sum."""
    tet = d["tet"][d["talive"]]
    va = d["valive"]
    return dict(V=int(va.sum()), T=int(tet.shape[0]), tet=digest(tet), tags=digest(d["tags"][va]),
                xyz=digest(d["xyz"][va]), metric=digest(d["metric"][va]), xyz_sum=float(d["xyz"][va].sum()))


def main():
    t0 = time.time()
    mi = inputs.psi_start3(N, target=TARGET)
    om = OracleMesh3.from_input(mi, seed=SEED)
    phases = []
    for it in range(ITERATIONS):
        phases.append(dict(iteration=it, coarsen=om.coarsen(it), refine=om.refine()))
        print(f"iteration {it}: {om.sizes()} ({time.time() - t0:.0f} s)", flush=True)
    smooth = om.smooth(0, 1)
    Q, qmin = om.quality()
    out = dict(workload=f"psi extruded along z, {N}^3 Kuhn grid, ~{TARGET:.0f} elements, priority seed {SEED}; "
                        f"{ITERATIONS} x (coarsen, refine), one smoothing sweep",
               input=mi.digest(), final=summary(om.export()), quality=[Q, qmin], phases=phases, smooth=smooth)
    with open(os.path.join(HERE, "psi3_29.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote psi3_29.json in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
