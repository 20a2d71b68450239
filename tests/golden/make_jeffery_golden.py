"""Writes tests/golden/jeffery_single_fiber.json: the tumbling period of the
single-fiber 32^3 shear cell (cylinder L = 16, d = 4, tau = 0.8, density
ratio 1, Lambda = 3/16, wall speed U) computed by the FP64 oracle.  Calls
only oracle/ (plus the seeded input generator and the period measurement).

    OMP_NUM_THREADS=6 python tests/golden/make_jeffery_golden.py --seed 0 --wall-u 0.02 --steps 62000

Entries are keyed "U<wall speed>/seed<seed>" (U = 0.005: 190000 steps,
about two periods; U = 0.02: 62000 steps).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

from oracle import pyoracle as O          # noqa: E402
from paper_1503_06869_amd import scenarios  # noqa: E402
from paper_1503_06869_amd import jeffery  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "jeffery_single_fiber.json")


def run(seed, steps, wall_u, chunk=10000):
    sc = scenarios.single_fiber(seed=seed, wall_u=wall_u)
    f = sc.fibers[0]
    s = O.Sim(sc.nx, sc.ny, sc.nz, tau=sc.tau, magic=sc.magic, wall_u=sc.wall_u,
              init_couette=True, coupling="implicit")
    s.add_fiber(f.X, f.q, f.length, f.radius, f.density_ratio, f.V, f.W)
    tx = np.zeros(steps)
    t0 = time.time()
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        s.step(k)
        h = s.history(done, k)
        tx[done:done + k] = jeffery.axis_from_quat(h[:, 0, 9:13])[:, 0]
        done += k
        print("seed %d: %d/%d steps, %.0f s" % (seed, done, steps, time.time() - t0), flush=True)
    T, cr = jeffery.period(tx)
    return {"period": T, "crossings": cr.tolist(), "steps": steps,
            "shear_rate": sc.shear_rate, "seconds": time.time() - t0,
            "axis0": jeffery.axis_from_quat(f.q).tolist(),
            "tx_every_100": tx[::100].tolist()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seed", type=int, action="append")
    ap.add_argument("--steps", type=int, default=62000)
    ap.add_argument("--wall-u", type=float, default=0.02)
    a = ap.parse_args()
    data = {}
    if os.path.exists(OUT):
        data = json.load(open(OUT))
    data.setdefault("about", "oracle (FP64) tumbling period of the single-fiber 32^3 shear "
                    "cell; crossings of the axis x-component; written by "
                    "tests/golden/make_jeffery_golden.py")
    for seed in a.seed or [0]:
        key = "U%g/seed%d" % (a.wall_u, seed)
        data[key] = run(seed, a.steps, a.wall_u)
        data[key]["wall_u"] = a.wall_u
        json.dump(data, open(OUT, "w"), indent=1)
        print(key, "period", data[key]["period"], flush=True)


if __name__ == "__main__":
    main()
