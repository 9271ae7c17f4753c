"""Writes ``sweep-seed0-20001-10r.npz``: the FP64 oracle's 10-round
trajectories of the precision sweep's seed-0 instances: grids of 20001
nodes, k in {0.05, 0.2, 0.5} x sigma in {1, 5, 10} (ranges and 5 x 16
search as the sweep takes them), the random 8-step initial controller of
seed 0.  Stored per instance: J after every round (J[0] is the initial
controller's), and u0 and u1 after round 10 on 1024 sampled x and y rows
(the rows stored beside them).

Calls only the oracle.  Run from the repository root (about 90 minutes on
8 cores):  python tests/golden/make_sweep_seed0_trajectories.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sweep-seed0-20001-10r.npz")
ROUNDS = 10
ROWS = 1024


def main():
    cases = W.sweep_cases(n=20001, seeds=[0])
    rng = np.random.default_rng(0)
    out = {"names": np.array([c.name for c in cases])}
    t0 = time.time()
    for q, c in enumerate(cases):
        p, s = c.prob, c.search
        u0, u1, J = oracle.solve(p, s, ROUNDS, c.u0_init)
        xr = np.sort(rng.choice(p.n_x, ROWS, replace=False))
        yr = np.sort(rng.choice(p.n_y, ROWS, replace=False))
        out[f"J_{q}"], out[f"xrows_{q}"], out[f"yrows_{q}"] = J, xr, yr
        out[f"u0_{q}"], out[f"u1_{q}"] = u0[xr], u1[yr]
        print(f"{c.name}: J {J[0]:.6f} -> {J[-1]:.6f} ({time.time() - t0:.0f} s)", flush=True)
    np.savez_compressed(OUT, **out)
    print(OUT)


if __name__ == "__main__":
    main()
