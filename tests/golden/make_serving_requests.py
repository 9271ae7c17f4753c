"""Writes ``serving-requests-64.npz``: whole FP64 oracle solves of 64
requests of the serving trace (Poisson arrivals, seed 0;
k ~ logU[0.05, 0.5], sigma ~ logU[1, 10], sign controller, 3 x 21 search,
20 rounds), stratified by size: the first 48 of 1001 nodes and the first 16
of 4001 nodes in arrival order (an oracle solve takes about 3 s and 47 s).
The GPU test serves them in a mix with larger requests and compares every
round's J and the final controllers with these.

Calls only the oracle.  Run from the repository root:
    python tests/golden/make_serving_requests.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "serving-requests-64.npz")


def pick(trace):
    small = [r for r, q in enumerate(trace) if q.case.prob.n_x == 1001][:48]
    mid = [r for r, q in enumerate(trace) if q.case.prob.n_x == 4001][:16]
    return sorted(small + mid)


def main():
    trace = W.serving_trace()
    idx = pick(trace)
    out = {"index": np.array(idx)}
    t0 = time.time()
    for r in idx:
        c = trace[r].case
        u0, u1, J = oracle.solve(c.prob, c.search, c.iters, c.u0_init)
        out[f"J_{r}"], out[f"u0_{r}"], out[f"u1_{r}"] = J, u0, u1
        print(f"request {r}: n = {c.prob.n_x}, k = {c.prob.k:.4f}, sigma = {c.sigma:.3f}, "
              f"J {J[0]:.6f} -> {J[-1]:.6f} ({time.time() - t0:.0f} s)", flush=True)
    np.savez_compressed(OUT, **out)
    print(OUT)


if __name__ == "__main__":
    main()
