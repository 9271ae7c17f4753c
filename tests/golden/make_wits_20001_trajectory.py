"""Writes ``wits-20001-5x16-30r.npz``: the FP64 oracle's whole trajectory of
the 20001-node Witsenhausen solve (k = 0.2, sigma = 5, grids of 20001 nodes
on [-25, 25], 5 levels x 16 candidates on [-30, 30], u0 = 5 sign(x) - x,
30 rounds), for the GPU trajectory test.

Calls only the oracle: each round is one call of the oracle's own solve loop
from the previous round's u0 (a solve resumed from its output continues the
same trajectory; the CPU pins check that).  Stored: J after every round
(J_hist[0] is the initial controller's), u0 after rounds 1 and 30, u1 after
round 30, and a SHA-256 of u0 after every round.

Run from the repository root:  python tests/golden/make_wits_20001_trajectory.py
(about 15 minutes on 8 cores).
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "wits-20001-5x16-30r.npz")


def main():
    c = W.paper_res_case()
    p, s = c.prob, c.search
    u0 = c.u0_init.copy()
    J = []
    sha = []
    u0_r1 = None
    t0 = time.time()
    for t in range(c.iters):
        u0, u1, Jh = oracle.solve(p, s, 1, u0)
        if t == 0:
            J.append(Jh[0])
            u0_r1 = u0.copy()
        J.append(Jh[1])
        sha.append(hashlib.sha256(u0.tobytes()).hexdigest())
        print(f"round {t + 1}: J = {Jh[1]:.17g}  ({time.time() - t0:.0f} s, {oracle.num_threads()} threads)",
              flush=True)
    np.savez_compressed(OUT, J_hist=np.array(J), u0_round1=u0_r1, u0_final=u0, u1_final=u1,
                        u0_sha256=np.array(sha), threads=oracle.num_threads())
    print(OUT)


if __name__ == "__main__":
    main()
