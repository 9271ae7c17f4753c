"""The expansion behind the Gauss-transform arithmetic (UCP_FP64_GT), checked
on the CPU against the oracle's dense B.  For z within half a spacing of a
y node y_k, with delta = z - y_k and t_j = (y_j - y_k) / s,
  dy sum_j phi_s(y_j - z)(z - u1_j)^2
    = dy/(s sqrt(2 pi)) e^{-(delta/s)^2/2} sum_n (delta/s)^n / n!
      [A2_n + 2 delta A1_n + delta^2 A0_n],
  A_a,n = sum_{|t_j| <= 11} e^{-t_j^2/2} t_j^n (y_k - u1_j)^a,
truncated at the order N whose term bound (h T)^{N+1} / (N+1)! is below
1e-17 (h = dy / (2 s), T the window).  Written here in numpy from that
statement alone; it shares nothing with the kernels.  It pins the reading
that the truncated, windowed expansion reproduces the dense cost to about
1e-15 (the GPU tests hold the kernels to 1e-13), and that one order less
than the bound asks for is visibly worse where h T is largest."""
import math

import numpy as np
import pytest

import workloads as W


def order(dy, s, win=11.0):
    h = 0.5 * dy / s
    T = (math.ceil(win * s / dy) + 0.5) * dy / s
    x = h * T
    term = x
    for n in range(0, 40):
        if term <= 1e-17:
            return max(n, 2)
        term *= x / (n + 2)


def gt_B(p, u1, x, u, N=None):
    s = getattr(p, "noise_sd", 1.0)
    dy = (p.y_hi - p.y_lo) / (p.n_y - 1)
    y = W.nodes(p.y_lo, p.y_hi, p.n_y)
    z = x + u
    k = int(np.clip(np.rint((z - p.y_lo) / dy), 0, p.n_y - 1))
    delta = z - y[k]
    assert abs(delta) <= 0.5 * dy * (1 + 1e-12)
    nw = min(math.ceil(11.0 * s / dy), p.n_y)
    j = np.arange(max(0, k - nw), min(p.n_y - 1, k + nw) + 1)
    t = (y[j] - y[k]) / s
    g = np.exp(-0.5 * t * t)
    v = y[k] - u1[j]
    N = order(dy, s) if N is None else N
    d = delta / s
    tot = 0.0
    for n in range(N, -1, -1):
        tn = t ** n
        C = np.sum(g * tn * v * v) + 2 * delta * np.sum(g * tn * v) + delta * delta * np.sum(g * tn)
        tot = C + tot * d / (n + 1)
    return p.k ** 2 * u * u + dy / (s * math.sqrt(2 * math.pi)) * math.exp(-0.5 * d * d) * tot


@pytest.mark.parametrize("n,half,sigma,k,sw", [(1001, 25.0, 5.0, 0.2, 1.0), (20001, 25.0, 5.0, 0.2, 1.0),
                                               (2001, 50.0, 10.0, 0.05, 1.0), (1201, 25.0, 4.0, 0.25, 0.7)])
def test_expansion_matches_dense_sum(orc, n, half, sigma, k, sw):
    p = W.gaussian_problem(k, sigma, n, half)
    p.noise_sd = sw
    u1 = orc.update_u1(p, W.init_sign(p, sigma))
    x = orc.grid(p.x_lo, p.x_hi, p.n_x)
    rng = np.random.default_rng(n)
    worst = 0.0
    for i in rng.choice(p.n_x, 24, replace=False):
        for u in rng.uniform(-half, half, 3).tolist() + [sigma * np.sign(x[i]) - x[i]]:
            z = x[i] + u
            if not p.y_lo <= z <= p.y_hi:
                continue
            ref = orc.B(p, u1, x[i], u)
            worst = max(worst, abs(gt_B(p, u1, x[i], u) - ref) / ref)
    assert worst <= 1e-14, worst


def test_truncation_matters():
    """On the coarsest admitted grid (dy / s = 0.05, order 12 by the bound)
    low orders leave visible error and the bound's order reaches rounding:
    the expansion is not exact by accident of a flat u1.  (The bound is
    conservative: the Gaussian weights make order 7 enough here.)"""
    p = W.gaussian_problem(0.2, 5.0, 1001, 25.0)
    assert order(0.05, 1.0) == 12
    y = W.nodes(p.y_lo, p.y_hi, p.n_y)
    u1 = 5.0 * np.tanh(y)
    import oracle

    oracle.lib()
    x, u = 0.3, 2.0 + 0.025  # half a spacing off the node
    ref = oracle.B(p, u1, x, u)
    err = [abs(gt_B(p, u1, x, u, N=N) - ref) / ref for N in (2, 4, 12)]
    assert err[0] > 1e-7 and err[1] > 1e-10 and err[2] <= 1e-14, err
