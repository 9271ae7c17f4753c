"""The expansion behind the moment table (the Gauss-transform arithmetic
UCP_FP64_GT, and the FP64 tie values of the FP32 searches), checked on the
CPU against the oracle's dense B.  About a centre c (delta = z - c,
d = delta / s, t_j = (y_j - c) / s),
  dy sum_j phi_s(y_j - z)(z - u1_j)^2
    = dy/(s sqrt(2 pi)) e^{-d^2/2} sum_n d^n / n! [A2_n + 2 delta A1_n + delta^2 A0_n],
  A_a,n = sum_{|j - k| <= nw} e^{-t_j^2/2} t_j^n (c - u1_j)^a,
truncated at order 12, the centres every m-th node (m the largest stride
with m dy / s <= 0.05 whose truncation bound x^13 / 13! / (1 - x / 14),
x = (m dy / 2s) (nw dy / s), is below 1e-17), running from nw nodes before
the grid to nw past it; a position with no centre within half a stride has
no grid node in its window and a noise sum of 0.  Written here in numpy from
that statement alone; it shares nothing with the kernels.  It pins the
reading that the strided, truncated, windowed expansion reproduces the dense
cost to rounding (1e-14; the dense reference sums themselves differ by
about that on 65536 nodes), over the whole grid and beyond both ends, and
that lower orders leave visible error where the stride is long."""
import math

import numpy as np
import pytest

import workloads as W

ORDER = 12


def stride(dy, s, win=11.0):
    r = dy / s
    if r > 0.05 * (1 + 1e-12):
        return 0
    nw = math.ceil(win * s / dy)
    T = nw * r
    for m in range(max(1, math.floor(0.05 / r * (1 + 1e-12))), 0, -1):
        x = 0.5 * m * r * T
        if x ** (ORDER + 1) / math.factorial(ORDER + 1) / (1 - x / (ORDER + 2)) <= 1e-17:
            return m
    return 0


def gt_B(p, u1, x, u, m, N=ORDER):
    s = getattr(p, "noise_sd", 1.0)
    dy = (p.y_hi - p.y_lo) / (p.n_y - 1)
    z = x + u
    nw = min(math.ceil(11.0 * s / dy), p.n_y)
    off = -(-nw // m) * m  # centres from -off to n_y - 1 + off (or just past)
    rows = (p.n_y - 1 + 2 * off + m - 1) // m + 1
    r = int(np.rint((z - p.y_lo) / (m * dy))) + off // m
    if not 0 <= r < rows:
        return p.k ** 2 * u * u  # no grid node within the window
    k = r * m - off
    c = p.y_lo + k * dy
    delta = z - c
    assert abs(delta) <= 0.5 * m * dy * (1 + 1e-12)
    j = np.arange(max(0, k - nw), min(p.n_y - 1, k + nw) + 1)
    y = W.nodes(p.y_lo, p.y_hi, p.n_y)
    t = (y[j] - c) / s
    g = np.exp(-0.5 * t * t)
    v = c - u1[j]
    d = delta / s
    tot = 0.0
    for n in range(N, -1, -1):
        tn = t ** n
        C = np.sum(g * tn * v * v) + 2 * delta * np.sum(g * tn * v) + delta * delta * np.sum(g * tn)
        tot = C + tot * d / (n + 1)
    return p.k ** 2 * u * u + dy / (s * math.sqrt(2 * math.pi)) * math.exp(-0.5 * d * d) * tot


def test_stride_rule():
    # the grids of the workloads: 65536 nodes on [-40, 40], 20001 and 4001 on
    # [-25, 25], and the coarsest admitted spacing (dy / s = 0.05)
    assert stride(80 / 65535, 1.0) == 40
    assert stride(50 / 20000, 1.0) == 20
    assert stride(50 / 4000, 1.0) == 4
    assert stride(0.05, 1.0) == 1
    assert stride(0.0501, 1.0) == 0


@pytest.mark.parametrize("n,half,sigma,k,sw", [(1001, 25.0, 5.0, 0.2, 1.0), (20001, 25.0, 5.0, 0.2, 1.0),
                                               (2001, 50.0, 10.0, 0.05, 1.0), (1601, 25.0, 4.0, 0.25, 0.7)])
def test_expansion_matches_dense_sum(orc, n, half, sigma, k, sw):
    p = W.gaussian_problem(k, sigma, n, half)
    p.noise_sd = sw
    m = stride((p.y_hi - p.y_lo) / (p.n_y - 1), sw)
    assert m >= 1
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
            worst = max(worst, abs(gt_B(p, u1, x[i], u, m) - ref) / ref)
    assert worst <= 1e-14, worst


def test_long_stride_whole_range(orc):
    """The 65536-node grid (stride 40, positions up to 0.0244 noise sds
    from their centre), a steep u1, positions over the whole grid and
    beyond either end (partial windows, and none at all past 11 sds)."""
    p = W.gaussian_problem(0.2, 5.0, 65536, 40.0)
    dy = (p.y_hi - p.y_lo) / (p.n_y - 1)
    m = stride(dy, 1.0)
    y = W.nodes(p.y_lo, p.y_hi, p.n_y)
    u1 = 5.0 * np.tanh(y) + 0.2 * np.sin(7 * y)
    rows = (p.n_y - 1 + m - 1) // m + 1
    rng = np.random.default_rng(3)
    zs = list(rng.uniform(p.y_lo, p.y_hi, 24))
    zs += [p.y_lo + (r + 0.49) * m * dy for r in rng.integers(0, rows - 1, 8)]  # far from centres
    zs += [p.y_lo - 3.0, p.y_hi + 7.5, p.y_lo - 10.99, p.y_hi + 10.99, p.y_hi + 11.5, p.y_lo - 25.0]  # beyond
    worst = 0.0
    for z in zs:
        ref = orc.B(p, u1, 0.3, z - 0.3)
        worst = max(worst, abs(gt_B(p, u1, 0.3, z - 0.3, m) - ref) / ref)
    assert worst <= 2e-14, worst


def test_truncation_matters(orc):
    """Where the stride is long (40 nodes, |d| up to 0.0244) low orders
    leave visible error and order 12 reaches rounding: the expansion is not
    exact by accident of a flat u1."""
    p = W.gaussian_problem(0.2, 5.0, 65536, 40.0)
    dy = (p.y_hi - p.y_lo) / (p.n_y - 1)
    m = stride(dy, 1.0)
    y = W.nodes(p.y_lo, p.y_hi, p.n_y)
    u1 = 5.0 * np.tanh(y)
    rows = (p.n_y - 1 + m - 1) // m + 1
    z = p.y_lo + (rows // 2 + 7 + 0.49) * m * dy  # 0.49 of a stride off a centre near y = 2
    x, u = 0.3, z - 0.3
    ref = orc.B(p, u1, x, u)
    err = [abs(gt_B(p, u1, x, u, m, N=N) - ref) / ref for N in (1, 3, ORDER)]
    assert err[0] > 1e-8 and err[1] > 1e-13 and err[2] <= 2e-14, err
