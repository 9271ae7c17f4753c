"""The u1 sums with several consecutive y nodes per lane, modelled in numpy
from their statement and checked against the oracle's u1 on the CPU; and
the generic solver's u1 partial exhaustion sums formed from moments.

Around the middle node y_c of a tile (eta_j = y_j - y_c, D_i = y_c - x1_i,
s the noise sd), the shifted log2 weight of x node i at y node j is
P_i + Q_j + E_j D_i with P_i = log2(e) (log f_i - D_i^2 / (2 s^2)),
Q_j = -log2(e) (M + eta_j^2 / (2 s^2)), E_j = -log2(e) eta_j / s^2.  A lane
holding nodes j0 .. j0 + 3 takes the first node's weight w_0 that way and
w_{m+1} = w_m R_i with R_i = exp2(-log2(e) dy D_i / s^2); w_m differs from
node j0 + m's weight by a factor that depends on neither i nor the x slice,
so u1_j = y_j - (sum w D + eta_j sum w) / sum w is unchanged by it.  One
shift M per lane, from its second node's logits.  Written here from that
statement alone; it shares nothing with the kernels.  It pins the reading
(the left-out factor cancels; one shift serves the lane) against the
oracle's u1 to rounding, and checks that the factor is not trivially 1."""
import math

import numpy as np
import pytest

import workloads as W

LOG2E = 1.0 / math.log(2.0)


def model_u1(orc, p, u0, npl=4, lanes=256):
    s = getattr(p, "noise_sd", 1.0)
    x = W.nodes(p.x_lo, p.x_hi, p.n_x)
    y = W.nodes(p.y_lo, p.y_hi, p.n_y)
    dy = (p.y_hi - p.y_lo) / (p.n_y - 1)
    _, logf = orc.prior(p)
    x1 = x + u0
    out = np.empty(p.n_y)
    factor_spread = 0.0
    tn = lanes * npl
    for j0 in range(0, p.n_y, tn):
        j1 = min(p.n_y, j0 + tn) - 1
        yc = p.y_lo + ((j0 + j1) // 2) * dy
        D = yc - x1
        P = LOG2E * (logf - D * D / (2 * s * s))
        R = np.exp2(-LOG2E * dy * D / (s * s))
        for jb in range(j0, j1 + 1, npl):
            eta0 = (p.y_lo + jb * dy) - yc
            etaR = eta0 + dy
            M = np.max(logf - (etaR + D) ** 2 / (2 * s * s))  # the second node's logits
            Q = -LOG2E * (M + eta0 * eta0 / (2 * s * s))
            E = -LOG2E * eta0 / (s * s)
            w = np.exp2(P + Q + E * D)
            for m in range(npl):
                j = jb + m
                if j > j1:
                    break
                if m:
                    w = w * R
                eta = (p.y_lo + j * dy) - yc
                num = np.sum(w * D) + eta * np.sum(w)
                out[j] = y[j] - num / np.sum(w)
                true = np.exp(logf - (y[j] - x1) ** 2 / (2 * s * s) - M)
                factor_spread = max(factor_spread, abs(np.sum(w) / np.sum(true) - 1.0))
    return out, factor_spread


@pytest.mark.parametrize("n_x,n_y,sw", [(301, 4096, 1.0), (257, 3001, 0.7), (199, 1537, 1.0)])
def test_nodes_per_lane_matches_oracle(orc, n_x, n_y, sw):
    p = W.Problem(0.2, [(0.5, -6.0, 2.0), (0.3, 3.0, 1.5), (0.2, 9.0, 3.0)], -20, 22, n_x, -40, 40, n_y)
    p.noise_sd = sw
    u0 = W.init_random_steps(p, 5.0, 3)
    ref = orc.update_u1(p, u0)
    got, spread = model_u1(orc, p, u0)
    # nodes with output density: the conditional mean is defined to rounding there
    f, _ = orc.prior(p)
    x1 = W.nodes(p.x_lo, p.x_hi, p.n_x) + u0
    y = W.nodes(p.y_lo, p.y_hi, p.n_y)
    py = np.array([np.sum(f * np.exp(-0.5 * ((yy - x1) / sw) ** 2)) for yy in y])
    m = py >= 1e-9 * py.max()
    assert np.max(np.abs(got[m] - ref[m])) <= 1e-11
    assert spread > 1e-6  # the left-out factor is real, and cancels


def test_partial_exhaustion_sums_from_moments(orc):
    """The u1 partial exhaustion of the generic solver forms each
    candidate's sum sum_i w (x1_i - c_m)^2 from the weighted moments about
    the node's own value, T_2 - 2 d T_1 + d^2 T_0 with d = c_m - u1_j.
    Checked against the direct sums, with u1 the conditional mean (as in
    the solver) and candidates up to jumps of the controller."""
    p = W.Problem(0.2, [(0.5, -6.0, 2.0), (0.3, 3.0, 1.5), (0.2, 9.0, 3.0)], -20, 22, 401, -40, 40, 1601)
    u0 = W.init_random_steps(p, 5.0, 5)
    u1 = orc.update_u1(p, u0)
    _, logf = orc.prior(p)
    x1 = W.nodes(p.x_lo, p.x_hi, p.n_x) + u0
    y = W.nodes(p.y_lo, p.y_hi, p.n_y)
    worst = 0.0
    for j in range(2, p.n_y - 2, 7):
        lw = logf - 0.5 * (y[j] - x1) ** 2
        w = np.exp(lw - lw.max())
        e = x1 - u1[j]
        T0, T1, T2 = np.sum(w), np.sum(w * e), np.sum(w * e * e)
        for c in list(u1[j - 2:j + 3]) + [u1[j] + 3.0, u1[j] - 7.5]:
            d = c - u1[j]
            direct = np.sum(w * (x1 - c) ** 2)
            worst = max(worst, abs(T2 - 2 * d * T1 + d * d * T0 - direct) / direct)
    assert worst <= 1e-13, worst
