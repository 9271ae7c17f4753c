"""Pins of the oracle's generic solver (Algorithm 1, Sections III-B to
III-D) on the Witsenhausen instance: its local update (modified Newton on
the marginal cost), partial exhaustion over the domain ball of Eq. (2), the
adaptive allocation of a round's iterations, and the whole loop.  Each pin
rests on a closed form, finite differences or a 40-digit evaluation, not on
the oracle itself."""
import math

import mpmath as mp
import numpy as np
import pytest

import workloads as W

K = 0.2


def wide(n=2401, half=60.0, n_y=None, y_half=None, sw=1.0):
    return W.Problem(k=K, comps=[(1.0, 0.0, 5.0)], x_lo=-half, x_hi=half, n_x=n, y_lo=-(y_half or half),
                     y_hi=(y_half or half), n_y=n_y or n, noise_sd=sw)


@pytest.mark.parametrize("sw", [1.0, 0.7])
def test_derivatives_linear_u1_closed_form(orc, sw):
    """u1 = a y: B = k^2 u^2 + (1-a)^2 z^2 + a^2 sw^2, so B' = 2 k^2 u + 2 (1-a)^2 z
    and B'' = 2 k^2 + 2 (1-a)^2 (z = x + u).  Catches a wrong sign of t, the
    missing 2e term, t^2 without the -1/sw^2, and sw left at 1."""
    p = wide(n=201, half=20.0, n_y=4001, y_half=50.0, sw=sw)
    y = orc.grid(p.y_lo, p.y_hi, p.n_y)
    for a, x, u in ((0.3, 1.7, -0.4), (0.8, -3.0, 2.5), (0.5, 0.25, 7.0)):
        z = x + u
        B, B1, B2 = orc.B_derivs(p, a * y, x, u)
        assert abs(B - (K * K * u * u + (1 - a) ** 2 * z * z + a * a * sw * sw)) < 1e-12 * B
        assert abs(B1 - (2 * K * K * u + 2 * (1 - a) ** 2 * z)) < 1e-11 * (1 + abs(B1))
        assert abs(B2 - (2 * K * K + 2 * (1 - a) ** 2)) < 1e-11


def test_derivatives_against_central_differences(orc):
    """A nonlinear u1 (the closed form of the sign controller): B' and B''
    against central differences of B with h = 1e-4 (errors h^2 B'''/6 and
    the rounding of B over h^2)."""
    p = W.gaussian_problem(0.2, 5.0, 1001, 25.0)
    u1 = orc.update_u1(p, W.init_sign(p, 5.0))
    h = 1e-4
    for x, u in ((0.3, 4.0), (-2.0, -3.5), (7.5, -1.2), (1.0, 0.9)):
        B, B1, B2 = orc.B_derivs(p, u1, x, u)
        bp, bm = orc.B(p, u1, x, u + h), orc.B(p, u1, x, u - h)
        assert abs(B1 - (bp - bm) / (2 * h)) <= 1e-6 * (1 + abs(B1)), (x, u)
        assert abs(B2 - (bp - 2 * B + bm) / (h * h)) <= 1e-4 * (1 + abs(B2)), (x, u)


def test_newton_step_lands_on_convex_minimiser(orc):
    """With u1 = a y, B is a convex quadratic: one local update from any u0
    lands on u* = -(1-a)^2 x / (k^2 + (1-a)^2)."""
    p = wide(n=201, half=20.0, n_y=4001, y_half=60.0)
    y = orc.grid(p.y_lo, p.y_hi, p.n_y)
    x = orc.grid(p.x_lo, p.x_hi, p.n_x)
    rng = np.random.default_rng(3)
    for a in (0.3, 0.8):
        u0 = rng.uniform(-10, 10, p.n_x)
        out = orc.alg1_local_u0(p, 0.1, a * y, u0)
        ustar = -(1 - a) ** 2 * x / (K * K + (1 - a) ** 2)
        assert np.max(np.abs(out - ustar)) < 1e-10


def test_gradient_step_where_curvature_is_not_positive(orc):
    """Where B'' <= 0 the update is u - tau B'; elsewhere u - B'/B''."""
    p = W.gaussian_problem(0.05, 5.0, 401, 25.0)
    y = orc.grid(p.y_lo, p.y_hi, p.n_y)
    x = orc.grid(p.x_lo, p.x_hi, p.n_x)
    u1 = 5.0 * np.sign(y)  # a step decoder: B is concave between the steps
    u0 = np.full(p.n_x, 0.3) - 0.05 * x
    tau = 0.37
    out = orc.alg1_local_u0(p, tau, u1, u0)
    seen = set()
    for i in range(0, p.n_x, 5):
        B, B1, B2 = orc.B_derivs(p, u1, x[i], u0[i])
        want = u0[i] - B1 / B2 if B2 > 0 else u0[i] - tau * B1
        assert abs(out[i] - want) <= 1e-12 * (1 + abs(want))
        seen.add(B2 > 0)
    assert seen == {True, False}  # both branches exercised


def test_u1_newton_step_is_the_closed_form(orc):
    """C_1 is quadratic in u with C_1'' > 0: the local update of u1 lands on
    the conditional mean from any starting u1."""
    c = W.small_case()
    p = c.prob
    u0 = W.init_random_steps(p, 5.0, 4)
    start = np.random.default_rng(1).uniform(-20, 20, p.n_y)
    got = orc.alg1_local_u1(p, u0, start)
    ref = orc.update_u1(p, u0)
    assert np.max(np.abs(got - ref)) < 1e-12


def test_partial_exhaustion_u0_denoises_and_never_raises_cost(orc):
    """A smooth controller with a three-point spike: with r = 2 the domain
    ball of each spike point reaches a good neighbour, so one sweep removes
    the spike (an isolated wrong value is what the domain-ball search
    repairs); no point's cost rises, and the set holds the point's own
    value."""
    p = W.gaussian_problem(0.2, 5.0, 401, 25.0)
    x = orc.grid(p.x_lo, p.x_hi, p.n_x)
    good = 5.0 * np.sign(x) - x
    u1 = orc.update_u1(p, good)
    u0 = good.copy()
    sp = [150, 151, 152]
    u0[sp] = 20.0
    out = orc.alg1_pe_u0(p, u1, u0, r=2)
    for i in sp:
        assert orc.B(p, u1, x[i], out[i]) < orc.B(p, u1, x[i], u0[i])
        assert out[i] != 20.0
    for i in range(0, p.n_x, 7):
        assert orc.B(p, u1, x[i], out[i]) <= orc.B(p, u1, x[i], u0[i]) * (1 + 1e-12)
    # r = 1: the middle spike point sees only spike values and its own
    out1 = orc.alg1_pe_u0(p, u1, u0, r=1)
    assert out1[151] == 20.0


def test_partial_exhaustion_u1_never_raises_J(orc):
    c = W.small_case()
    p = c.prob
    u0 = W.init_random_steps(p, 5.0, 6)
    u1 = orc.update_u1(p, W.init_sign(p, 5.0))  # not the closed form of u0
    J0 = orc.objective(p, u0, u1)
    out = orc.alg1_pe_u1(p, u0, u1, r=2)
    J1 = orc.objective(p, u0, out)
    assert J1 < J0
    # each node moves to the candidate nearest the conditional mean of u0
    m = orc.update_u1(p, u0)
    for j in range(2, p.n_y - 2, 37):
        cands = u1[j - 2:j + 3]
        assert abs(out[j] - m[j]) <= np.min(np.abs(cands - m[j])) + 1e-12


@pytest.mark.parametrize("IL,IP,prev,want", [(3.0, 1.0, 10, (15, 5)), (0.0, 5.0, 10, (1, 19)), (5.0, 0.0, 10, (19, 1)),
                                             (1.0, 1.0, 3, (10, 10)), (0.0, 0.0, 7, (7, 13)),
                                             (1e-12, 2e-12, 10, (6, 14))])
def test_adaptive_allocation(orc, IL, IP, prev, want):
    """N_L = min(max(floor(I_L N / (I_L + I_P)), 1), N - 1), N_P = N - N_L,
    the previous split kept when both improvements vanish."""
    assert orc.alg1_allocate(20, IL, IP, prev) == want


def test_solve_loop(orc):
    """From the identity controllers (Section III-D, Initialization): J never
    rises over a partial-exhaustion phase, the first round splits N evenly,
    later rounds follow the allocation rule, and the loop stops once a
    round's improvements sum to at most p."""
    p = W.gaussian_problem(0.2, 5.0, 401, 25.0)
    x = orc.grid(p.x_lo, p.x_hi, p.n_x)
    y = orc.grid(p.y_lo, p.y_hi, p.n_y)
    u0, u1, J, NL = orc.alg1_solve(p, x.copy(), y.copy(), N=20, prec=1e-10, max_rounds=60)
    rounds = len(NL)
    assert 2 <= rounds < 60
    assert NL[0] == 10
    for t in range(rounds):
        assert J[2 + 2 * t] <= J[1 + 2 * t] * (1 + 1e-12)  # partial exhaustion phase
        if t + 1 < rounds:
            IL, IP = abs(J[2 * t] - J[1 + 2 * t]), abs(J[1 + 2 * t] - J[2 + 2 * t])
            assert orc.alg1_allocate(20, IL, IP, NL[t])[0] == NL[t + 1]
    IL, IP = abs(J[-3] - J[-2]), abs(J[-2] - J[-1])
    assert IL + IP <= 1e-10
    assert J[-1] < 0.2 < J[0]
    assert abs(J[-1] - orc.objective(p, u0, u1)) <= 1e-15 * J[-1]


def test_one_step_each_against_mpmath(orc):
    """One local update of u0 (derivatives by 40-digit numerical
    differentiation of B, not by the formula) and one partial exhaustion of
    u0 and of u1 (costs at 40 digits) on a 21 x 31 instance."""
    from oracle import mp_oracle

    p = W.Problem(k=0.2, comps=[(0.6, -3.0, 2.0), (0.4, 4.0, 3.0)], x_lo=-12, x_hi=12, n_x=21, y_lo=-15, y_hi=15,
                  n_y=31)
    u0 = W.init_random_steps(p, 4.0, 5)
    u1 = orc.update_u1(p, W.init_random_steps(p, 4.0, 8))
    got = orc.alg1_local_u0(p, 0.2, u1, u0)
    ref = mp_oracle.alg1_local_u0(p, 0.2, u1, u0)
    assert max(abs(a - float(b)) for a, b in zip(got, ref)) < 1e-10
    assert np.array_equal(orc.alg1_pe_u0(p, u1, u0, r=2), np.array(mp_oracle.alg1_pe_u0(p, u1, u0, 2)))
    assert np.array_equal(orc.alg1_pe_u1(p, u0, u1, r=2), np.array(mp_oracle.alg1_pe_u1(p, u0, u1, 2)))
