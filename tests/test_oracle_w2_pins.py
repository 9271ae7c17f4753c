"""Pins of the oracle's two-dimensional Witsenhausen functions (Section
V-D) against the one-dimensional oracle, which the other CPU tests pin to
closed forms.  With a separable controller and independent coordinates the
2-D sums factor into 1-D ones: J_2D = J_1D * Mx with Mx = dx sum f (the
prior's mass on the grid), and B_2D is the mean of the two 1-D costs with
each noise term weighted by the other coordinate's noise mass
My(z) = dy sum_j phi(y_j - z).
"""
import numpy as np
import pytest

import workloads as W


def base(n=21, n_y=101):
    # dy = 0.5: the rectangle rule of the N(0,1) density errs by ~exp(-2 pi^2 / dy^2) = 1e-34
    return W.w2_problem(n, n_y)


def test_separable_decoder_and_objective(orc):
    # catches a swapped plane, a missing 1/2, a dx or dy power, a wrong prior product
    p = base()
    x = W.nodes(p.x_lo, p.x_hi, p.n_x)
    g = 5.0 * np.sign(x) - x + 0.3 * np.sin(x)
    u0 = W.w2_separable(p, g)
    u1 = orc.w2_update_u1(p, u0)
    v = orc.update_u1(p, g)
    ny = p.n_y
    assert np.max(np.abs(u1[0] - np.repeat(v, ny))) < 1e-11
    assert np.max(np.abs(u1[1] - np.tile(v, ny))) < 1e-11
    J2 = orc.w2_objective(p, u0, u1)
    J1 = orc.objective(p, g, v)
    f, _ = orc.prior(p)
    Mx = (p.x_hi - p.x_lo) / (p.n_x - 1) * f.sum()
    assert abs(J2 - J1 * Mx) < 1e-12 * J1


def test_separable_marginal_cost(orc):
    p = base(n=11)
    x = W.nodes(p.x_lo, p.x_hi, p.n_x)
    rng = np.random.default_rng(2)
    v = rng.uniform(-8, 8, p.n_y)
    u1 = np.stack([np.repeat(v, p.n_y), np.tile(v, p.n_y)])
    y = W.nodes(p.y_lo, p.y_hi, p.n_y)
    dy = (p.y_hi - p.y_lo) / (p.n_y - 1)
    My = lambda z: dy * np.sum(np.exp(-0.5 * (y - z) ** 2)) / np.sqrt(2 * np.pi)
    k2 = p.k ** 2
    for (i1, i2, ua, ub) in [(3, 7, 1.5, -2.0), (0, 10, -6.0, 4.0), (5, 5, 0.0, 0.0)]:
        B2 = orc.w2_B(p, u1, (x[i1], x[i2]), (ua, ub))
        S1 = orc.B(p, v, x[i1], ua) - k2 * ua * ua
        S2 = orc.B(p, v, x[i2], ub) - k2 * ub * ub
        ref = 0.5 * (k2 * (ua * ua + ub * ub) + S1 * My(x[i2] + ub) + S2 * My(x[i1] + ua))
        assert abs(B2 - ref) < 1e-12 * ref
    # L_0 = f(x1) f(x2) B
    f, _ = orc.prior(p)
    u = rng.uniform(-5, 5, (2, p.n_x ** 2, 3))
    L = orc.w2_marginal_cost(p, u1, u)
    for i, c in [(0, 0), (17, 2), (120, 1)]:
        B2 = orc.w2_B(p, u1, (x[i // p.n_x], x[i % p.n_x]), (u[0, i, c], u[1, i, c]))
        assert abs(L[i, c] - f[i // p.n_x] * f[i % p.n_x] * B2) <= 1e-14 * abs(L[i, c])


def test_search_linear_decoder_closed_form(orc):
    # u1(y) = a y gives |z - u1|^2 = |(1 - a) z - a w|^2, so
    # B = 1/2 [k^2 |u|^2 + (1 - a)^2 |x + u|^2 + 2 a^2] (interior z), which
    # the search must minimise: u* = -(1 - a)^2 x / (k^2 + (1 - a)^2).  The
    # search range keeps every candidate's z = x + u well inside the y grid
    # (a z outside it would see no noise cost, an artefact of the truncation)
    p = W.w2_problem(11, 61)
    a = 0.5
    y = W.nodes(p.y_lo, p.y_hi, p.n_y)
    u1 = a * np.stack([np.repeat(y, p.n_y), np.tile(y, p.n_y)])
    x = W.nodes(p.x_lo, p.x_hi, p.n_x)
    xs = np.stack([np.repeat(x, p.n_x), np.tile(x, p.n_x)])
    s = W.Search(-12.0, 12.0, 4, 9)
    u, B = orc.w2_argmin(p, s, u1, np.zeros((2, p.n_x ** 2)))
    ustar = -(1 - a) ** 2 * xs / (p.k ** 2 + (1 - a) ** 2)
    inner = np.all(np.abs(xs) <= 10.0, axis=0)
    assert np.max(np.abs(u[:, inner] - ustar[:, inner])) < 0.1
    Bstar = 0.5 * (p.k ** 2 * (ustar ** 2).sum(0) + (1 - a) ** 2 * ((xs + ustar) ** 2).sum(0) + 2 * a * a)
    assert np.all(B[inner] >= Bstar[inner] - 1e-6) and np.all(B[inner] - Bstar[inner] < 0.01)


def test_coordinate_swap_symmetry(orc):
    p = W.w2_problem(13, 17)
    u0 = W.w2_init(p, 4)
    n = p.n_x
    sw = lambda a, m: a.reshape(2, m, m).transpose(0, 2, 1)[::-1].reshape(2, m * m)
    u1 = orc.w2_update_u1(p, u0)
    u1s = orc.w2_update_u1(p, sw(u0, n))
    assert np.max(np.abs(u1s - sw(u1, p.n_y))) < 1e-12
    assert abs(orc.w2_objective(p, u0, u1) - orc.w2_objective(p, sw(u0, n), u1s)) < 1e-12


def test_solve_monotone_and_rows(orc):
    c = W.w2_small_case()
    u0, u1, J = orc.w2_solve(c.prob, c.search, 2, c.u0_init)
    assert np.all(np.diff(J) <= 1e-12 * J[:-1]) and J[-1] < J[0]
    rows = np.array([0, 7, 220, 440])
    full, _ = orc.w2_argmin(c.prob, c.search, u1, u0)
    part, _ = orc.w2_argmin(c.prob, c.search, u1, u0, rows)
    assert np.array_equal(full[:, rows], part)


def test_tie_rule_on_mirror_symmetric_minima(orc):
    # x = (0, 0) with an odd decoder u1 = 5 sign(y) per coordinate on a
    # symmetric grid: B(u) is even in each coordinate, its four minima
    # (+-5, +-5) tie and lie at equal distance from the incumbent (0, 0),
    # whose own cost is far higher.  The rule (nearest, then the smaller
    # first coordinate, then the smaller second) must pick (-5, -5); a
    # reversed comparison or swapped coordinates pick another corner.
    p = W.w2_problem(21, 41)
    y = W.nodes(p.y_lo, p.y_hi, p.n_y)
    v = 5.0 * np.sign(y)
    u1 = np.stack([np.repeat(v, p.n_y), np.tile(v, p.n_y)])
    i0 = (p.n_x // 2) * p.n_x + p.n_x // 2  # the node x = (0, 0)
    B = [orc.w2_B(p, u1, (0.0, 0.0), (a, b)) for a in (-5.0, 5.0) for b in (-5.0, 5.0)]
    assert max(B) - min(B) <= 1e-13 * min(B)
    for s in (W.Search(-10.0, 10.0, 1, 5), W.Search(-10.0, 10.0, 2, 5)):
        u, _ = orc.w2_argmin(p, s, u1, np.zeros((2, p.n_x ** 2)), [i0])
        assert tuple(u[:, 0]) == (-5.0, -5.0)
    # with the incumbent at a corner, the nearest corner wins instead
    u0 = np.zeros((2, p.n_x ** 2))
    u0[:, i0] = (4.0, -4.0)
    u, _ = orc.w2_argmin(p, W.Search(-10.0, 10.0, 1, 5), u1, u0, [i0])
    assert tuple(u[:, 0]) == (5.0, -5.0)


def test_tie_rule_orders_the_coordinates(orc):
    # u1(y) = 5 sign(y1 - y2) (1, -1) is odd under y -> -y, so B(u) = B(-u)
    # at x = (0, 0); its two minima (-5, 5) and (5, -5) tie at equal
    # distance from the incumbent (0, 0).  The first coordinate decides
    # first: (-5, 5).  Deciding by the second first would give (5, -5).
    p = W.w2_problem(21, 41)
    y = W.nodes(p.y_lo, p.y_hi, p.n_y)
    s = 5.0 * np.sign(np.repeat(y, p.n_y) - np.tile(y, p.n_y))
    u1 = np.stack([s, -s])
    Bm = orc.w2_B(p, u1, (0.0, 0.0), (-5.0, 5.0))
    assert abs(Bm - orc.w2_B(p, u1, (0.0, 0.0), (5.0, -5.0))) <= 1e-13 * Bm
    assert orc.w2_B(p, u1, (0.0, 0.0), (5.0, 5.0)) > 2 * Bm
    i0 = (p.n_x // 2) * p.n_x + p.n_x // 2
    u, _ = orc.w2_argmin(p, W.Search(-10.0, 10.0, 1, 5), u1, np.zeros((2, p.n_x ** 2)), [i0])
    assert tuple(u[:, 0]) == (-5.0, 5.0)


def test_solve_round_order(orc):
    """u0 searched with the previous round's u1, then u1 of the new u0, and
    J_t on that pair (J before the u1 update is larger)."""
    c = W.w2_small_case()
    p, s = c.prob, c.search
    u0_prev, u1_prev = c.u0_init, orc.w2_update_u1(p, c.u0_init)
    for t in (1, 2):
        u0, u1, J = orc.w2_solve(p, s, t, c.u0_init)
        step, _ = orc.w2_argmin(p, s, u1_prev, u0_prev)
        assert np.array_equal(u0, step)
        assert np.array_equal(u1, orc.w2_update_u1(p, u0))
        assert J[t] == orc.w2_objective(p, u0, u1)
        assert J[t] < orc.w2_objective(p, u0, u1_prev) * (1 - 1e-9)
        u0_prev, u1_prev = u0, u1
