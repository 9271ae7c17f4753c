"""Pins of the FP64 oracle against facts fixed by the paper and by the
mathematics, not by the oracle itself.

Each test names the piece of the oracle it pins and the mistake it would
catch.  The closed forms come from the Witsenhausen problem statement
(Section V-A): x0 ~ N(0, sigma^2), x1 = x0 + u0, y = x1 + w, w ~ N(0, 1).
"""
import math

import mpmath as mp
import numpy as np
import pytest

import workloads as W

K, SIGMA = 0.2, 5.0


def wide(n=2401, half=60.0, k=K, sigma=SIGMA, n_y=None, y_half=None):
    """A grid wide enough (12 sigma) that truncation is below 1e-30."""
    return W.Problem(k=k, comps=[(1.0, 0.0, sigma)], x_lo=-half, x_hi=half, n_x=n,
                     y_lo=-(y_half or half), y_hi=(y_half or half), n_y=n_y or n)


# ---------------------------------------------------------------- grid, prior

def test_grid_is_linspace(orc):
    g = orc.grid(-25.0, 25.0, 1001)
    assert g[0] == -25.0 and abs(g[-1] - 25.0) < 1e-12
    assert np.allclose(np.diff(g), 0.05, rtol=0, atol=1e-13)


def test_prior_density_and_log(orc):
    # single Gaussian: f integrates to 1 and log f matches -x^2/2s^2 - log(s sqrt(2 pi))
    p = wide()
    f, lf = orc.prior(p)
    dx = (p.x_hi - p.x_lo) / (p.n_x - 1)
    assert abs(dx * f.sum() - 1.0) < 1e-12
    x = orc.grid(p.x_lo, p.x_hi, p.n_x)
    ref = -x * x / (2 * SIGMA ** 2) - math.log(SIGMA * math.sqrt(2 * math.pi))
    assert np.max(np.abs(lf - ref)) < 1e-12
    # far tail where f underflows to 0: log f stays exact
    q = W.Problem(k=0.2, comps=[(1.0, 0.0, 1.0)], x_lo=-60, x_hi=60, n_x=121, y_lo=-60, y_hi=60, n_y=121)
    f1, lf1 = orc.prior(q)
    assert f1[0] == 0.0 and abs(lf1[0] - (-1800.0 - 0.5 * math.log(2 * math.pi))) < 1e-9


def test_prior_mixture(orc):
    comps = [(0.2, -7.0, 1.5), (0.5, 2.0, 3.0), (0.3, 9.0, 2.5)]
    p = W.Problem(k=0.2, comps=comps, x_lo=-60, x_hi=60, n_x=4801, y_lo=-60, y_hi=60, n_y=11)
    f, lf = orc.prior(p)
    dx = 120.0 / 4800
    assert abs(dx * f.sum() - 1.0) < 1e-12
    x = orc.grid(-60, 60, 4801)
    # mean of the mixture
    assert abs(dx * (x * f).sum() - sum(w * m for w, m, _ in comps)) < 1e-11
    ok = f > 1e-300
    assert np.max(np.abs(lf[ok] - np.log(f[ok]))) < 1e-12


# --------------------------------------------------- marginal cost (pin P1)

@pytest.mark.parametrize("a", [0.0, 0.5, 1.0, 1.3])
@pytest.mark.parametrize("x,u", [(0.0, 0.0), (3.7, -1.2), (-10.0, 4.5), (12.0, 2.0)])
def test_marginal_cost_linear_u1_closed_form(orc, a, x, u):
    """u1(y) = a y  =>  B(u; x) = k^2 u^2 + (1-a)^2 z^2 + a^2, z = x + u.
    Catches: dropped dy, wrong noise normalisation, sign of (y - z), k vs k^2,
    u1 indexed on the wrong grid (n_x != n_y here)."""
    p = wide(n=801, half=40.0, n_y=1601, y_half=40.0)
    y = orc.grid(p.y_lo, p.y_hi, p.n_y)
    b = orc.B(p, a * y, x, u)
    z = x + u
    ref = K * K * u * u + (1 - a) ** 2 * z * z + a * a
    assert abs(b - ref) <= 1e-12 * ref


def test_marginal_cost_is_f_times_B(orc):
    p = wide(n=401, half=30.0, n_y=601, y_half=30.0)
    y = orc.grid(p.y_lo, p.y_hi, p.n_y)
    x = orc.grid(p.x_lo, p.x_hi, p.n_x)
    f, _ = orc.prior(p)
    a = 0.7
    u = np.stack([np.full(p.n_x, -1.0), np.linspace(-2, 2, p.n_x)], axis=1)
    L0 = orc.marginal_cost(p, a * y, u)
    z = x[:, None] + u
    Bref = K * K * u * u + (1 - a) ** 2 * z * z + a * a
    inner = np.abs(z) < 20
    assert np.max(np.abs(L0[inner] - (f[:, None] * Bref)[inner]) / (f[:, None] * Bref)[inner]) < 1e-12


# ------------------------------------------------------- u1 update (P3, P4, P7)

@pytest.mark.parametrize("lam", [1.0, 0.5, 0.0417424305])
def test_u1_affine_conjugacy(orc, lam):
    """Affine u0 = (lam - 1) x gives x1 = lam x0 ~ N(0, lam^2 sigma^2) and the
    exact conditional mean u1(y) = lam^2 sigma^2 / (1 + lam^2 sigma^2) y.
    Catches: missing prior weight, wrong sign of the logit, wrong noise
    variance."""
    p = wide()
    u0 = W.init_affine(p, lam)
    u1 = orc.update_u1(p, u0)
    y = orc.grid(p.y_lo, p.y_hi, p.n_y)
    g = lam * lam * SIGMA ** 2 / (1 + lam * lam * SIGMA ** 2)
    sy = math.sqrt(lam * lam * SIGMA ** 2 + 1)
    inner = np.abs(y) <= 4 * sy
    assert np.max(np.abs(u1[inner] - g * y[inner])) < 1e-10


def test_u1_three_level_exact(orc):
    """u0 = sigma sign(x) - x puts x1 on {-sigma, 0, +sigma}; the discrete
    conditional mean is then sigma (P+ e^{-(y-s)^2/2} - P- e^{-(y+s)^2/2}) /
    (P+ e^{-(y-s)^2/2} + P- e^{-(y+s)^2/2} + P0 e^{-y^2/2}) with P+- the prior
    mass on each side and P0 = f(0).  Also covers |y| = 25 where the raw
    weights are ~e^{-450}.  Computed here by grouping, at 40 digits."""
    c = W.small_case()
    p = c.prob
    u1 = orc.update_u1(p, c.u0_init)
    f, _ = orc.prior(p)
    x = orc.grid(p.x_lo, p.x_hi, p.n_x)
    y = orc.grid(p.y_lo, p.y_hi, p.n_y)
    with mp.workdps(40):
        Pp = mp.fsum(mp.mpf(v) for v in f[x > 0])
        Pm = mp.fsum(mp.mpf(v) for v in f[x < 0])
        P0 = mp.mpf(f[x == 0][0])
        s = mp.mpf(SIGMA)
        worst = 0.0
        for j in range(0, p.n_y, 7):
            yy = mp.mpf(y[j])
            ep = Pp * mp.e ** (-(yy - s) ** 2 / 2)
            em = Pm * mp.e ** (-(yy + s) ** 2 / 2)
            e0 = P0 * mp.e ** (-yy ** 2 / 2)
            ref = s * (ep - em) / (ep + em + e0)
            worst = max(worst, abs(float(ref) - u1[j]))
    assert worst < 1e-13


def test_u1_stationarity(orc):
    """u1_j minimises sum_i f_i phi(y_j - x1_i)(x1_i - v)^2 over v, so the
    weighted residual vanishes (discrete first-order condition)."""
    c = W.small_case()
    p = c.prob
    u0 = W.init_random_steps(p, 5.0, 3)
    u1 = orc.update_u1(p, u0)
    f, _ = orc.prior(p)
    x1 = orc.grid(p.x_lo, p.x_hi, p.n_x) + u0
    y = orc.grid(p.y_lo, p.y_hi, p.n_y)
    for j in range(0, p.n_y, 50):
        w = f * np.exp(-0.5 * (y[j] - x1) ** 2)
        res = np.sum(w * (x1 - u1[j]))
        scale = np.sum(w * np.abs(x1)) + 1e-300
        assert abs(res) <= 1e-13 * scale


# ------------------------------------------------------------ objective (P5, P6)

def affine_cost(k, sigma, lam):
    return k * k * (lam - 1) ** 2 * sigma ** 2 + lam * lam * sigma ** 2 / (1 + lam * lam * sigma ** 2)


@pytest.mark.parametrize("lam,expect", [
    (1.0, 25.0 / 26.0), (0.0, 1.0), (0.0417424305044, 0.96), (0.958257569496, 0.96),
    (0.3031960455, 1.1823397054),
])
def test_objective_affine_closed_form(orc, lam, expect):
    """J of an affine u0 with its linear MMSE u1:
    k^2 (lam-1)^2 sigma^2 + lam^2 sigma^2 / (1 + lam^2 sigma^2); at k=0.2,
    sigma=5 both stationary minima give exactly 0.96.  Checked once with the
    closed-form u1 (objective alone) and once with the oracle's own u1."""
    assert abs(affine_cost(K, SIGMA, lam) - expect) < 1e-9
    p = wide()
    u0 = W.init_affine(p, lam)
    y = orc.grid(p.y_lo, p.y_hi, p.n_y)
    g = lam * lam * SIGMA ** 2 / (1 + lam * lam * SIGMA ** 2)
    J1 = orc.objective(p, u0, g * y)
    J2 = orc.objective(p, u0, orc.update_u1(p, u0))
    ref = affine_cost(K, SIGMA, lam)
    assert abs(J1 - ref) <= 1e-10 * ref
    assert abs(J2 - ref) <= 1e-10 * ref


def test_objective_equals_sum_of_marginal_costs(orc):
    """J = dx * sum_i L_0(u0_i; x_i) for the same u1 (the decomposition of
    Eq. (1) for the first controller)."""
    c = W.small_case()
    p = c.prob
    u0 = W.init_random_steps(p, 5.0, 1)
    u1 = orc.update_u1(p, u0)
    L0 = orc.marginal_cost(p, u1, u0[:, None])[:, 0]
    dx = (p.x_hi - p.x_lo) / (p.n_x - 1)
    J = orc.objective(p, u0, u1)
    assert abs(J - dx * L0.sum()) <= 1e-13 * J


def test_init_cost_sanity(orc):
    """Continuum cost of u0 = sigma sign(x) - x at k=0.2, sigma=5 is
    2 k^2 sigma^2 (1 - sqrt(2/pi)) + (two-point MMSE) = 0.40425; the
    1001-node grid adds the x0 = 0 node (x1 = 0), a few percent."""
    stage1 = 2 * K * K * SIGMA ** 2 * (1 - math.sqrt(2 / math.pi))
    assert abs(stage1 - 0.404230878394) < 1e-11
    c = W.small_case()
    u1 = orc.update_u1(c.prob, c.u0_init)
    J = orc.objective(c.prob, c.u0_init, u1)
    assert 0.404 < J < 0.404 * 1.05


# ---------------------------------------------------- refinement argmin (P2)

def test_argmin_convex_closed_form(orc):
    """With u1 = a y, B is the convex quadratic k^2 u^2 + (1-a)^2 (x+u)^2 + a^2
    with minimiser u* = -(1-a)^2 x / (k^2 + (1-a)^2).  The coarse-to-fine
    search must land within the last spacing of u*.  Catches wrong bracket
    widths, wrong spacing recursion, a lost best-so-far."""
    p = wide(n=201, half=20.0, n_y=1601, y_half=40.0)
    s = W.Search(-30.0, 30.0, 4, 16)
    h = orc.spacings(s)
    assert np.allclose(h, [4.0, 8.0 / 15, 16.0 / 225, 32.0 / 3375], rtol=1e-15)
    y = orc.grid(p.y_lo, p.y_hi, p.n_y)
    x = orc.grid(p.x_lo, p.x_hi, p.n_x)
    for a in (0.3, 0.8):
        u0o, Bo = orc.argmin(p, s, a * y, np.full(p.n_x, 29.0))
        ustar = -(1 - a) ** 2 * x / (K * K + (1 - a) ** 2)
        assert np.max(np.abs(u0o - ustar)) <= h[-1]
        Bref = K * K * u0o ** 2 + (1 - a) ** 2 * (x + u0o) ** 2 + a * a
        assert np.max(np.abs(Bo - Bref) / Bref) < 1e-12


def test_argmin_never_worse_than_coarse_grid_or_incumbent(orc):
    """Against exhaustive evaluation on a tiny instance: the result is no
    worse than every level-0 candidate and than the incumbent (the best so
    far and the incumbent are always in the final set)."""
    p = W.gaussian_problem(0.2, 5.0, 41, 25.0)
    s = W.Search(-30.0, 30.0, 3, 9)
    rng = np.random.default_rng(0)
    u0 = W.init_random_steps(p, 5.0, 2)
    u1 = orc.update_u1(p, u0)
    u0o, Bo = orc.argmin(p, s, u1, u0)
    x = orc.grid(p.x_lo, p.x_hi, p.n_x)
    lvl0 = -30.0 + np.arange(9) * 7.5
    for i in range(p.n_x):
        b0 = min(orc.B(p, u1, x[i], c) for c in lvl0)
        binc = orc.B(p, u1, x[i], u0[i])
        assert Bo[i] <= min(b0, binc) * (1 + 1e-12)
    # exhaustive search on a fine grid: report how close the refinement gets
    fine = np.linspace(-30, 30, 2401)
    gaps = []
    for i in rng.choice(p.n_x, 10, replace=False):
        bex = min(orc.B(p, u1, x[i], c) for c in fine)
        gaps.append((Bo[i] - bex) / bex)
    assert min(gaps) > -1e-3  # the fine grid is denser than the last level


def test_argmin_tie_rule(orc):
    """At x0 = 0 with a symmetric problem and an odd u1, B(u) = B(-u): the two
    mirror minima tie exactly; the rule takes the one nearer the incumbent,
    and the smaller u when the incumbent is equidistant."""
    p = W.gaussian_problem(0.2, 5.0, 201, 25.0)
    s = W.Search(-30.0, 30.0, 3, 21)
    y = orc.grid(p.y_lo, p.y_hi, p.n_y)
    u1 = 5.0 * np.tanh(5.0 * y)
    mid = p.n_x // 2
    for inc, sign in ((0.0, -1), (1.0, +1), (-1.0, -1)):
        u0 = np.full(p.n_x, inc)
        out, _ = orc.argmin(p, s, u1, u0, rows=[mid])
        assert np.sign(out[0]) == sign and abs(abs(out[0]) - 5.0) < 0.5


def test_argmin_fixed_point_and_rows(orc):
    """Feeding the result back with the same u1 changes nothing (incumbent
    kept on ties), and a row subset reproduces the full update exactly."""
    c = W.small_case()
    p, s = c.prob, c.search
    u1 = orc.update_u1(p, c.u0_init)
    a, Ba = orc.argmin(p, s, u1, c.u0_init)
    b, Bb = orc.argmin(p, s, u1, a)
    assert np.array_equal(a, b)
    rows = np.array([0, 5, 500, 777, 1000])
    r, Br = orc.argmin(p, s, u1, c.u0_init, rows=rows)
    assert np.array_equal(r, a[rows]) and np.array_equal(Br, Ba[rows])
    ur = orc.update_u1(p, a, rows=rows)
    assert np.array_equal(ur, orc.update_u1(p, a)[rows])


def test_argmin_clamps_to_range(orc):
    """When u* lies beyond u_hi the search ends on the bound."""
    p = wide(n=101, half=10.0, n_y=1601, y_half=40.0)
    s = W.Search(-2.0, 2.0, 3, 11)
    y = orc.grid(p.y_lo, p.y_hi, p.n_y)
    # a = 0: u* = -x / (k^2 + 1): beyond [-2, 2] for |x| > 2.08
    out, _ = orc.argmin(p, s, 0.0 * y, np.zeros(p.n_x))
    x = orc.grid(p.x_lo, p.x_hi, p.n_x)
    assert np.all(out[x > 5] == -2.0) and np.all(out[x < -5] == 2.0)


# --------------------------------------------------------- the solve (P8, P10)

def test_solve_monotone_and_resumable(orc):
    c = W.small_case()
    u0, u1, J = orc.solve(c.prob, c.search, 4, c.u0_init)
    assert np.all(J[1:] <= J[:-1] * (1 + 1e-12))
    assert J[-1] < J[0] - 0.01
    a0, a1, Ja = orc.solve(c.prob, c.search, 2, c.u0_init)
    b0, b1, Jb = orc.solve(c.prob, c.search, 2, a0)
    assert np.array_equal(b0, u0) and np.array_equal(b1, u1) and np.array_equal(Jb[1:], J[3:])


def test_symmetry(orc):
    """Symmetric prior and grids: an odd u0 gives an odd u1, and for any u0 the
    mirrored controller x -> -u0(-x) has the mirrored u1 and the same J."""
    p = W.gaussian_problem(0.2, 5.0, 1001, 25.0)
    g = W.init_random_steps(p, 5.0, 4)
    odd = 0.5 * (g - g[::-1])
    u1 = orc.update_u1(p, odd)
    assert np.max(np.abs(u1 + u1[::-1])) < 1e-12
    w1 = orc.update_u1(p, g)
    J = orc.objective(p, g, w1)
    v0 = -g[::-1].copy()
    v1 = orc.update_u1(p, v0)
    assert np.max(np.abs(v1 + w1[::-1])) < 1e-12
    assert abs(orc.objective(p, v0, v1) - J) <= 1e-13 * J


# ------------------------------------------- 40-digit brute force (P9)

def test_against_mpmath_tiny(orc):
    """The whole oracle (u1 update, objective, refinement decisions) against an
    independent 40-digit evaluation of the same discrete problem."""
    from oracle import mp_oracle

    p = W.Problem(k=0.2, comps=[(0.6, -3.0, 2.0), (0.4, 4.0, 3.0)], x_lo=-12, x_hi=12, n_x=25,
                  y_lo=-15, y_hi=15, n_y=31)
    s = W.Search(-8.0, 8.0, 3, 7)
    u0 = W.init_random_steps(p, 4.0, 5)
    u1 = orc.update_u1(p, u0)
    u1m = mp_oracle.u1_update(p, u0)
    assert max(abs(float(a) - b) for a, b in zip(u1m, u1)) < 1e-13
    J = orc.objective(p, u0, u1)
    Jm = mp_oracle.objective(p, u0, u1)
    assert abs(float(Jm) - J) <= 1e-13 * J
    a, _ = orc.argmin(p, s, u1, u0)
    am = mp_oracle.argmin(p, s, u1, u0)
    assert np.array_equal(a, np.array(am))


# ------------------------------------------ order within a round (Q7 reading)

def test_solve_round_order(orc):
    """Each round updates u0 with the u1 of the previous round, then replaces
    u1 by the closed form of the new u0, and J_t is taken on that pair.
    Catches J taken before the u1 update (J(u0_t, u1_{t-1}) is strictly
    larger: the update is the exact minimiser over u1) and a round that
    updates u1 before searching u0."""
    c = W.small_case()
    p, s = c.prob, c.search
    u0_prev, u1_prev = c.u0_init, orc.update_u1(p, c.u0_init)
    for t in (1, 2, 3):
        u0, u1, J = orc.solve(p, s, t, c.u0_init)
        step, _ = orc.argmin(p, s, u1_prev, u0_prev)
        assert np.array_equal(u0, step)
        assert np.array_equal(u1, orc.update_u1(p, u0))
        assert J[t] == orc.objective(p, u0, u1)
        before = orc.objective(p, u0, u1_prev)
        assert J[t] < before * (1 - 1e-9), (t, J[t], before)
        u0_prev, u1_prev = u0, u1


def test_against_mpmath_two_round_solve(orc):
    """Two whole rounds of the oracle's solve loop against the same loop run
    at 40 digits from the definitions (P9): J_hist to 1e-13, u0 equal."""
    from oracle import mp_oracle

    p = W.Problem(k=0.2, comps=[(0.6, -3.0, 2.0), (0.4, 4.0, 3.0)], x_lo=-12, x_hi=12, n_x=25,
                  y_lo=-15, y_hi=15, n_y=31)
    s = W.Search(-8.0, 8.0, 3, 7)
    u0i = W.init_random_steps(p, 4.0, 5)
    u0, u1, J = orc.solve(p, s, 2, u0i)
    m0, m1, Jm = mp_oracle.solve(p, s, 2, u0i)
    assert np.array_equal(u0, np.array(m0))
    assert max(abs(float(a) - b) for a, b in zip(m1, u1)) < 1e-13
    for a, b in zip(Jm, J):
        assert abs(float(a) - b) <= 1e-13 * b
    assert float(Jm[2]) < float(Jm[0])


def test_argmin_tie_band_parameter(orc):
    """The selection rule's relative tie band comes from the search record.
    With u1 = a y, B(u; 0) = (k^2 + (1-a)^2) u^2 + a^2 in closed form, so an
    incumbent at u = d costs a relative delta = (k^2 + (1-a)^2) d^2 / a^2
    more than the minimum u = 0 (a level-0 node).  A band wider than delta
    keeps the incumbent; the default band or one narrower than delta moves
    the point to 0.  Catches a band that ignores the parameter, and one
    applied to the absolute instead of the relative gap."""
    p = wide(n=101, half=10.0, n_y=1601, y_half=40.0)
    y = orc.grid(p.y_lo, p.y_hi, p.n_y)
    a, d = 0.5, 0.01
    delta = (K * K + (1 - a) ** 2) * d * d / (a * a)
    mid = p.n_x // 2
    u0 = np.full(p.n_x, d)
    for tau, expect in ((0.0, 0.0), (0.5 * delta, 0.0), (2.0 * delta, d)):
        s = W.Search(-2.0, 2.0, 1, 11, tie_rel64=tau)
        out, B = orc.argmin(p, s, a * y, u0, rows=[mid])
        assert out[0] == expect, (tau, out[0])
        assert abs(B[0] - (K * K + (1 - a) ** 2) * expect ** 2 - a * a) < 1e-12


# ------------------------------------------------ noise standard deviation

@pytest.mark.parametrize("sw", [0.5, 2.0])
def test_noise_sd_closed_forms(orc, sw):
    """w ~ N(0, sw^2).  With u1 = a y, B(u; x) = k^2 u^2 + (1-a)^2 z^2 + a^2 sw^2
    (z = x + u); affine u0 = (lam - 1) x gives u1 = lam^2 s^2 / (lam^2 s^2 + sw^2) y
    and J = k^2 (lam - 1)^2 s^2 + lam^2 s^2 sw^2 / (lam^2 s^2 + sw^2).  Catches
    a missing 1/sw in the density, the noise variance left at 1 in the
    exponent of the u1 weights, and sw in place of sw^2."""
    p = wide(n=4801, half=60.0)
    p.noise_sd = sw
    y = orc.grid(p.y_lo, p.y_hi, p.n_y)
    for a, x, u in ((0.3, 1.7, -0.4), (0.8, -3.0, 2.5)):
        z = x + u
        ref = K * K * u * u + (1 - a) ** 2 * z * z + a * a * sw * sw
        assert abs(orc.B(p, a * y, x, u) - ref) <= 1e-12 * ref
    for lam in (0.3, 1.0):
        u0 = W.init_affine(p, lam)
        u1 = orc.update_u1(p, u0)
        g = lam ** 2 * SIGMA ** 2 / (lam ** 2 * SIGMA ** 2 + sw * sw)
        inner = np.abs(y) < 12  # x1 spans [-18, 18] at lam = 0.3: stay clear of its ends
        assert np.max(np.abs(u1[inner] - g * y[inner])) < 1e-9
        J = orc.objective(p, u0, g * y)
        ref = K * K * (lam - 1) ** 2 * SIGMA ** 2 + lam ** 2 * SIGMA ** 2 * sw * sw / (lam ** 2 * SIGMA ** 2 + sw * sw)
        assert abs(J - ref) <= 1e-10 * ref


def test_noise_sd_scaling_is_exact(orc):
    """Doubling every length (grids, prior, search range) and the noise sd
    scales the discrete problem exactly: positions double, B and J
    quadruple, in binary64.  Two whole rounds of the solve loop must show it
    bit for bit."""
    c = W.small_case()
    p1, s1 = c.prob, c.search
    p2 = W.Problem(k=p1.k, comps=[(1.0, 0.0, 10.0)], x_lo=-50.0, x_hi=50.0, n_x=p1.n_x, y_lo=-50.0, y_hi=50.0,
                   n_y=p1.n_y, noise_sd=2.0)
    s2 = W.Search(2 * s1.u_lo, 2 * s1.u_hi, s1.levels, s1.cands)
    a0, a1, Ja = orc.solve(p1, s1, 2, c.u0_init)
    b0, b1, Jb = orc.solve(p2, s2, 2, 2.0 * c.u0_init)
    assert np.array_equal(b0, 2.0 * a0)
    assert np.max(np.abs(b1 - 2.0 * a1)) <= 1e-13 * np.max(np.abs(b1))
    assert np.max(np.abs(Jb - 4.0 * Ja) / Jb) <= 1e-14
