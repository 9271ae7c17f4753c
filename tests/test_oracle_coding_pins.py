"""Pins of the oracle's source-channel coding functions (Section V-B:
x0 ~ N(0, 1), x1 = u0(x0) + w, w ~ U(-1, 1), J = E[lam u0^2 + (u1(x1) - x0)^2])
against closed forms and exact discrete identities that do not come from
the oracle itself.
"""
import math

import numpy as np
import pytest

import workloads as W


def prob(n_x=1600, n_y=4001, lam=2.0, comps=((1.0, 0.0, 1.0),), x=8.0, y=5.0):
    return W.CodingProblem(lam=lam, comps=list(comps), x_lo=-x, x_hi=x, n_x=n_x, y_lo=-y, y_hi=y, n_y=n_y)


def test_zero_encoder_closed_form(orc):
    # u0 = 0: x1 = w carries no information, so u1 = E[x0] on the noise's
    # support and J = Var(x0) = 1 (continuum); on the grid exactly
    # dx (dy/2) N1 sum_i f_i (x_i - m)^2 with N1 = #{j: |y_j| <= 1}.
    # Catches: a dropped 1/2 of the density, a wrong window, a wrong mean.
    p = prob()
    x = W.nodes(p.x_lo, p.x_hi, p.n_x)
    y = W.nodes(p.y_lo, p.y_hi, p.n_y)
    f, _ = orc.prior(p)
    dx = (p.x_hi - p.x_lo) / (p.n_x - 1)
    dy = (p.y_hi - p.y_lo) / (p.n_y - 1)
    u0 = np.zeros(p.n_x)
    u1 = orc.coding_update_u1(p, u0)
    m = (f * x).sum() / f.sum()
    inside = np.abs(y) <= 1.0
    assert np.max(np.abs(u1[inside] - m)) < 1e-15 and np.all(u1[~inside] == 0.0)
    J = orc.coding_objective(p, u0, u1)
    exact = dx * (dy / 2) * inside.sum() * (f * (x - m) ** 2).sum()
    assert abs(J - exact) < 1e-13
    assert abs(J - 1.0) < dy  # window holds 2/dy + 1 nodes


@pytest.mark.parametrize("c", [1.25, 2.0])
def test_one_bit_encoder_closed_form(orc, c):
    # u0 = c sign(x0) with c > 1: the two noise windows are disjoint, so the
    # decoder is E[x0 | x0 > 0] = sqrt(2/pi) on (c-1, c+1) and
    # J = lam c^2 + 1 - 2/pi.  Catches: sign errors, x vs x1 in the decoder.
    p = prob(n_x=3200, n_y=8001)
    x = W.nodes(p.x_lo, p.x_hi, p.n_x)  # even n_x: no node at 0
    y = W.nodes(p.y_lo, p.y_hi, p.n_y)
    u0 = c * np.sign(x)
    u1 = orc.coding_update_u1(p, u0)
    pos = (y > c - 1 + 1e-9) & (y < c + 1 - 1e-9)
    assert np.max(np.abs(u1[pos] - math.sqrt(2 / math.pi))) < 1e-5
    neg = (y < -c + 1 - 1e-9) & (y > -c - 1 + 1e-9)
    assert np.max(np.abs(u1[neg] + math.sqrt(2 / math.pi))) < 1e-5
    J = orc.coding_objective(p, u0, u1)
    assert abs(J - (p.lam * c * c + 1 - 2 / math.pi)) < 3e-3


def test_one_bit_overlap_is_symmetric(orc):
    # c < 1: on |y| <= 1 - c both windows cover y, the posterior is the
    # symmetric prior, and the decoder is 0.
    p = prob(n_x=3200, n_y=8001)
    x = W.nodes(p.x_lo, p.x_hi, p.n_x)
    y = W.nodes(p.y_lo, p.y_hi, p.n_y)
    u1 = orc.coding_update_u1(p, 0.5 * np.sign(x))
    mid = np.abs(y) < 0.5 - 1e-9
    assert np.max(np.abs(u1[mid])) < 1e-13


def test_window_holds_its_end_points(orc):
    # dy = 0.25 (exact): for u = 0.5 the nodes -0.5 .. 1.5 are within
    # |y - u| <= 1, the end points exactly at distance 1 included: 9 nodes.
    # With u1 = a constant: B = lam u^2 + dy * 0.5 * 9 * (a - x)^2.
    p = prob(n_x=11, n_y=41)  # y nodes -5 .. 5 step 0.25
    u1 = np.full(p.n_y, 0.75)
    B = orc.coding_B(p, u1, 0.3, 0.5)
    assert abs(B - (p.lam * 0.25 + 0.25 * (0.5 * 9 * (0.75 - 0.3) ** 2))) < 1e-14  # 7 nodes: 0.05 less


@pytest.mark.parametrize("x,u", [(0.0, 0.0), (1.0, 0.4), (-2.0, -1.0), (0.5, 2.5)])
def test_B_with_linear_decoder(orc, x, u):
    # u1(y) = y: B = lam u^2 + E[(u + w - x)^2] = lam u^2 + (u - x)^2 + 1/3.
    p = prob(n_y=20001)
    y = W.nodes(p.y_lo, p.y_hi, p.n_y)
    dy = (p.y_hi - p.y_lo) / (p.n_y - 1)
    B = orc.coding_B(p, y, x, u)
    assert abs(B - (p.lam * u * u + (u - x) ** 2 + 1 / 3)) < 3 * dy * (1 + (u - x) ** 2)


def test_argmin_with_linear_decoder(orc):
    # the same B is minimised at u = x / (1 + lam)
    p = prob(n_x=161, n_y=20001)
    y = W.nodes(p.y_lo, p.y_hi, p.n_y)
    x = W.nodes(p.x_lo, p.x_hi, p.n_x)
    s = W.Search(-4.0, 4.0, 4, 17)
    u0, _ = orc.coding_argmin(p, s, y, np.zeros(p.n_x))
    inner = np.abs(x) < 3.0
    assert np.max(np.abs(u0[inner] - x[inner] / (1 + p.lam))) < 0.02


def test_objective_is_dx_sum_f_B(orc):
    # J(u0, u1) = dx sum_i L_0(u0_i, x_i): objective and marginal cost agree
    p = prob(n_x=400, n_y=1201)
    rng = np.random.default_rng(3)
    u0 = W.coding_init(p, 5)
    u1 = rng.uniform(-2, 2, p.n_y)
    L = orc.coding_marginal_cost(p, u1, u0[:, None])[:, 0]
    dx = (p.x_hi - p.x_lo) / (p.n_x - 1)
    J = orc.coding_objective(p, u0, u1)
    assert abs(J - dx * L.sum()) < 1e-13 * max(1.0, J)


def test_u1_minimises_J(orc):
    # the closed form is the minimiser of J over u1: any perturbation of one
    # decoder value with mass under it raises J
    p = prob(n_x=400, n_y=801)
    u0 = W.coding_init(p, 2)
    u1 = orc.coding_update_u1(p, u0)
    J0 = orc.coding_objective(p, u0, u1)
    rng = np.random.default_rng(4)
    y = W.nodes(p.y_lo, p.y_hi, p.n_y)
    live = np.flatnonzero(np.min(np.abs(y[:, None] - u0[None, :]), axis=1) <= 1.0)
    for j in rng.choice(live, 8, replace=False):
        for eps in (1e-3, -1e-3):
            v = u1.copy()
            v[j] += eps
            assert orc.coding_objective(p, u0, v) > J0


def test_rows_and_solve_monotone(orc):
    c = W.coding_small_case()
    u0, u1, J = orc.coding_solve(c.prob, c.search, c.iters, c.u0_init)
    assert np.all(np.diff(J) <= 1e-12 * J[:-1])
    assert J[-1] < J[0]
    # a listed-rows update equals the full one on those rows
    rows = np.array([0, 5, 400, 800])
    full, _ = orc.coding_argmin(c.prob, c.search, u1, u0)
    part, _ = orc.coding_argmin(c.prob, c.search, u1, u0, rows)
    assert np.array_equal(full[rows], part)
    ufull = orc.coding_update_u1(c.prob, u0)
    assert np.array_equal(ufull[[1, 600, 1200]], orc.coding_update_u1(c.prob, u0, [1, 600, 1200]))


def test_solve_round_order(orc):
    """u0 searched with the previous round's decoder, then the decoder of the
    new u0, and J_t on that pair (J before the decoder update is larger)."""
    c = W.coding_small_case()
    p, s = c.prob, c.search
    u0_prev, u1_prev = c.u0_init, orc.coding_update_u1(p, c.u0_init)
    for t in (1, 2):
        u0, u1, J = orc.coding_solve(p, s, t, c.u0_init)
        step, _ = orc.coding_argmin(p, s, u1_prev, u0_prev)
        assert np.array_equal(u0, step)
        assert np.array_equal(u1, orc.coding_update_u1(p, u0))
        assert J[t] == orc.coding_objective(p, u0, u1)
        assert J[t] < orc.coding_objective(p, u0, u1_prev) * (1 - 1e-9)
        u0_prev, u1_prev = u0, u1
