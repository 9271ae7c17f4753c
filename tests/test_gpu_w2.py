"""GPU parity of the two-dimensional Witsenhausen calls (Section V-D)
against the FP64 oracle, on identical seeded inputs.

Tolerances: both sides FP64; the GPU's search sums the noise over a window
of floor(10 / dy) nodes either side of the nearest node per coordinate
(the explicit-candidate and objective sums with a per-row recurrence for
the Gaussian, relative error ~1e-14), the oracle densely with exp:
  - marginal cost and objective: relative 1e-11;
  - u1: 1e-10 absolute (segmented max-shifted sums against one pass);
  - search and solve: decisions equal to the oracle's.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_04489_amd as U

    import oracle

    oracle.lib()
    return U, oracle, torch


def dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def ragged():
    # 19 x-nodes and 23 y-nodes per coordinate on different ranges, a
    # two-component prior, 4 x 4 candidates on 3 levels
    p = W.Problem(0.3, [(0.6, -2.0, 3.0), (0.4, 4.0, 2.0)], -16.0, 18.0, 19, -20.0, 22.0, 23)
    return W.W2Case("w2-ragged", p, W.Search(-12.0, 14.0, 3, 4), 2, W.w2_init(W.w2_problem(19), 2))


CASES = {"small": W.w2_small_case, "ragged": ragged}


@pytest.mark.parametrize("name", list(CASES))
def test_marginal_cost(env, name):
    U, orc, torch = env
    c = CASES[name]()
    p = c.prob
    rng = np.random.default_rng(3)
    u1 = rng.uniform(-10, 10, (2, p.n_y ** 2))
    u = rng.uniform(-30, 30, (2, p.n_x ** 2, 3))
    L = host(U.w2_marginal_cost(p, dev(torch, u1), dev(torch, u)))
    ref = orc.w2_marginal_cost(p, u1, u)
    assert np.max(np.abs(L - ref) / np.maximum(np.abs(ref), 1e-300)) < 1e-11


@pytest.mark.parametrize("name", list(CASES))
def test_u1_and_objective(env, name):
    U, orc, torch = env
    c = CASES[name]()
    p = c.prob
    u1 = host(U.w2_update_u1(p, dev(torch, c.u0_init)))
    ref = orc.w2_update_u1(p, c.u0_init)
    assert np.max(np.abs(u1 - ref)) < 1e-10
    J = float(host(U.w2_objective(p, dev(torch, c.u0_init), dev(torch, ref)))[0])
    Jr = orc.w2_objective(p, c.u0_init, ref)
    assert abs(J - Jr) < 1e-11 * Jr


@pytest.mark.parametrize("name", list(CASES))
def test_argmin(env, name):
    U, orc, torch = env
    c = CASES[name]()
    p = c.prob
    u1 = orc.w2_update_u1(p, c.u0_init)
    out, L0 = U.w2_argmin(p, c.search, dev(torch, u1), dev(torch, c.u0_init), want_l0=True)
    ref, Bref = orc.w2_argmin(p, c.search, u1, c.u0_init)
    assert np.array_equal(host(out), ref)
    f, _ = orc.prior(p)
    Lr = np.outer(f, f).ravel() * Bref
    assert np.max(np.abs(host(L0) - Lr) / np.maximum(np.abs(Lr), 1e-300)) < 1e-11


@pytest.mark.parametrize("name", list(CASES))
def test_solve(env, name):
    U, orc, torch = env
    c = CASES[name]()
    u0, u1, J = U.w2_solve(c.prob, c.search, c.iters, dev(torch, c.u0_init))
    r0, r1, rJ = orc.w2_solve(c.prob, c.search, c.iters, c.u0_init)
    assert np.array_equal(host(u0), r0)
    assert np.max(np.abs(host(u1) - r1)) < 1e-10
    assert np.max(np.abs(host(J) - rJ) / rJ) < 1e-11


def test_paper_size_sampled(env):
    """160 x 160 nodes, 4 levels x 8 x 8 candidates, 2 rounds on the GPU;
    sampled points of a further update against the oracle."""
    U, orc, torch = env
    c = W.w2_paper_case(iters=2)
    p = c.prob
    u0, u1, J = U.w2_solve(p, c.search, c.iters, dev(torch, c.u0_init))
    Jh = host(J)
    assert np.all(np.diff(Jh) <= 1e-12 * Jh[:-1])
    rows = np.random.default_rng(8).choice(p.n_x ** 2, 24, replace=False)
    nxt = host(U.w2_argmin(p, c.search, u1, u0))
    ref, _ = orc.w2_argmin(p, c.search, host(u1), host(u0), rows)
    assert np.array_equal(nxt[:, rows], ref)
    yrows = np.random.default_rng(9).choice(p.n_y ** 2, 24, replace=False)
    assert np.max(np.abs(host(u1)[:, yrows] - orc.w2_update_u1(p, host(u0), yrows))) < 1e-10


def test_solve_kernel_timing(env):
    U, orc, torch = env
    c = W.w2_small_case()
    ref = U.w2_solve(c.prob, c.search, c.iters, dev(torch, c.u0_init))
    U.profile(["marginal_cost"])
    out = U.w2_solve(c.prob, c.search, c.iters, dev(torch, c.u0_init))
    prof = U.profile_read()
    U.profile(None)
    assert prof["marginal_cost"][1] == c.iters and prof["u1"][1] == 0
    assert all(torch.equal(a, b) for a, b in zip(ref, out))


@pytest.mark.parametrize("case", ["two-nodes", "k0", "one-level"])
def test_degenerate(env, case):
    """2 x 2 grids; k = 0; a single level of 2 x 2 candidates."""
    U, orc, torch = env
    if case == "two-nodes":
        p = W.Problem(0.2, [(1.0, 0.0, 5.0)], -5.0, 5.0, 2, -8.0, 8.0, 2)
        s, u0 = W.Search(-6.0, 6.0, 2, 3), np.array([[1.0, -1.0, 2.0, 0.0], [0.0, 3.0, -2.0, 1.0]])
    elif case == "k0":
        p = W.w2_problem(15, 21, k=0.0)
        s, u0 = W.Search(-30.0, 30.0, 2, 4), W.w2_init(p, 6)
    else:
        p = W.w2_problem(17, 19)
        s, u0 = W.Search(-20.0, 20.0, 1, 2), W.w2_init(p, 7)
    u0g, u1g, Jg = U.w2_solve(p, s, 2, dev(torch, u0))
    r0, r1, rJ = orc.w2_solve(p, s, 2, u0)
    assert np.array_equal(host(u0g), r0)
    assert np.max(np.abs(host(u1g) - r1)) < 1e-10
    assert np.max(np.abs(host(Jg) - rJ) / np.maximum(rJ, 1e-300)) < 1e-11
