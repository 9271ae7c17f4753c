"""GPU parity of the source-channel coding calls (Section V-B) against the
FP64 oracle, on identical seeded inputs.

Tolerances (FP64 on both sides; the GPU takes window sums from
double-double prefix sums, the oracle sums every node in index order):
  - marginal cost and objective: relative 1e-11;
  - decoder u1: 1e-12 absolute (sums of the same terms in two orders);
  - encoder update and solve: decisions equal to the oracle's (the
    relative tie band 1e-12 lies far above the two sides' rounding).
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


def tiny():
    # fewer nodes than one tile; dy = 0.25 exactly, so windows meet nodes at
    # distance exactly 1
    p = W.CodingProblem(2.0, [(1.0, 0.0, 1.0)], -4.0, 4.0, 37, -5.0, 5.0, 41)
    return W.CodingCase("tiny-37x41", p, W.Search(-4.0, 4.0, 2, 5), 3, W.coding_init(p, 3, 4))


def mixture():
    # two decoder segments (2500 x nodes), lam = 0.5, an asymmetric prior
    p = W.CodingProblem(0.5, [(0.3, -1.0, 0.5), (0.7, 1.0, 0.8)], -6.0, 6.0, 2500, -5.5, 5.5, 1500)
    return W.CodingCase("mixture-2500x1500", p, W.Search(-4.5, 4.5, 4, 11), 3, W.coding_init(p, 9, 8))


CASES = {"small": W.coding_small_case, "tiny": tiny, "mixture": mixture}


@pytest.mark.parametrize("name", list(CASES))
def test_marginal_cost(env, name):
    U, orc, torch = env
    c = CASES[name]()
    p = c.prob
    rng = np.random.default_rng(11)
    u1 = rng.uniform(-2.0, 2.0, p.n_y)
    # candidates inside, at the edges of and beyond the y grid
    u = rng.uniform(-7.0, 7.0, (p.n_x, 6))
    u[:, 0] = 0.0
    u[:, 1] = p.y_hi + 1.0  # window holds the last node only
    u[:, 2] = p.y_lo - 1.5  # empty window
    L = host(U.coding_marginal_cost(p, dev(torch, u1), dev(torch, u)))
    ref = orc.coding_marginal_cost(p, u1, u)
    assert np.max(np.abs(L - ref) / np.maximum(np.abs(ref), 1e-300)) < 1e-11


@pytest.mark.parametrize("name", list(CASES))
def test_update_u1_and_objective(env, name):
    U, orc, torch = env
    c = CASES[name]()
    p = c.prob
    u0 = c.u0_init.copy()
    u0[::7] = 6.0   # |y - 6| <= 1 meets only y = 5 (distance 1 on the grid's edge)
    u0[3::11] = 9.0  # reaches no y node
    u1 = host(U.coding_update_u1(p, dev(torch, u0)))
    ref = orc.coding_update_u1(p, u0)
    assert np.max(np.abs(u1 - ref)) < 1e-12
    assert np.array_equal(u1 == 0.0, ref == 0.0)
    J = float(host(U.coding_objective(p, dev(torch, u0), dev(torch, ref)))[0])
    Jr = orc.coding_objective(p, u0, ref)
    assert abs(J - Jr) < 1e-11 * Jr


@pytest.mark.parametrize("name", list(CASES))
def test_argmin(env, name):
    U, orc, torch = env
    c = CASES[name]()
    p = c.prob
    u1 = orc.coding_update_u1(p, c.u0_init)
    out, L0 = U.coding_argmin(p, c.search, dev(torch, u1), dev(torch, c.u0_init), want_l0=True)
    ref, Bref = orc.coding_argmin(p, c.search, u1, c.u0_init)
    assert np.array_equal(host(out), ref)
    f, _ = orc.prior(p)
    Lr = f * Bref
    assert np.max(np.abs(host(L0) - Lr) / np.maximum(np.abs(Lr), 1e-300)) < 1e-11


@pytest.mark.parametrize("name", list(CASES))
def test_solve(env, name):
    U, orc, torch = env
    c = CASES[name]()
    u0, u1, J = U.coding_solve(c.prob, c.search, c.iters, dev(torch, c.u0_init))
    r0, r1, rJ = orc.coding_solve(c.prob, c.search, c.iters, c.u0_init)
    assert np.array_equal(host(u0), r0)
    assert np.max(np.abs(host(u1) - r1)) < 1e-12
    assert np.max(np.abs(host(J) - rJ) / rJ) < 1e-11


def test_solve_in_place_and_repeatable(env):
    U, orc, torch = env
    c = W.coding_small_case()
    P, S = U.make_coding_problem(c.prob), U.make_search(c.search)
    import ctypes as C

    u0 = dev(torch, c.u0_init)
    u1 = torch.empty(c.prob.n_y, dtype=torch.float64, device="cuda")
    J = torch.empty(c.iters + 1, dtype=torch.float64, device="cuda")
    h = U.handle(0)
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    U._check(U.library().ucp_coding_solve(h, C.byref(P), C.byref(S), c.iters, C.c_void_p(u0.data_ptr()),
                                          C.c_void_p(u0.data_ptr()), C.c_void_p(u1.data_ptr()),
                                          C.c_void_p(J.data_ptr()), st))
    a0, a1, aJ = U.coding_solve(c.prob, c.search, c.iters, dev(torch, c.u0_init))
    assert torch.equal(u0, a0) and torch.equal(u1, a1) and torch.equal(J, aJ)


def test_fullsize_sampled(env):
    """The 20001-node workload: one GPU solve of 30 rounds; the final state
    checked against the oracle on sampled rows (encoder update, decoder)
    and in full (objective)."""
    U, orc, torch = env
    c = W.coding_paper_case()
    p = c.prob
    u0, u1, J = U.coding_solve(p, c.search, c.iters, dev(torch, c.u0_init))
    u0h, u1h, Jh = host(u0), host(u1), host(J)
    assert np.all(np.diff(Jh) <= 1e-12 * Jh[:-1]) and Jh[-1] < Jh[0]
    Jr = orc.coding_objective(p, u0h, u1h)
    assert abs(Jh[-1] - Jr) < 1e-11 * Jr
    rows = np.random.default_rng(5).choice(p.n_x, 48, replace=False)
    nxt = host(U.coding_argmin(p, c.search, u1, u0))
    ref, _ = orc.coding_argmin(p, c.search, u1h, u0h, rows)
    assert np.array_equal(nxt[rows], ref)
    yrows = np.random.default_rng(6).choice(p.n_y, 48, replace=False)
    assert np.max(np.abs(u1h[yrows] - orc.coding_update_u1(p, u0h, yrows))) < 1e-12


def test_solve_kernel_timing(env):
    # ucp_profile around a coding solve: one timed search per round, the
    # results unchanged by the timing
    U, orc, torch = env
    c = W.coding_small_case()
    ref = U.coding_solve(c.prob, c.search, c.iters, dev(torch, c.u0_init))
    U.profile(True)
    out = U.coding_solve(c.prob, c.search, c.iters, dev(torch, c.u0_init))
    prof = U.profile_read()
    U.profile(None)
    assert prof["marginal_cost"][1] == c.iters and prof["marginal_cost"][0] > 0.0
    assert prof["u1"][1] == c.iters + 1 and prof["objective"][1] == c.iters + 1
    assert all(torch.equal(a, b) for a, b in zip(ref, out))


@pytest.mark.parametrize("case", ["two-nodes", "lam0-offgrid", "one-level"])
def test_degenerate(env, case):
    """Two-node grids; lam = 0 with every encoder value off the y grid
    (every window empty: u1 = 0 everywhere and B = 0 for all candidates,
    so the tie rule alone decides); a single level of two candidates."""
    U, orc, torch = env
    if case == "two-nodes":
        p = W.CodingProblem(2.0, [(1.0, 0.0, 1.0)], -1.0, 1.0, 2, -2.0, 2.0, 2)
        s, u0 = W.Search(-1.0, 1.0, 2, 3), np.array([0.5, -0.5])
    elif case == "lam0-offgrid":
        p = W.CodingProblem(0.0, [(1.0, 0.0, 1.0)], -3.0, 3.0, 301, -2.0, 2.0, 101)
        s, u0 = W.Search(6.0, 9.0, 3, 5), np.full(301, 7.5)
    else:
        p = W.coding_problem(513, 257)
        s, u0 = W.Search(-3.0, 3.0, 1, 2), W.coding_init(p, 4)
    u0g, u1g, Jg = U.coding_solve(p, s, 2, dev(torch, u0))
    r0, r1, rJ = orc.coding_solve(p, s, 2, u0)
    assert np.array_equal(host(u0g), r0)
    assert np.max(np.abs(host(u1g) - r1)) < 1e-12
    assert np.max(np.abs(host(Jg) - rJ) / np.maximum(rJ, 1e-300)) < 1e-11
    if case == "lam0-offgrid":
        assert np.all(r1 == 0.0) and np.array_equal(r0, u0)  # ties keep the incumbent
