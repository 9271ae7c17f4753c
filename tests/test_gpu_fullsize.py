"""Parity at full benchmark sizes, on sampled outputs the oracle computes row
by row (rows of one update are independent of each other, so the oracle on
a sample checks those rows exactly).

  - 20001-node grids, 5 x 16 search (the benchmark workload, in the launch
    configuration the benchmark times): after a few GPU rounds, one GPU u0
    update and one GPU u1 update from that state are compared with the
    oracle on sampled rows given the same inputs; the FP64 objective of the
    state is compared in full.
  - 65536-node grids with a 3-component mixture prior, 4 x 32 search (the
    largest single-instance size of the batched workload), four instances
    in one batched launch: 259 sampled u0 rows each (the update given the
    GPU's u1), 259 sampled u1 rows (FP32 and FP64 arithmetic) and J.
"""
import numpy as np
import pytest

import workloads as W
from tolerances import near_tie

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


def _check_rows(orc, p, s, u1, u0, got, rows):
    ref, Bref = orc.argmin(p, s, u1, u0, rows=rows)
    x = orc.grid(p.x_lo, p.x_hi, p.n_x)
    diff = [r for r in range(len(rows)) if got[rows[r]] != ref[r]]
    for r in diff:  # only FP64 near-ties may differ
        bg = orc.B(p, u1, x[rows[r]], got[rows[r]])
        assert bg <= Bref[r] * (1 + near_tie()), (rows[r], got[rows[r]], ref[r], bg, Bref[r])
    return len(diff)


def test_paper_resolution_sampled(env):
    U, orc, torch = env
    c = W.paper_res_case()
    p, s = c.prob, c.search
    u0g, u1g, Jg = U.solve(p, s, 4, torch.as_tensor(c.u0_init).cuda(), "fp32_kahan")
    u0 = u0g.cpu().numpy()
    u1 = u1g.cpu().numpy()
    # objective of the state, in full
    Jo = orc.objective(p, u0, u1)
    assert abs(Jg.cpu().numpy()[-1] - Jo) <= 1e-12 * Jo
    # one more u0 update from this state, sampled rows
    got = U.argmin_adaptive(p, s, u1g, u0g, "fp32_kahan").cpu().numpy()
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(p.n_x, 192, replace=False))
    rows = np.concatenate([rows, [0, 1, p.n_x // 2, p.n_x - 2, p.n_x - 1]])  # edges and the x = 0 node
    assert _check_rows(orc, p, s, u1, u0, got, rows) <= 1
    # u1 of the updated u0 (four y nodes per lane), sampled rows
    u1n = U.update_u1(p, torch.as_tensor(got).cuda(), "fp32_kahan").cpu().numpy()
    yr = np.sort(rng.choice(p.n_y, 256, replace=False))
    ref = orc.update_u1(p, got, rows=yr)
    assert np.max(np.abs(u1n[yr] - ref)) <= 2e-5


def test_large_mixture_batch_sampled(env):
    U, orc, torch = env
    cases = [W.mixture_case(s, n=65536, iters=1) for s in (0, 1, 2, 3)]
    u0s, u1s, Js = U.solve_batch([c.prob for c in cases], [c.search for c in cases], [1] * len(cases),
                                 [torch.as_tensor(c.u0_init).cuda() for c in cases])
    rng = np.random.default_rng(1)
    for b, c in enumerate(cases):
        p, s = c.prob, c.search
        # round 1 started from u0 = 0 with u1 of u0 = 0: recompute that u1 with the oracle on
        # sampled rows would not give the GPU's input exactly, so take the GPU u1 of the
        # initial state and check the u0 update against the oracle given it
        u1_0 = U.update_u1(p, torch.as_tensor(c.u0_init).cuda(), "fp32_kahan")
        # u1 at full size (four y nodes per lane) on sampled rows, in the
        # FP32 modes' arithmetic and in FP64
        yr = np.sort(np.concatenate([rng.choice(p.n_y, 256, replace=False), [0, p.n_y // 2, p.n_y - 1]]))
        ref1 = orc.update_u1(p, c.u0_init, rows=yr)
        assert np.max(np.abs(u1_0.cpu().numpy()[yr] - ref1)) <= 2e-5
        u1_64 = U.update_u1(p, torch.as_tensor(c.u0_init).cuda(), "fp64").cpu().numpy()
        assert np.max(np.abs(u1_64[yr] - ref1)) <= 1e-11
        got = U.argmin_adaptive(p, s, u1_0, torch.as_tensor(c.u0_init).cuda(), "fp32_kahan").cpu().numpy()
        assert np.array_equal(got, u0s[b].cpu().numpy())  # the same update as inside the batched solve
        rows = np.sort(np.concatenate([rng.choice(p.n_x, 256, replace=False), [0, p.n_x // 2, p.n_x - 1]]))
        assert _check_rows(orc, p, s, u1_0.cpu().numpy(), c.u0_init, got, rows) <= 1
        Jo = orc.objective(p, u0s[b].cpu().numpy(), u1s[b].cpu().numpy())
        assert abs(Js[b].cpu().numpy()[-1] - Jo) <= 1e-12 * Jo


@pytest.mark.parametrize("prec", ["fp32_kahan", "fp32"])
def test_marginal_cost_spread_blocks_sampled(env, prec):
    """Blocks whose positions spread over more nodes than the LDS stage holds.
    Candidates 30 apart between neighbouring points and between the two
    halves of each block of 256 points (global reads), 6 apart (one stage,
    residual form), 3.4 apart (reference form), and uniform over the search
    range (global reads).  Sampled (point, candidate) pairs against the
    oracle's B."""
    U, orc, torch = env
    p = W.gaussian_problem(0.2, 5.0, 20001, 25.0)
    x = orc.grid(p.x_lo, p.x_hi, p.n_x)
    y = orc.grid(p.y_lo, p.y_hi, p.n_y)
    u1 = 5.0 * np.tanh(y / 5.0)  # a smooth synthetic second controller
    n = p.n_x
    sgn = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    rng = np.random.default_rng(4)
    halves = np.where(np.arange(n) % 256 < 128, 1.0, -1.0)
    u = np.stack([15.0 * sgn, 0.3 - 15.0 * sgn, 3.0 * sgn, 1.7 * sgn, rng.uniform(-30.0, 30.0, n), 15.0 * halves],
                 axis=1)
    got = U.marginal_cost(p, torch.as_tensor(u1).cuda(), torch.as_tensor(u).cuda(), prec).cpu().numpy()
    f, _ = orc.prior(p)
    rows = np.sort(rng.choice(n, 120, replace=False))
    worst = 0.0
    for i in rows:
        if not f[i] > 1e-280:
            continue
        for q in range(u.shape[1]):
            ref = f[i] * orc.B(p, u1, x[i], u[i, q])
            worst = max(worst, abs(got[i, q] - ref) / ref)
    assert worst <= 2e-5, worst
