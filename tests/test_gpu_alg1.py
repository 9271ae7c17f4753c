"""GPU parity of the generic solver (Algorithm 1) against the FP64 oracle.

  - one local update of u0 (modified Newton on B): within 1e-10 of the
    oracle's step (the FP64 moments agree to ~1e-13; the step divides B' by
    B'');
  - one partial exhaustion of u0 and of u1: decisions equal to the
    oracle's, a differing point an FP64 near-tie;
  - whole solves on 401- and 1001-node grids from the identity controllers
    (the paper's initialisation), N = 20, r = 2, p = 1e-10: the same number
    of rounds, the same allocation of each round, J at termination within
    1e-9 of the oracle's and after every phase within 1e-4.  The early
    phases are ill-conditioned: from the identity, Newton steps at points
    of small positive curvature amplify rounding, and the oracle itself,
    its u0 perturbed by 1e-14 relative after each local update, moves J
    after the first phase by 1.6e-5 and after the fifth by 2e-7, while its
    J at termination moves by 1e-15;
  - at 20001 nodes (sampled rows): a local update and a partial exhaustion
    of u0 from a state several rounds into the solve.
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


def dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def _state(orc, p, seed):
    """A state partway through a solve: the sign controller with a seeded
    perturbation, and the closed-form u1 of another controller (so neither
    update is at its fixed point)."""
    rng = np.random.default_rng(seed)
    x = orc.grid(p.x_lo, p.x_hi, p.n_x)
    u0 = 5.0 * np.sign(x) - x + rng.normal(0.0, 0.3, p.n_x)
    u1 = orc.update_u1(p, W.init_random_steps(p, 5.0, seed))
    return u0, u1


CASES = {
    "401": lambda: W.gaussian_problem(0.2, 5.0, 401, 25.0),
    "ragged": lambda: W.Problem(0.3, [(0.7, -2.0, 3.0), (0.3, 6.0, 2.0)], -20, 22, 577, -24, 26, 801),
    "noise0.7": lambda: W.Problem(0.25, [(1.0, 0.0, 4.0)], -25, 25, 601, -25, 25, 601, noise_sd=0.7),
}


@pytest.mark.parametrize("name", list(CASES))
def test_local_update_u0(env, name):
    U, orc, torch = env
    p = CASES[name]()
    u0, u1 = _state(orc, p, 1)
    for tau in (0.1, 0.5):
        ref = orc.alg1_local_u0(p, tau, u1, u0)
        got = host(U.alg1_local_u0(p, tau, dev(torch, u1), dev(torch, u0)))
        assert np.max(np.abs(got - ref) / (1.0 + np.abs(ref))) <= 1e-10, (name, tau)


@pytest.mark.parametrize("r", [1, 2])
@pytest.mark.parametrize("name", list(CASES))
def test_partial_exhaustion(env, name, r):
    U, orc, torch = env
    p = CASES[name]()
    u0, u1 = _state(orc, p, 2)
    x = orc.grid(p.x_lo, p.x_hi, p.n_x)
    ref = orc.alg1_pe_u0(p, u1, u0, r=r)
    got = host(U.alg1_pe_u0(p, dev(torch, u1), dev(torch, u0), r=r))
    for i in np.nonzero(got != ref)[0]:
        assert orc.B(p, u1, x[i], got[i]) <= orc.B(p, u1, x[i], ref[i]) * (1 + near_tie()), (name, i)
    assert np.sum(got != ref) <= max(1, p.n_x // 1000)
    ref1 = orc.alg1_pe_u1(p, u0, u1, r=r)
    got1 = host(U.alg1_pe_u1(p, dev(torch, u0), dev(torch, u1), r=r))
    assert np.sum(got1 != ref1) <= max(1, p.n_y // 1000), name


@pytest.mark.parametrize("n", [401, 1001])
def test_whole_solve(env, n):
    U, orc, torch = env
    p = W.gaussian_problem(0.2, 5.0, n, 25.0)
    x = orc.grid(p.x_lo, p.x_hi, p.n_x)
    y = orc.grid(p.y_lo, p.y_hi, p.n_y)
    u0r, u1r, Jr, NLr = orc.alg1_solve(p, x.copy(), y.copy(), max_rounds=60)
    u0g, u1g, Jg, NLg = U.alg1_solve(p, dev(torch, x), dev(torch, y), max_rounds=60)
    Jg = host(Jg)
    print(f"n = {n}: {len(NLr)} rounds, J {Jr[0]:.6f} -> {Jr[-1]:.9f}; GPU {len(NLg)} rounds, J {Jg[-1]:.9f}")
    rel = np.abs(Jg - Jr) / Jr
    print(f"J rel err per phase: max {rel.max():.2e} (phase {rel.argmax()}), at termination {rel[-1]:.2e}")
    assert len(NLg) == len(NLr) and list(NLg) == list(NLr)
    assert rel[-1] <= 1e-9
    assert rel.max() <= 1e-4


def test_full_size_sampled(env):
    U, orc, torch = env
    p = W.gaussian_problem(0.2, 5.0, 20001, 25.0)
    u0, u1 = _state(orc, W.gaussian_problem(0.2, 5.0, 20001, 25.0), 3)
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(p.n_x, 96, replace=False))
    ref = orc.alg1_local_u0(p, 0.1, u1, u0, rows=rows)
    got = host(U.alg1_local_u0(p, 0.1, dev(torch, u1), dev(torch, u0)))[rows]
    assert np.max(np.abs(got - ref) / (1.0 + np.abs(ref))) <= 1e-10
    ref = orc.alg1_pe_u0(p, u1, u0, rows=rows)
    got = host(U.alg1_pe_u0(p, dev(torch, u1), dev(torch, u0)))[rows]
    assert np.sum(got != ref) <= 1
    yrows = np.sort(rng.choice(p.n_y, 48, replace=False))
    ref1 = orc.alg1_pe_u1(p, u0, u1, rows=yrows)
    got1 = host(U.alg1_pe_u1(p, dev(torch, u0), dev(torch, u1)))[yrows]
    assert np.sum(got1 != ref1) <= 1
