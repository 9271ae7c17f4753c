"""Edge cases of the GPU path against the FP64 oracle: extreme search
shapes, clamped and duplicated candidates, positions far outside the y grid,
k = 0, minimal and coarse grids, zero rounds, non-finite input."""
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


def check_update(U, orc, torch, p, s, u0, prec="fp32_kahan"):
    u1 = orc.update_u1(p, u0)
    ref, Bref = orc.argmin(p, s, u1, u0)
    got = U.argmin_adaptive(p, s, dev(torch, u1), dev(torch, u0), prec).cpu().numpy()
    x = orc.grid(p.x_lo, p.x_hi, p.n_x)
    diff = np.nonzero(got != ref)[0]
    for i in diff:
        bg = orc.B(p, u1, x[i], got[i])
        assert bg <= Bref[i] * (1 + near_tie(s.tie_rel64 or 1e-12)) + 1e-300, (i, got[i], ref[i], bg, Bref[i])
    assert len(diff) <= max(1, p.n_x // 1000)
    return got


def check_solve(U, orc, torch, p, s, iters, u0, prec="fp32_kahan"):
    u0r, u1r, Jr = orc.solve(p, s, iters, u0)
    u0g, u1g, Jg = (t.cpu().numpy() for t in U.solve(p, s, iters, dev(torch, u0), prec))
    rel = np.abs(Jg - Jr) / np.abs(Jr)
    assert rel.max() <= 1e-6, rel
    assert np.all(Jg[1:] <= Jg[:-1] * (1 + 1e-12))
    return u0g, u1g, Jg


SEARCHES = [
    ("one-level", W.Search(-30, 30, 1, 21)),
    ("two-cands", W.Search(-30, 30, 6, 2)),
    ("max-cands", W.Search(-30, 30, 2, 63)),
    ("max-levels", W.Search(-30, 30, 16, 4)),
    ("narrow-clamped", W.Search(-0.5, 0.5, 4, 9)),
]


@pytest.mark.parametrize("name,s", SEARCHES, ids=[n for n, _ in SEARCHES])
def test_search_shapes(env, name, s):
    U, orc, torch = env
    p = W.gaussian_problem(0.2, 5.0, 301, 25.0)
    u0 = W.init_random_steps(p, 5.0, 3)
    check_update(U, orc, torch, p, s, u0)
    check_solve(U, orc, torch, p, s, 3, u0)


def test_positions_far_outside_y_grid(env):
    """x grid wider than the y grid: many x + u lie beyond the y grid, some by
    more than the window (the window then covers the nodes at the edge)."""
    U, orc, torch = env
    p = W.Problem(0.3, [(1.0, 0.0, 6.0)], -40.0, 40.0, 401, -12.0, 12.0, 481)
    s = W.Search(-20, 20, 3, 11)
    u0 = W.init_random_steps(p, 6.0, 1)
    check_update(U, orc, torch, p, s, u0)
    check_solve(U, orc, torch, p, s, 3, u0)
    u1 = orc.update_u1(p, u0)
    u = np.stack([u0, np.full(p.n_x, 15.0), np.full(p.n_x, -15.0)], axis=1)
    ref = orc.marginal_cost(p, u1, u)
    for prec, tol in (("fp64", 1e-12), ("fp32_kahan", 2e-5)):
        got = U.marginal_cost(p, dev(torch, u1), dev(torch, u), prec).cpu().numpy()
        ok = ref > 1e-290
        assert np.max(np.abs(got[ok] - ref[ok]) / ref[ok]) <= tol


def test_zero_stage_one_cost(env):
    U, orc, torch = env
    p = W.Problem(0.0, [(1.0, 0.0, 3.0)], -15.0, 15.0, 301, -22.0, 22.0, 441)
    s = W.Search(-6, 6, 3, 13)
    u0 = W.init_random_steps(p, 3.0, 2)
    check_update(U, orc, torch, p, s, u0)
    check_solve(U, orc, torch, p, s, 2, u0)


def test_minimal_and_coarse_grids(env):
    U, orc, torch = env
    # two nodes each
    p = W.Problem(0.2, [(1.0, 0.0, 2.0)], -1.0, 1.0, 2, -3.0, 3.0, 2)
    s = W.Search(-2, 2, 2, 5)
    check_solve(U, orc, torch, p, s, 2, np.array([0.3, -0.1]))
    # y spacing larger than one noise sd: the window spans the whole grid
    p = W.Problem(0.2, [(1.0, 0.0, 5.0)], -25.0, 25.0, 101, -25.0, 25.0, 21)
    s = W.Search(-30, 30, 3, 9)
    u0 = W.init_sign(p, 5.0)
    check_update(U, orc, torch, p, s, u0)
    check_solve(U, orc, torch, p, s, 3, u0)


def test_zero_rounds(env):
    U, orc, torch = env
    c = W.small_case()
    u0g, u1g, Jg = (t.cpu().numpy() for t in U.solve(c.prob, c.search, 0, dev(torch, c.u0_init)))
    u1 = orc.update_u1(c.prob, c.u0_init)
    assert np.array_equal(u0g, c.u0_init)
    assert Jg.shape == (1,) and abs(Jg[0] - orc.objective(c.prob, c.u0_init, u1)) <= 1e-12 * Jg[0]


def test_nonfinite_input_is_reported(env):
    U, orc, torch = env
    c = W.small_case()
    bad = c.u0_init.copy()
    bad[10] = np.inf
    with pytest.raises(U.UcpError) as e:
        U.solve(c.prob, c.search, 2, dev(torch, bad))
    assert e.value.code == U.ENONFINITE
    # the handle stays usable
    check_solve(U, orc, torch, c.prob, c.search, 2, c.u0_init)


def test_invalid_arguments_on_device(env):
    U, orc, torch = env
    c = W.small_case()
    with pytest.raises(TypeError):
        U.solve(c.prob, c.search, 2, torch.as_tensor(c.u0_init))  # host tensor
    with pytest.raises(ValueError):
        U.solve(c.prob, c.search, 2, dev(torch, c.u0_init[:-1]))
    with pytest.raises(U.UcpError) as e:
        U.solve(c.prob, W.Search(1.0, -1.0, 3, 21), 2, dev(torch, c.u0_init))
    assert e.value.code == U.EINVAL
