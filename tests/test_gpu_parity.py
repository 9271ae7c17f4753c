"""GPU parity of every C-ABI call against the FP64 oracle, on identical
seeded inputs.

Tolerances (derived in the design notes from the arithmetic):
  - objective (FP64 throughout): relative 1e-12;
  - marginal cost, FP64 mode: relative 1e-12; FP32 modes: relative 2e-5
    (FP32 terms with centred arguments, worst case on small costs);
  - u1: FP64 mode 1e-11 absolute; FP32 modes 2e-5 absolute, on the nodes
    carrying output density p_y >= 1e-9 max p_y;
  - argmin: decisions equal to the oracle's; a differing point must be an
    FP64 near-tie (oracle cost at the GPU's choice within the tie band plus
    twice the GPU's FP64 error, ``tolerances.near_tie``);
  - solve: J relative error <= 1e-6 at every round.
"""
import math

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


def py_mask(orc, p, u0, u1):
    """Nodes whose output density p_y(j) = sum_i f_i phi(y_j - x1_i) is at
    least 1e-9 of its maximum."""
    f, _ = orc.prior(p)
    x1 = orc.grid(p.x_lo, p.x_hi, p.n_x) + u0
    y = orc.grid(p.y_lo, p.y_hi, p.n_y)
    sw = getattr(p, "noise_sd", 1.0)
    py = np.array([np.sum(f * np.exp(-0.5 * ((yy - x1) / sw) ** 2)) for yy in y])
    return py >= 1e-9 * py.max()


CASES = {
    "small": lambda: W.small_case(),
    "ragged": lambda: W.Case("ragged-n_x!=n_y", W.Problem(0.3, [(0.7, -2.0, 3.0), (0.3, 6.0, 2.0)], -20, 22, 777,
                                                          -24, 26, 1201), W.Search(-9, 11, 3, 13), 4,
                             W.init_random_steps(W.Problem(0.3, [(1, 0, 3)], -20, 22, 777, -24, 26, 1201), 4.0, 7)),
    "tiny": lambda: W.Case("tiny", W.gaussian_problem(0.2, 5.0, 21, 25.0), W.Search(-30, 30, 2, 5), 3,
                           W.init_sign(W.gaussian_problem(0.2, 5.0, 21, 25.0), 5.0)),
    # more candidates than half a wave holds: the selection runs one point per wave
    "wide": lambda: W.Case("wide-k40", W.gaussian_problem(0.2, 3.0, 401, 25.0), W.Search(-30, 30, 2, 40), 3,
                           W.init_random_steps(W.gaussian_problem(0.2, 3.0, 401, 25.0), 3.0, 5)),
    # the largest set that still runs two points per wave (30 candidates, the
    # carried best and the incumbent's queue lane fill 32 lanes); odd n_x
    "k30": lambda: W.Case("k30-two-per-wave", W.gaussian_problem(0.3, 4.0, 333, 25.0), W.Search(-30, 30, 3, 30), 3,
                          W.init_random_steps(W.gaussian_problem(0.3, 4.0, 333, 25.0), 4.0, 9)),
    # sigma = 10 with the sign controller and k = 0.05: points at x = +-sigma
    # map onto flat steps of u1, where B falls to ~1e-6 and a window of 9
    # noise sds loses 3.5e-12 of it (the FP64 window is 11 sds)
    "s10": lambda: W.Case("sigma10-k0.05-sign", W.gaussian_problem(0.05, 10.0, 2001, 50.0), W.Search(-55, 55, 3, 21),
                          3, W.init_sign(W.gaussian_problem(0.05, 10.0, 2001, 50.0), 10.0), 10.0),
    # noise w ~ N(0, 0.7^2): every window, weight and normalisation in noise sds
    "noise0.7": lambda: _noise_case(0.7),
}


def _noise_case(sw):
    p = W.gaussian_problem(0.25, 4.0, 1201, 25.0)
    p.noise_sd = sw
    return W.Case(f"noise{sw}", p, W.Search(-30, 30, 3, 21), 3, W.init_random_steps(p, 4.0, 12), 4.0)


# ------------------------------------------------------------- objective

@pytest.mark.parametrize("name", list(CASES))
def test_objective(env, name):
    U, orc, torch = env
    c = CASES[name]()
    p = c.prob
    u1 = orc.update_u1(p, c.u0_init)
    J = orc.objective(p, c.u0_init, u1)
    Jg = host(U.objective(p, dev(torch, c.u0_init), dev(torch, u1)))[0]
    assert abs(Jg - J) <= 1e-12 * abs(J), (Jg, J)


def test_objective_affine_closed_form(env):
    """The GPU objective against the closed form too (not only the oracle)."""
    U, orc, torch = env
    p = W.gaussian_problem(0.2, 5.0, 2401, 60.0)
    for lam, ref in [(1.0, 25 / 26), (0.0417424305044, 0.96)]:
        u0 = W.init_affine(p, lam)
        y = orc.grid(p.y_lo, p.y_hi, p.n_y)
        g = lam * lam * 25 / (1 + lam * lam * 25)
        Jg = host(U.objective(p, dev(torch, u0), dev(torch, g * y)))[0]
        assert abs(Jg - ref) <= 1e-10 * ref


# ----------------------------------------------------------- u1 update

@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32_kahan", 2e-5), ("fp32", 2e-5)])
@pytest.mark.parametrize("name", list(CASES))
def test_update_u1(env, name, prec, tol):
    U, orc, torch = env
    c = CASES[name]()
    p = c.prob
    u0 = W.init_random_steps(p, 5.0, 11) if name == "small" else c.u0_init
    ref = orc.update_u1(p, u0)
    got = host(U.update_u1(p, dev(torch, u0), prec))
    m = py_mask(orc, p, u0, ref)
    err = np.max(np.abs(got[m] - ref[m]))
    assert err <= tol, err
    assert np.all(np.isfinite(got))


# Grids of at least 16384 y nodes spaced at most 0.05 noise sds take four
# consecutive y nodes per lane in the u1 sums (one exponential per x node
# and lane, the other nodes by a staged ratio).  Narrow x grids keep the
# oracle quick; 33001 nodes end on a ragged tile whose last lane holds one
# node; 16384 nodes sit on the threshold, 16383 stay at one node per lane.
NPL_CASES = {
    "mix-33001": lambda: W.Problem(0.2, [(0.5, -6.0, 2.0), (0.3, 3.0, 1.5), (0.2, 9.0, 3.0)], -20, 22, 2001,
                                   -40, 40, 33001),
    "gauss-16384": lambda: W.Problem(0.2, [(1.0, 0.0, 5.0)], -25, 25, 1501, -40, 40, 16384),
    "noise0.7-40001": lambda: _with_noise(W.Problem(0.25, [(1.0, 0.0, 4.0)], -25, 25, 1201, -30, 30, 40001), 0.7),
    "one-per-lane-16383": lambda: W.Problem(0.2, [(1.0, 0.0, 5.0)], -25, 25, 1501, -40, 40, 16383),
}


def _with_noise(p, sw):
    p.noise_sd = sw
    return p


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32_kahan", 2e-5), ("fp32", 2e-5)])
@pytest.mark.parametrize("name", list(NPL_CASES))
def test_update_u1_nodes_per_lane(env, name, prec, tol):
    U, orc, torch = env
    p = NPL_CASES[name]()
    u0 = W.init_random_steps(p, 5.0, 17)
    ref = orc.update_u1(p, u0)
    got = host(U.update_u1(p, dev(torch, u0), prec))
    m = py_mask(orc, p, u0, ref)
    err = np.max(np.abs(got[m] - ref[m]))
    assert err <= tol, err
    assert np.all(np.isfinite(got))
    # the ragged tile's last nodes and the grid's ends
    assert np.all(np.abs(got[-5:] - ref[-5:])[m[-5:]] <= tol) and np.all(np.abs(got[:5] - ref[:5])[m[:5]] <= tol)


# -------------------------------------------------------- marginal cost

@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32_kahan", 2e-5), ("fp32", 2e-5)])
@pytest.mark.parametrize("name", list(CASES))
def test_marginal_cost(env, name, prec, tol):
    U, orc, torch = env
    c = CASES[name]()
    p, s = c.prob, c.search
    u1 = orc.update_u1(p, c.u0_init)
    rng = np.random.default_rng(3)
    n_c = 7
    u = rng.uniform(s.u_lo, s.u_hi, (p.n_x, n_c))
    u[:, 0] = c.u0_init
    u[:, 1] = 0.0
    ref = orc.marginal_cost(p, u1, u)
    got = host(U.marginal_cost(p, dev(torch, u1), dev(torch, u), prec))
    f, _ = orc.prior(p)
    ok = f > 1e-280  # f underflows to 0 in FP64 beyond ~37 prior sds
    rel = np.abs(got[ok] - ref[ok]) / np.abs(ref[ok])
    assert np.max(rel) <= tol, np.max(rel)


# --------------------------------------------------------------- argmin

@pytest.mark.parametrize("prec", ["fp32_kahan", "fp32", "fp64"])
@pytest.mark.parametrize("name", list(CASES))
def test_argmin_decisions(env, name, prec):
    U, orc, torch = env
    c = CASES[name]()
    p, s = c.prob, c.search
    u0 = c.u0_init
    u1 = orc.update_u1(p, u0)
    ref, Bref = orc.argmin(p, s, u1, u0)
    got, L0 = U.argmin_adaptive(p, s, dev(torch, u1), dev(torch, u0), prec, want_l0=True)
    got, L0 = host(got), host(L0)
    diff = np.nonzero(got != ref)[0]
    x = orc.grid(p.x_lo, p.x_hi, p.n_x)
    for i in diff:  # only FP64 near-ties may differ
        bg = orc.B(p, u1, x[i], got[i])
        assert bg <= Bref[i] * (1 + near_tie()), (i, got[i], ref[i], bg, Bref[i])
    assert len(diff) <= max(1, p.n_x // 1000)
    f, _ = orc.prior(p)
    ok = f > 1e-280
    Lref = f * np.array([orc.B(p, u1, x[i], got[i]) for i in range(p.n_x)])
    assert np.max(np.abs(L0[ok] - Lref[ok]) / Lref[ok]) <= 1e-12


# ---------------------------------------------------------------- solve

@pytest.mark.parametrize("prec", ["fp32_kahan", "fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_solve(env, name, prec):
    U, orc, torch = env
    c = CASES[name]()
    p, s = c.prob, c.search
    u0r, u1r, Jr = orc.solve(p, s, c.iters, c.u0_init)
    u0g, u1g, Jg = (host(t) for t in U.solve(p, s, c.iters, dev(torch, c.u0_init), prec))
    rel = np.abs(Jg - Jr) / Jr
    print(f"{name} {prec} J rel err per round: {rel.max():.2e}; u0 differs at {np.sum(u0g != u0r)} points")
    assert rel.max() <= 1e-6
    assert np.all(Jg[1:] <= Jg[:-1] * (1 + 1e-12))  # monotone (the incumbent is always a candidate)


def test_solve_is_deterministic_and_resumable(env):
    U, orc, torch = env
    c = W.small_case()
    p, s = c.prob, c.search
    a = [host(t) for t in U.solve(p, s, 4, dev(torch, c.u0_init))]
    b = [host(t) for t in U.solve(p, s, 4, dev(torch, c.u0_init))]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    h1 = [host(t) for t in U.solve(p, s, 2, dev(torch, c.u0_init))]
    h2 = [host(t) for t in U.solve(p, s, 2, dev(torch, h1[0]))]
    assert np.array_equal(h2[0], a[0]) and np.array_equal(h2[1], a[1])
    assert np.array_equal(h2[2][1:], a[2][3:])


# ------------------------------------------------------- batch / serving

def _mix():
    out = [W.small_case(), CASES["ragged"](), CASES["tiny"](), CASES["wide"]()]
    p = W.gaussian_problem(0.1, 2.0, 4001, 25.0)
    out.append(W.Case("n4001", p, W.Search(-30, 30, 3, 21), 2, W.init_sign(p, 2.0), 2.0))
    return out


def test_batch_equals_alone(env):
    U, orc, torch = env
    cases = _mix()
    alone = [[host(t) for t in U.solve(c.prob, c.search, c.iters, dev(torch, c.u0_init))] for c in cases]
    u0s, u1s, Js = U.solve_batch([c.prob for c in cases], [c.search for c in cases], [c.iters for c in cases],
                                 [dev(torch, c.u0_init) for c in cases])
    for b, c in enumerate(cases):
        assert np.array_equal(host(u0s[b]), alone[b][0]), c.name
        assert np.array_equal(host(u1s[b]), alone[b][1]), c.name
        assert np.array_equal(host(Js[b]), alone[b][2]), c.name


def test_server_mix_equals_alone(env):
    U, orc, torch = env
    cases = _mix() * 2
    alone = [[host(t) for t in U.solve(c.prob, c.search, c.iters, dev(torch, c.u0_init))] for c in cases]
    srv = U.Server(max_slots=3)
    tickets = []
    for k, c in enumerate(cases):  # staggered arrivals: submit while others run
        tickets.append(srv.submit(c.prob, c.search, c.iters, c.u0_init))
        if k % 2:
            srv.step()
    res = {}
    for _ in range(200):
        n = srv.step()
        for t in tickets:
            if t not in res:
                r = srv.poll(t)
                if r is not None:
                    res[t] = r
        if len(res) == len(tickets):
            break
    assert len(res) == len(tickets)
    for t, c, a in zip(tickets, cases, alone):
        u0, u1, J = res[t]
        assert np.array_equal(u0, a[0]) and np.array_equal(u1, a[1]) and np.array_equal(J, a[2]), c.name
    srv.close()


def test_server_budget_cancel_and_nan(env):
    U, orc, torch = env
    c = W.small_case()
    srv = U.Server(max_slots=8, hbm_budget=1)
    with pytest.raises(U.UcpError):  # can never fit
        srv.submit(c.prob, c.search, 2, c.u0_init)
    srv.close()
    # a budget that fits exactly one request: the second waits for the first
    fp = U.footprint(c.prob, c.search, 3)
    srv = U.Server(max_slots=8, hbm_budget=fp + fp // 2)
    t1 = srv.submit(c.prob, c.search, 3, c.u0_init)
    t2 = srv.submit(c.prob, c.search, 3, c.u0_init)
    srv.step()
    q, r, d = srv.stats()
    assert (q, r) == (1, 1)
    bad = c.u0_init.copy()
    bad[500] = np.nan
    t3 = srv.submit(c.prob, c.search, 2, bad)
    t4 = srv.submit(c.prob, c.search, 2, c.u0_init)
    srv.cancel(t4)
    out = {}
    for _ in range(50):
        srv.step()
        for t in (t1, t2):
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        if t3 not in out:
            try:
                r = srv.poll(t3)
                if r is not None:
                    out[t3] = r
            except U.UcpError as e:
                assert e.code == U.ENONFINITE
                out[t3] = "nonfinite"
        if len(out) == 3:
            break
    assert out[t3] == "nonfinite"
    ref = [host(t) for t in U.solve(c.prob, c.search, 3, dev(torch, c.u0_init))]
    for t in (t1, t2):
        assert np.array_equal(out[t][2], ref[2])
    srv.close()


# ------------------------------------------------- search-record fields

def test_tie_band_parameter(env):
    """The relative tie band of the search record, as in the oracle's pin:
    with u1 = a y the incumbent at u = d costs (k^2 + (1-a)^2) d^2 / a^2 more
    than the minimum u = 0; a band wider than that keeps it.  GPU decisions
    equal the oracle's for the default band, a narrower and a wider one, in
    every arithmetic."""
    U, orc, torch = env
    p = W.Problem(k=0.2, comps=[(1.0, 0.0, 5.0)], x_lo=-10.0, x_hi=10.0, n_x=101, y_lo=-40.0, y_hi=40.0, n_y=1601)
    y = orc.grid(p.y_lo, p.y_hi, p.n_y)
    a, d = 0.5, 0.01
    delta = (0.04 + (1 - a) ** 2) * d * d / (a * a)
    u0 = np.full(p.n_x, d)
    for tau in (0.0, 0.5 * delta, 2.0 * delta):
        s = W.Search(-2.0, 2.0, 1, 11, tie_rel64=tau)
        ref, _ = orc.argmin(p, s, a * y, u0)
        for prec in ("fp32_kahan", "fp32", "fp64"):
            got = host(U.argmin_adaptive(p, s, dev(torch, a * y), dev(torch, u0), prec))
            assert np.array_equal(got, ref), (tau, prec)
        assert (ref[p.n_x // 2] == d) == (tau > delta)


def test_wider_fp32_band_same_result_more_fp64_sums(env):
    """A wider FP32 pre-selection band only sends more candidates to the FP64
    re-evaluation: the solve is bitwise the same and counts more FP64 sums."""
    U, orc, torch = env
    c = W.small_case()
    a = [host(t) for t in U.solve(c.prob, c.search, 3, dev(torch, c.u0_init))]
    _, _, e0 = U.last_counts()
    s = W.Search(c.search.u_lo, c.search.u_hi, c.search.levels, c.search.cands, band_rel32=1e-4)
    b = [host(t) for t in U.solve(c.prob, s, 3, dev(torch, c.u0_init))]
    _, _, e1 = U.last_counts()
    for x, z in zip(a, b):
        assert np.array_equal(x, z)
    assert e1 > e0


def test_noise_sd_scaling_is_exact_on_gpu(env):
    """Doubling every length and the noise sd scales the discrete problem
    exactly in binary64 (the log prior only shifts by log 2, which the u1
    weights' max-shift removes up to rounding), and the kernels' FP32 forms
    too (alpha halves as the differences double; the offsets in noise sds
    are unchanged): the GPU solve of the doubled problem is the unit one
    times 2 (u0 bit for bit, u1 to rounding) and 4 (J), in every
    arithmetic.  (In the FP32 modes u1's weights are FP32 exponentials of
    logits that differ by that rounding, so u1 agrees to the FP32 weights'
    precision there.)"""
    U, orc, torch = env
    c = W.small_case()
    p1, s1 = c.prob, c.search
    p2 = W.Problem(k=p1.k, comps=[(1.0, 0.0, 10.0)], x_lo=-50.0, x_hi=50.0, n_x=p1.n_x, y_lo=-50.0, y_hi=50.0,
                   n_y=p1.n_y, noise_sd=2.0)
    s2 = W.Search(2 * s1.u_lo, 2 * s1.u_hi, s1.levels, s1.cands)
    for prec in ("fp32_kahan", "fp32", "fp64"):
        a = [host(t) for t in U.solve(p1, s1, 3, dev(torch, c.u0_init), prec)]
        b = [host(t) for t in U.solve(p2, s2, 3, dev(torch, 2.0 * c.u0_init), prec)]
        assert np.array_equal(b[0], 2.0 * a[0]), prec
        tol = 1e-13 if prec == "fp64" else 1e-7
        assert np.max(np.abs(b[1] - 2.0 * a[1])) <= tol * np.max(np.abs(b[1])), prec
        assert np.max(np.abs(b[2] - 4.0 * a[2]) / b[2]) <= 1e-13, prec


def test_handle_budget(env):
    """ucp_create's workspace budget: a solve whose workspace exceeds it
    fails with UCP_ENOMEM and enqueues nothing; one that fits runs."""
    import ctypes as C

    U, orc, torch = env
    lib = U.library()
    c = W.small_case()
    P, S = U.make_problem(c.prob), U.make_search(c.search)
    fp = U.footprint(c.prob, c.search, 2)
    u0 = dev(torch, c.u0_init)
    out0 = torch.empty_like(u0)
    out1 = torch.empty(c.prob.n_y, dtype=torch.float64, device="cuda")
    J = torch.empty(3, dtype=torch.float64, device="cuda")
    for budget, want in ((fp // 4, U.ENOMEM), (4 * fp, U.OK)):
        h = C.c_void_p()
        assert lib.ucp_create(C.byref(h), 0, budget) == U.OK
        rc = lib.ucp_solve(h, C.byref(P), C.byref(S), 1, 2, C.c_void_p(u0.data_ptr()), C.c_void_p(out0.data_ptr()),
                           C.c_void_p(out1.data_ptr()), C.c_void_p(J.data_ptr()), None)
        lib.ucp_destroy(h)
        assert rc == want, (budget, rc, U.last_error())
    ref = [host(t) for t in U.solve(c.prob, c.search, 2, u0)]
    assert np.array_equal(host(J), ref[2])


def test_far_apart_positions_coarse_grid(env):
    """FP64 passes over the union of several positions' windows (the
    objective's rows four at a time, the selection's winner with a distant
    incumbent) on a coarse grid (dy = 0.1, so one wave step spans 6.4 noise
    sds): x1 alternates between -30 and +30 from point to point, so each
    union starts 60 sds away from half its positions, whose weights must
    still be seeded exactly before their windows.  Objective within 1e-12 of
    the oracle; an update from there matches the oracle's decisions and L_0."""
    U, orc, torch = env
    p = W.gaussian_problem(0.2, 5.0, 801, 40.0)
    x = orc.grid(p.x_lo, p.x_hi, p.n_x)
    u0 = np.where(np.arange(p.n_x) % 2 == 0, 30.0, -30.0) - x
    u1 = orc.update_u1(p, u0)
    J = orc.objective(p, u0, u1)
    Jg = host(U.objective(p, dev(torch, u0), dev(torch, u1)))[0]
    assert abs(Jg - J) <= 1e-12 * J, (Jg, J)
    s = W.Search(-75, 75, 3, 21)
    ref, Bref = orc.argmin(p, s, u1, u0)
    f, _ = orc.prior(p)
    for prec in ("fp32_kahan", "fp64"):
        got, L0 = U.argmin_adaptive(p, s, dev(torch, u1), dev(torch, u0), prec, want_l0=True)
        got, L0 = host(got), host(L0)
        diff = np.nonzero(got != ref)[0]
        for i in diff:
            assert orc.B(p, u1, x[i], got[i]) <= Bref[i] * (1 + near_tie()), (prec, i)
        assert len(diff) <= 1
        ok = f > 1e-280
        Lref = f * np.array([orc.B(p, u1, x[i], got[i]) for i in range(p.n_x)])
        assert np.max(np.abs(L0[ok] - Lref[ok]) / Lref[ok]) <= 1e-12, prec
