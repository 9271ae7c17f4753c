"""The allocation-free u0 update (ucp_argmin_adaptive_noalloc, through the C
ABI) against ucp_argmin_adaptive on the same inputs: u0 and L_0 bitwise
equal (the same kernels on the same layout), on two calls in a row, the
second on a smaller problem, so the scratch array's leftovers from the
first call cannot show in the second.  Each case is also checked against
the FP64 oracle on sampled rows."""
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


def _case(U, orc, torch, c, prec):
    p, s = c.prob, c.search
    u0 = torch.as_tensor(c.u0_init).cuda()
    u1 = U.update_u1(p, u0, prec)
    ref, l0r = U.argmin_adaptive(p, s, u1, u0, prec, want_l0=True)
    out = torch.full_like(u0, float("nan"))
    l0 = torch.full_like(u0, float("nan"))
    U.argmin_adaptive_noalloc(p, s, u1, u0, out, l0, prec)
    torch.cuda.synchronize()
    assert torch.equal(out, ref) and torch.equal(l0, l0r), c.name
    # and against the oracle on sampled rows, given the same u1
    rows = np.sort(np.random.default_rng(0).choice(p.n_x, 64, replace=False))
    u1h, got = u1.cpu().numpy(), out.cpu().numpy()
    want, Bw = orc.argmin(p, s, u1h, c.u0_init, rows=rows)
    x = orc.grid(p.x_lo, p.x_hi, p.n_x)
    for r in np.nonzero(got[rows] != want)[0]:
        assert orc.B(p, u1h, x[rows[r]], got[rows[r]]) <= Bw[r] * (1 + near_tie())


@pytest.mark.parametrize("prec", ["fp32_kahan", "fp64"])
def test_noalloc_equals_argmin_two_calls(env, prec):
    U, orc, torch = env
    _case(U, orc, torch, W.paper_res_case(), prec)  # 20001 nodes, 5 x 16
    _case(U, orc, torch, W.small_case(), prec)      # then 1001 nodes, 3 x 21


def test_noalloc_in_place_and_limit(env):
    U, orc, torch = env
    c = W.small_case()
    p, s = c.prob, c.search
    u0 = torch.as_tensor(c.u0_init).cuda()
    u1 = U.update_u1(p, u0)
    ref = U.argmin_adaptive(p, s, u1, u0)
    inplace = u0.clone()
    U.argmin_adaptive_noalloc(p, s, u1, inplace, inplace)  # u0_in and u0_out alias
    assert torch.equal(inplace, ref)
    # a problem beyond the fixed scratch is refused with an error, nothing run
    big = W.gaussian_problem(0.2, 5.0, 400001, 25.0)
    z = torch.zeros(big.n_x, dtype=torch.float64, device="cuda")
    with pytest.raises(U.UcpError) as e:
        U.argmin_adaptive_noalloc(big, W.Search(-30, 30, 2, 32), torch.zeros(big.n_y, dtype=torch.float64,
                                                                           device="cuda"), z, z.clone())
    assert e.value.code == U.EINVAL
