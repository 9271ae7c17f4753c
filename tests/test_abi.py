"""CPU checks of the C ABI: the library loads, exports every function that
include/ucp.h declares, and rejects invalid arguments before touching a
device.  No compute call is made here (there is no GPU)."""
import ctypes as C
import os
import re

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def U():
    lib = os.path.join(ROOT, "paper_1908_04489_amd", "libucp.so")
    if not os.path.exists(lib):
        import importlib.util

        spec = importlib.util.spec_from_file_location("ucp_build",
                                                      os.path.join(ROOT, "paper_1908_04489_amd", "build.py"))
        B = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(B)
        B.build()
    import paper_1908_04489_amd as U

    return U


def test_exports_every_declared_function(U):
    names = U.header_functions()
    assert len(names) >= 17
    for n in ["ucp_marginal_cost", "ucp_argmin_adaptive", "ucp_update_u1", "ucp_objective", "ucp_solve",
              "ucp_solve_batch", "ucp_server_create", "ucp_server_submit", "ucp_server_step", "ucp_server_poll"]:
        assert n in names
    lib = U.library()
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_error_codes(U):
    assert U.library().ucp_version().startswith(b"ucp-mi355x")
    txt = open(os.path.join(ROOT, "include", "ucp.h")).read()
    codes = dict((m.group(1), int(m.group(2))) for m in re.finditer(r"(UCP_E\w+|UCP_OK) = (-?\d+)", txt))
    assert codes["UCP_OK"] == U.OK and codes["UCP_EINVAL"] == U.EINVAL and codes["UCP_EAGAIN"] == U.EAGAIN
    assert codes["UCP_ENONFINITE"] == U.ENONFINITE


def test_struct_layout_matches_header(U):
    # ucp_problem: k, n_comp, pad, 3 x 8 doubles, x range + n, y range + n
    assert C.sizeof(U.Problem) == 8 + 4 + 4 + 3 * 8 * 8 + 8 + 8 + 8 + 8 + 8 + 8 + 8  # ... noise_sd
    # ucp_search: range, levels, cands, tie_rel64, band_rel32
    assert C.sizeof(U.Search) == 8 + 8 + 4 + 4 + 8 + 8


def test_create_without_device_or_with_null(U):
    lib = U.library()
    assert lib.ucp_create(None, 0, 0) == U.EINVAL
    h = C.c_void_p()
    rc = lib.ucp_create(C.byref(h), 0, 0)
    assert rc in (U.EHIP, U.OK)  # no GPU in this container: EHIP
    if rc == U.OK:
        lib.ucp_destroy(h)
    lib.ucp_destroy(None)


def _bad_problems():
    good = W.gaussian_problem(0.2, 5.0, 101, 25.0)
    out = []
    for field, val in [("n_x", 1), ("n_y", 0), ("k", -1.0), ("k", float("nan")), ("x_lo", 30.0),
                       ("y_hi", -30.0), ("noise_sd", -1.0), ("noise_sd", float("nan")), ("noise_sd", 1e-9)]:
        p = W.gaussian_problem(0.2, 5.0, 101, 25.0)
        setattr(p, field, val)
        out.append(p)
    p = W.gaussian_problem(0.2, 5.0, 101, 25.0)
    p.comps = [(0.5, 0.0, 1.0)]  # weights do not sum to 1
    out.append(p)
    p = W.gaussian_problem(0.2, 5.0, 101, 25.0)
    p.comps = [(1.0, 0.0, 0.0)]  # sd 0
    out.append(p)
    p = W.gaussian_problem(0.2, 5.0, 101, 25.0)
    p.comps = [(0.1, 0.0, 1.0)] * 10  # too many components
    out.append(p)
    return good, out


def test_invalid_problem_rejected_before_device_use(U):
    """Argument checks come before any use of the handle or the device, so a
    placeholder handle is never dereferenced on these paths."""
    lib = U.library()
    fake = C.c_void_p(1)
    good, bad = _bad_problems()
    S = U.make_search(W.Search(-30, 30, 3, 21))
    for p in bad:
        if len(p.comps) > 8:
            P = U.Problem()
            P.k, P.n_comp, P.n_x, P.n_y = 0.2, 9, 101, 101
            P.x_lo, P.x_hi, P.y_lo, P.y_hi = -1, 1, -1, 1
        else:
            P = U.make_problem(p)
        assert lib.ucp_objective(fake, C.byref(P), C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), None) == U.EINVAL
        assert lib.ucp_argmin_adaptive(fake, C.byref(P), C.byref(S), 1, C.c_void_p(8), C.c_void_p(8),
                                       C.c_void_p(8), None, None) == U.EINVAL
        assert U.last_error() != ""
    P = U.make_problem(good)
    # bad search / precision / null arrays / null handle
    for s in [W.Search(30, -30, 3, 21), W.Search(-30, 30, 0, 21), W.Search(-30, 30, 3, 1),
              W.Search(-30, 30, 17, 21), W.Search(-30, 30, 3, 64),
              W.Search(-30, 30, 3, 21, tie_rel64=-1e-12), W.Search(-30, 30, 3, 21, tie_rel64=float("nan")),
              W.Search(-30, 30, 3, 21, tie_rel64=1e-2), W.Search(-30, 30, 3, 21, band_rel32=-1e-7),
              W.Search(-30, 30, 3, 21, band_rel32=0.5)]:
        S2 = U.make_search(s)
        assert lib.ucp_argmin_adaptive(fake, C.byref(P), C.byref(S2), 1, C.c_void_p(8), C.c_void_p(8),
                                       C.c_void_p(8), None, None) == U.EINVAL
    assert lib.ucp_argmin_adaptive(fake, C.byref(P), C.byref(S), 7, C.c_void_p(8), C.c_void_p(8),
                                   C.c_void_p(8), None, None) == U.EINVAL
    assert lib.ucp_update_u1(fake, C.byref(P), 1, None, C.c_void_p(8), None) == U.EINVAL
    assert lib.ucp_marginal_cost(fake, C.byref(P), 1, C.c_void_p(8), C.c_void_p(8), 0, C.c_void_p(8),
                                 None) == U.EINVAL
    assert lib.ucp_objective(None, C.byref(P), C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), None) == U.EINVAL
    its = (C.c_int32 * 1)(-1)
    arr = (C.c_void_p * 1)(8)
    assert lib.ucp_solve_batch(fake, 1, C.byref(P), C.byref(S), 1, its, arr, arr, arr, arr, None) == U.EINVAL
    assert lib.ucp_solve_batch(fake, 0, C.byref(P), C.byref(S), 1, its, arr, arr, arr, arr, None) == U.EINVAL


def test_coding_struct_and_argument_checks(U):
    # ucp_coding_problem: the fields of ucp_problem up to n_y, lam in place of
    # k, no noise_sd (its noise is U(-1, 1))
    assert C.sizeof(U.CodingProblem) == C.sizeof(U.Problem) - 8
    lib = U.library()
    fake = C.c_void_p(1)
    S = U.make_search(W.Search(-4, 4, 3, 9))
    good = W.coding_problem(101, 101)
    bad = []
    for field, val in [("lam", -1.0), ("lam", float("nan")), ("n_x", 1), ("n_y", 1), ("x_lo", 9.0),
                       ("y_hi", -6.0)]:
        p = W.coding_problem(101, 101)
        setattr(p, field, val)
        bad.append(p)
    p = W.coding_problem(101, 101)
    p.comps = [(0.5, 0.0, 1.0)]
    bad.append(p)
    v = C.c_void_p(8)
    for p in bad:
        P = U.make_coding_problem(p)
        assert lib.ucp_coding_objective(fake, C.byref(P), v, v, v, None) == U.EINVAL
        assert lib.ucp_coding_update_u1(fake, C.byref(P), v, v, None) == U.EINVAL
        assert lib.ucp_coding_argmin(fake, C.byref(P), C.byref(S), v, v, v, None, None) == U.EINVAL
        assert lib.ucp_coding_marginal_cost(fake, C.byref(P), v, v, 4, v, None) == U.EINVAL
        assert lib.ucp_coding_solve(fake, C.byref(P), C.byref(S), 2, v, v, v, v, None) == U.EINVAL
        assert U.last_error() != ""
    P = U.make_coding_problem(good)
    for s in [W.Search(4, -4, 3, 9), W.Search(-4, 4, 0, 9), W.Search(-4, 4, 3, 1), W.Search(-4, 4, 3, 64)]:
        S2 = U.make_search(s)
        assert lib.ucp_coding_argmin(fake, C.byref(P), C.byref(S2), v, v, v, None, None) == U.EINVAL
        assert lib.ucp_coding_solve(fake, C.byref(P), C.byref(S2), 2, v, v, v, v, None) == U.EINVAL
    assert lib.ucp_coding_argmin(fake, C.byref(P), None, v, v, v, None, None) == U.EINVAL
    assert lib.ucp_coding_solve(fake, C.byref(P), C.byref(S), -1, v, v, v, v, None) == U.EINVAL
    assert lib.ucp_coding_solve(fake, C.byref(P), C.byref(S), 2, v, None, v, v, None) == U.EINVAL
    assert lib.ucp_coding_marginal_cost(fake, C.byref(P), v, v, 0, v, None) == U.EINVAL
    assert lib.ucp_coding_update_u1(fake, C.byref(P), None, v, None) == U.EINVAL
    assert lib.ucp_coding_objective(None, C.byref(P), v, v, v, None) == U.EINVAL


def test_w2_argument_checks(U):
    lib = U.library()
    fake = C.c_void_p(1)
    v = C.c_void_p(8)
    P = U.make_problem(W.w2_problem(21, 31))
    S = U.make_search(W.Search(-30, 30, 3, 5))
    big = U.make_problem(W.w2_problem(4097, 31))
    for Pb in (big, U.make_problem(W.gaussian_problem(-1.0, 5.0, 21, 25.0))):
        assert lib.ucp_w2_objective(fake, C.byref(Pb), v, v, v, None) == U.EINVAL
        assert lib.ucp_w2_update_u1(fake, C.byref(Pb), v, v, None) == U.EINVAL
        assert lib.ucp_w2_marginal_cost(fake, C.byref(Pb), v, v, 2, v, None) == U.EINVAL
        assert lib.ucp_w2_argmin(fake, C.byref(Pb), C.byref(S), v, v, v, None, None) == U.EINVAL
        assert lib.ucp_w2_solve(fake, C.byref(Pb), C.byref(S), 1, v, v, v, v, None) == U.EINVAL
    S9 = U.make_search(W.Search(-30, 30, 3, 9))  # 9 x 9 candidates exceed one wave
    assert lib.ucp_w2_argmin(fake, C.byref(P), C.byref(S9), v, v, v, None, None) == U.EINVAL
    assert lib.ucp_w2_solve(fake, C.byref(P), C.byref(S), -1, v, v, v, v, None) == U.EINVAL
    assert lib.ucp_w2_solve(fake, C.byref(P), None, 1, v, v, v, v, None) == U.EINVAL
    assert lib.ucp_w2_marginal_cost(fake, C.byref(P), v, v, 0, v, None) == U.EINVAL
    assert lib.ucp_w2_objective(None, C.byref(P), v, v, v, None) == U.EINVAL


def test_footprint_without_device(U):
    c = W.small_case()
    n = U.footprint(c.prob, c.search, 10)
    n2 = U.footprint(W.paper_res_case().prob, W.paper_res_case().search, 30)
    assert 100_000 < n < n2 < 1 << 30
    with pytest.raises(U.UcpError):
        U.footprint(c.prob, W.Search(1, -1, 3, 21), 10)


def test_server_rejects_without_device(U):
    lib = U.library()
    s = C.c_void_p()
    assert lib.ucp_server_create(None, 0, 0, 4, 1) == U.EINVAL
    assert lib.ucp_server_create(C.byref(s), 0, 0, 0, 1) == U.EINVAL
    assert lib.ucp_server_create(C.byref(s), 0, 0, 4, 9) == U.EINVAL
    rc = lib.ucp_server_create(C.byref(s), 0, 0, 4, 1)
    assert rc in (U.EHIP, U.OK)
    if rc == U.OK:
        lib.ucp_server_destroy(s)
    assert lib.ucp_server_step(None, None) == U.EINVAL
    assert lib.ucp_server_poll(None, 1, None, None, None) == U.EINVAL


def test_no_oracle_in_product_path():
    """The product package never imports or loads the oracle."""
    pkg = os.path.join(ROOT, "paper_1908_04489_amd")
    for dp, _, fs in os.walk(pkg):
        for f in fs:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(dp, f)).read()
                assert "oracle" not in txt.replace("Oracle", "oracle").lower().replace("no cpu fallback", ""), f


def test_bench_reads_committed_traffic_only_for_its_kernel_source(tmp_path):
    """bench.py reports the HBM traffic of the PMC summary only while the
    summary's kernel-source hash matches (the hash key itself holds a colon)."""
    import bench

    p = tmp_path / "pmc-traffic_x.md"
    p.write_text("# HBM traffic\n\n- kernel source sha256[:16]: `0123456789abcdef`\n"
                 "- marginal-cost kernel HBM bytes per launch: 49956841\n")
    assert bench.parse_traffic(str(p), "0123456789abcdef") == 49956841.0
    assert bench.parse_traffic(str(p), "fedcba9876543210") is None
    assert bench.parse_traffic(str(tmp_path / "missing.md"), "0123456789abcdef") is None


def test_kernel_source_hash_covers_kernels_and_header(tmp_path, monkeypatch):
    """The traffic figure goes stale when either the kernels or the header
    holding their tile sizes and layouts changes."""
    import shutil

    import bench

    src = os.path.join(ROOT, "paper_1908_04489_amd", "csrc")
    dst = tmp_path / "paper_1908_04489_amd" / "csrc"
    dst.mkdir(parents=True)
    for name in ("ucp_kernels.hip", "ucp_internal.h"):
        shutil.copy(os.path.join(src, name), dst / name)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    for name in ("ucp_kernels.hip", "ucp_internal.h"):
        with open(dst / name, "a") as f:
            f.write("\n")
        h1 = bench.kernel_source_hash()
        assert h1 != h0, name
        h0 = h1
