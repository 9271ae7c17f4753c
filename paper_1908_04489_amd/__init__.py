"""Python binding of the MI355X marginal-cost solver (C ABI in include/ucp.h).

Argument marshalling only: every step of the solver runs in the HIP kernels
of ``libucp.so``.  PyTorch provides device memory (tensors) and the stream
(``torch.cuda.current_stream()``).  The library must be built first
(``paper_1908_04489_amd.build.build()``); importing this module without it
raises immediately - there is no CPU fallback.

Problem and search objects are duck-typed: ``k``, ``comps`` (sequence of
``(weight, mean, sd)``), ``x_lo``, ``x_hi``, ``n_x``, ``y_lo``, ``y_hi``,
``n_y``; and ``u_lo``, ``u_hi``, ``levels``, ``cands`` (optionally
``tie_rel64``, ``band_rel32``; 0 selects the library's defaults).
"""
from __future__ import annotations

import ctypes as C
import os
import re
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
# UCP_LIBRARY selects another build of the library (e.g. one compiled with different flags)
LIB_PATH = os.environ.get("UCP_LIBRARY") or os.path.join(HERE, "libucp.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "ucp.h")

FP32, FP32_KAHAN, FP64, FP64_GT = 0, 1, 2, 3
PRECS = {"fp32": FP32, "fp32_kahan": FP32_KAHAN, "kahan": FP32_KAHAN, "fp64": FP64, "fp64_gt": FP64_GT, "gt": FP64_GT}
OK, EINVAL, ENOMEM, EHIP, EAGAIN, ENONFINITE, ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
MAX_COMP = 8


class UcpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ucp error {code}: {msg}")
        self.code = code


class Problem(C.Structure):
    _fields_ = [
        ("k", C.c_double), ("n_comp", C.c_int32), ("pad_", C.c_int32),
        ("w", C.c_double * MAX_COMP), ("mu", C.c_double * MAX_COMP), ("sd", C.c_double * MAX_COMP),
        ("x_lo", C.c_double), ("x_hi", C.c_double), ("n_x", C.c_int64),
        ("y_lo", C.c_double), ("y_hi", C.c_double), ("n_y", C.c_int64),
        ("noise_sd", C.c_double),
    ]


class CodingProblem(C.Structure):
    _fields_ = [
        ("lam", C.c_double), ("n_comp", C.c_int32), ("pad_", C.c_int32),
        ("w", C.c_double * MAX_COMP), ("mu", C.c_double * MAX_COMP), ("sd", C.c_double * MAX_COMP),
        ("x_lo", C.c_double), ("x_hi", C.c_double), ("n_x", C.c_int64),
        ("y_lo", C.c_double), ("y_hi", C.c_double), ("n_y", C.c_int64),
    ]


class Alg1Params(C.Structure):
    _fields_ = [("N", C.c_int32), ("r", C.c_int32), ("p", C.c_double), ("tau", C.c_double),
                ("tie_rel64", C.c_double), ("max_rounds", C.c_int32), ("pad_", C.c_int32)]


class Search(C.Structure):
    _fields_ = [("u_lo", C.c_double), ("u_hi", C.c_double), ("levels", C.c_int32), ("cands", C.c_int32),
                ("tie_rel64", C.c_double), ("band_rel32", C.c_double)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_1908_04489_amd.build.build() "
                      "(the solver has no CPU fallback)")
# torch is loaded first so that its bundled HIP runtime (soname
# libamdhip64.so.7) is the one this library's dependency of that name
# binds to.  In the other order the library brings in the system runtime,
# torch then loads its own copy beside it (it asks for libamdhip64.so by
# file name), and the library's copy finds no device once torch's has
# initialised the GPU.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

_vp = C.c_void_p
_P = C.POINTER
_sigs = {
    "ucp_version": ([], C.c_char_p),
    "ucp_last_error": ([], C.c_char_p),
    "ucp_create": ([_P(_vp), C.c_int, C.c_size_t], C.c_int),
    "ucp_destroy": ([_vp], None),
    "ucp_marginal_cost": ([_vp, _P(Problem), C.c_int, _vp, _vp, C.c_int64, _vp, _vp], C.c_int),
    "ucp_argmin_adaptive": ([_vp, _P(Problem), _P(Search), C.c_int, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "ucp_argmin_adaptive_noalloc": ([_vp, _P(Problem), _P(Search), C.c_int, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "ucp_update_u1": ([_vp, _P(Problem), C.c_int, _vp, _vp, _vp], C.c_int),
    "ucp_alg1_local_u0": ([_vp, _P(Problem), C.c_double, _vp, _vp, _vp, _vp], C.c_int),
    "ucp_alg1_pe_u0": ([_vp, _P(Problem), C.c_double, C.c_int32, _vp, _vp, _vp, _vp], C.c_int),
    "ucp_alg1_pe_u1": ([_vp, _P(Problem), C.c_double, C.c_int32, _vp, _vp, _vp, _vp], C.c_int),
    "ucp_alg1_solve": ([_vp, _P(Problem), _vp, _vp, _vp, _vp, _vp, _vp, _P(C.c_int32), _P(C.c_int32), _vp],
                       C.c_int),
    "ucp_objective": ([_vp, _P(Problem), _vp, _vp, _vp, _vp], C.c_int),
    "ucp_solve": ([_vp, _P(Problem), _P(Search), C.c_int, C.c_int32, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "ucp_solve_batch": ([_vp, C.c_int32, _P(Problem), _P(Search), C.c_int, _P(C.c_int32), _P(_vp), _P(_vp),
                         _P(_vp), _P(_vp), _vp], C.c_int),
    "ucp_profile": ([_vp, C.c_int], C.c_int),
    "ucp_peak_probe": ([C.c_int, C.c_int, C.c_int32, C.c_int32, _P(C.c_double), _vp], C.c_int),
    "ucp_profile_read": ([_vp, C.c_int, _P(C.c_double), _P(C.c_int64)], C.c_int),
    "ucp_last_counts": ([_vp, _P(C.c_uint64), _P(C.c_uint64), _P(C.c_uint64)], C.c_int),
    "ucp_footprint": ([_P(Problem), _P(Search), C.c_int, C.c_int32, _P(C.c_size_t)], C.c_int),
    "ucp_coding_marginal_cost": ([_vp, _P(CodingProblem), _vp, _vp, C.c_int64, _vp, _vp], C.c_int),
    "ucp_coding_argmin": ([_vp, _P(CodingProblem), _P(Search), _vp, _vp, _vp, _vp, _vp], C.c_int),
    "ucp_coding_update_u1": ([_vp, _P(CodingProblem), _vp, _vp, _vp], C.c_int),
    "ucp_coding_objective": ([_vp, _P(CodingProblem), _vp, _vp, _vp, _vp], C.c_int),
    "ucp_coding_solve": ([_vp, _P(CodingProblem), _P(Search), C.c_int32, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "ucp_w2_marginal_cost": ([_vp, _P(Problem), _vp, _vp, C.c_int64, _vp, _vp], C.c_int),
    "ucp_w2_argmin": ([_vp, _P(Problem), _P(Search), _vp, _vp, _vp, _vp, _vp], C.c_int),
    "ucp_w2_update_u1": ([_vp, _P(Problem), _vp, _vp, _vp], C.c_int),
    "ucp_w2_objective": ([_vp, _P(Problem), _vp, _vp, _vp, _vp], C.c_int),
    "ucp_w2_solve": ([_vp, _P(Problem), _P(Search), C.c_int32, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "ucp_server_create": ([_P(_vp), C.c_int, C.c_size_t, C.c_int32, C.c_int], C.c_int),
    "ucp_server_destroy": ([_vp], None),
    "ucp_server_submit": ([_vp, _P(Problem), _P(Search), C.c_int32, _vp, _P(C.c_int64)], C.c_int),
    "ucp_server_step": ([_vp, _P(C.c_int32)], C.c_int),
    "ucp_server_poll": ([_vp, C.c_int64, _vp, _vp, _vp], C.c_int),
    "ucp_server_cancel": ([_vp, C.c_int64], C.c_int),
    "ucp_server_stats": ([_vp, _P(C.c_int32), _P(C.c_int32), _P(C.c_int32)], C.c_int),
}
for _name, (_args, _res) in _sigs.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


def header_functions():
    """Names of the functions declared in include/ucp.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]*?\b(ucp_\w+)\s*\(", txt, re.M)))


def library():
    return _lib


def last_error() -> str:
    return _lib.ucp_last_error().decode()


def _check(rc):
    if rc != OK:
        raise UcpError(rc, last_error())
    return rc


def make_problem(p) -> Problem:
    comps = list(p.comps)
    s = Problem()
    s.k = float(p.k)
    s.n_comp = len(comps)
    for c, (w, mu, sd) in enumerate(comps):
        s.w[c], s.mu[c], s.sd[c] = float(w), float(mu), float(sd)
    s.x_lo, s.x_hi, s.n_x = float(p.x_lo), float(p.x_hi), int(p.n_x)
    s.y_lo, s.y_hi, s.n_y = float(p.y_lo), float(p.y_hi), int(p.n_y)
    s.noise_sd = float(getattr(p, "noise_sd", 1.0))
    return s


def make_search(s) -> Search:
    r = Search()
    r.u_lo, r.u_hi, r.levels, r.cands = float(s.u_lo), float(s.u_hi), int(s.levels), int(s.cands)
    r.tie_rel64 = float(getattr(s, "tie_rel64", 0.0))
    r.band_rel32 = float(getattr(s, "band_rel32", 0.0))
    return r


def _prec(prec) -> int:
    if isinstance(prec, str):
        return PRECS[prec.lower()]
    return int(prec)


# ------------------------------------------------------------ torch plumbing

def _torch():
    import torch

    return torch


def _dev_f64(t, n, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float64")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, has {t.numel()}")
    return t


def _stream(device):
    torch = _torch()
    return _vp(torch.cuda.current_stream(device).cuda_stream)


_handles = threading.local()


def handle(device: int = 0):
    """Per-thread, per-device library handle."""
    d = getattr(_handles, "d", None)
    if d is None:
        d = _handles.d = {}
    if device not in d:
        h = _vp()
        _check(_lib.ucp_create(C.byref(h), int(device), 0))
        d[device] = h
    return d[device]


def _dev(t):
    return t.device.index if t.device.index is not None else 0


def marginal_cost(prob, u1, u, prec="fp32_kahan"):
    """L_0 = f(x_i) B(u; x_i) for candidates u [n_x, n_cand] (device, FP64)."""
    torch = _torch()
    P = make_problem(prob)
    _dev_f64(u1, P.n_y, "u1")
    _dev_f64(u, None, "u")
    if u.dim() != 2 or u.shape[0] != P.n_x:
        raise ValueError("u must be [n_x, n_cand]")
    out = torch.empty_like(u)
    d = _dev(u1)
    _check(_lib.ucp_marginal_cost(handle(d), C.byref(P), _prec(prec), _vp(u1.data_ptr()), _vp(u.data_ptr()),
                                  u.shape[1], _vp(out.data_ptr()), _stream(d)))
    return out


def argmin_adaptive(prob, search, u1, u0, prec="fp32_kahan", want_l0=False):
    """One coarse-to-fine u0 update with u1 fixed.  Returns u0_out (and L0)."""
    torch = _torch()
    P, S = make_problem(prob), make_search(search)
    _dev_f64(u1, P.n_y, "u1")
    _dev_f64(u0, P.n_x, "u0")
    out = torch.empty_like(u0)
    l0 = torch.empty_like(u0) if want_l0 else None
    d = _dev(u0)
    _check(_lib.ucp_argmin_adaptive(handle(d), C.byref(P), C.byref(S), _prec(prec), _vp(u1.data_ptr()),
                                    _vp(u0.data_ptr()), _vp(out.data_ptr()),
                                    _vp(l0.data_ptr() if l0 is not None else 0), _stream(d)))
    return (out, l0) if want_l0 else out


def argmin_adaptive_noalloc(prob, search, u1, u0, out, l0=None, prec="fp32_kahan"):
    """ucp_argmin_adaptive_noalloc: the u0 update into the caller's tensors
    ``out`` (and ``l0``), with the library's fixed scratch array; nothing is
    allocated by the library."""
    P, S = make_problem(prob), make_search(search)
    _dev_f64(u1, P.n_y, "u1")
    _dev_f64(u0, P.n_x, "u0")
    _dev_f64(out, P.n_x, "out")
    if l0 is not None:
        _dev_f64(l0, P.n_x, "l0")
    d = _dev(u0)
    _check(_lib.ucp_argmin_adaptive_noalloc(handle(d), C.byref(P), C.byref(S), _prec(prec), _vp(u1.data_ptr()),
                                            _vp(u0.data_ptr()), _vp(out.data_ptr()),
                                            _vp(l0.data_ptr() if l0 is not None else 0), _stream(d)))
    return out


def update_u1(prob, u0, prec="fp32_kahan"):
    torch = _torch()
    P = make_problem(prob)
    _dev_f64(u0, P.n_x, "u0")
    out = torch.empty(P.n_y, dtype=torch.float64, device=u0.device)
    d = _dev(u0)
    _check(_lib.ucp_update_u1(handle(d), C.byref(P), _prec(prec), _vp(u0.data_ptr()), _vp(out.data_ptr()),
                              _stream(d)))
    return out


def objective(prob, u0, u1):
    """J as a 1-element device tensor (FP64)."""
    torch = _torch()
    P = make_problem(prob)
    _dev_f64(u0, P.n_x, "u0")
    _dev_f64(u1, P.n_y, "u1")
    out = torch.empty(1, dtype=torch.float64, device=u0.device)
    d = _dev(u0)
    _check(_lib.ucp_objective(handle(d), C.byref(P), _vp(u0.data_ptr()), _vp(u1.data_ptr()),
                              _vp(out.data_ptr()), _stream(d)))
    return out


def solve(prob, search, iters, u0_init, prec="fp32_kahan"):
    """Returns (u0, u1, J_hist[iters + 1]) as device tensors."""
    torch = _torch()
    P, S = make_problem(prob), make_search(search)
    _dev_f64(u0_init, P.n_x, "u0_init")
    dev = u0_init.device
    u0 = torch.empty(P.n_x, dtype=torch.float64, device=dev)
    u1 = torch.empty(P.n_y, dtype=torch.float64, device=dev)
    J = torch.empty(int(iters) + 1, dtype=torch.float64, device=dev)
    d = _dev(u0_init)
    _check(_lib.ucp_solve(handle(d), C.byref(P), C.byref(S), _prec(prec), int(iters), _vp(u0_init.data_ptr()),
                          _vp(u0.data_ptr()), _vp(u1.data_ptr()), _vp(J.data_ptr()), _stream(d)))
    return u0, u1, J


def solve_batch(probs, searches, iters, u0_inits, prec="fp32_kahan"):
    """Independent solves in shared launches.  Returns lists (u0, u1, J)."""
    torch = _torch()
    B = len(probs)
    Ps = (Problem * B)(*[make_problem(p) for p in probs])
    Ss = (Search * B)(*[make_search(s) for s in searches])
    its = (C.c_int32 * B)(*[int(t) for t in iters])
    u0o, u1o, Jo = [], [], []
    for b in range(B):
        _dev_f64(u0_inits[b], Ps[b].n_x, f"u0_init[{b}]")
        dev = u0_inits[b].device
        u0o.append(torch.empty(Ps[b].n_x, dtype=torch.float64, device=dev))
        u1o.append(torch.empty(Ps[b].n_y, dtype=torch.float64, device=dev))
        Jo.append(torch.empty(int(iters[b]) + 1, dtype=torch.float64, device=dev))

    def ptrs(ts):
        return (_vp * B)(*[t.data_ptr() for t in ts])

    d = _dev(u0_inits[0])
    _check(_lib.ucp_solve_batch(handle(d), B, Ps, Ss, _prec(prec), its, ptrs(u0_inits), ptrs(u0o), ptrs(u1o),
                                ptrs(Jo), _stream(d)))
    return u0o, u1o, Jo


PROF_KINDS = {"marginal_cost": 0, "select": 1, "u1": 2, "objective": 3}


def profile(kinds=None, device: int = 0):
    """Set per-kernel HIP-event timing of solves (resets totals): ``kinds`` is
    an iterable of names from PROF_KINDS, True for all, and None/False/empty
    for off."""
    if kinds is True:
        mask = (1 << len(PROF_KINDS)) - 1
    elif not kinds:
        mask = 0
    else:
        mask = 0
        for k in kinds:
            mask |= 1 << PROF_KINDS[k]
    _check(_lib.ucp_profile(handle(device), mask))


def profile_read(device: int = 0):
    """{kind: (total_ms, launches)} accumulated since profiling was switched on."""
    out = {}
    for name, k in PROF_KINDS.items():
        ms, n = C.c_double(), C.c_int64()
        _check(_lib.ucp_profile_read(handle(device), k, C.byref(ms), C.byref(n)))
        out[name] = (ms.value, n.value)
    return out


def last_counts(device: int = 0):
    """(algorithmic marginal-cost terms, terms evaluated, FP64 tie
    re-evaluations) of the last solve on this thread's handle."""
    n, v, e = C.c_uint64(), C.c_uint64(), C.c_uint64()
    _check(_lib.ucp_last_counts(handle(device), C.byref(n), C.byref(v), C.byref(e)))
    return n.value, v.value, e.value


def footprint(prob, search, iters, prec="fp32_kahan") -> int:
    """Device bytes of one solve (the server's admission footprint)."""
    P, S = make_problem(prob), make_search(search)
    n = C.c_size_t()
    _check(_lib.ucp_footprint(C.byref(P), C.byref(S), _prec(prec), int(iters), C.byref(n)))
    return n.value


class Server:
    """Continuous-batching server (host arrays in and out)."""

    def __init__(self, device=0, hbm_budget=0, max_slots=64, prec="fp32_kahan"):
        self._s = _vp()
        _check(_lib.ucp_server_create(C.byref(self._s), int(device), int(hbm_budget), int(max_slots),
                                      _prec(prec)))
        self._meta = {}

    def close(self):
        if self._s:
            _lib.ucp_server_destroy(self._s)
            self._s = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, prob, search, iters, u0_init) -> int:
        import numpy as np

        P, S = make_problem(prob), make_search(search)
        a = np.ascontiguousarray(u0_init, dtype=np.float64)
        if a.shape != (P.n_x,):
            raise ValueError("u0_init must be [n_x]")
        t = C.c_int64()
        _check(_lib.ucp_server_submit(self._s, C.byref(P), C.byref(S), int(iters), _vp(a.ctypes.data),
                                      C.byref(t)))
        self._meta[t.value] = (int(P.n_x), int(P.n_y), int(iters))
        return t.value

    def step(self) -> int:
        n = C.c_int32()
        _check(_lib.ucp_server_step(self._s, C.byref(n)))
        return n.value

    def poll(self, ticket):
        """(u0, u1, J) numpy arrays when done, None while queued/running."""
        import numpy as np

        nx, ny, it = self._meta[ticket]
        u0 = np.empty(nx)
        u1 = np.empty(ny)
        J = np.empty(it + 1)
        rc = _lib.ucp_server_poll(self._s, int(ticket), _vp(u0.ctypes.data), _vp(u1.ctypes.data),
                                  _vp(J.ctypes.data))
        if rc == EAGAIN:
            return None
        if rc == ENONFINITE:
            del self._meta[ticket]
            raise UcpError(rc, last_error())
        _check(rc)
        del self._meta[ticket]
        return u0, u1, J

    def cancel(self, ticket):
        _check(_lib.ucp_server_cancel(self._s, int(ticket)))

    def stats(self):
        q, r, d = C.c_int32(), C.c_int32(), C.c_int32()
        _check(_lib.ucp_server_stats(self._s, C.byref(q), C.byref(r), C.byref(d)))
        return q.value, r.value, d.value


# ------------------------------------------- source-channel coding (Section V-B)

def make_coding_problem(p) -> CodingProblem:
    """From a duck-typed problem with ``lam`` (weight of the encoder's power)
    and the fields of ``make_problem`` other than ``k``."""
    comps = list(p.comps)
    s = CodingProblem()
    s.lam = float(p.lam)
    s.n_comp = len(comps)
    for c, (w, mu, sd) in enumerate(comps):
        s.w[c], s.mu[c], s.sd[c] = float(w), float(mu), float(sd)
    s.x_lo, s.x_hi, s.n_x = float(p.x_lo), float(p.x_hi), int(p.n_x)
    s.y_lo, s.y_hi, s.n_y = float(p.y_lo), float(p.y_hi), int(p.n_y)
    return s


def coding_marginal_cost(prob, u1, u):
    """L_0 = f(x_i) B(u; x_i) for candidates u [n_x, n_cand] (device, FP64)."""
    torch = _torch()
    P = make_coding_problem(prob)
    _dev_f64(u1, P.n_y, "u1")
    _dev_f64(u, None, "u")
    if u.dim() != 2 or u.shape[0] != P.n_x:
        raise ValueError("u must be [n_x, n_cand]")
    out = torch.empty_like(u)
    d = _dev(u1)
    _check(_lib.ucp_coding_marginal_cost(handle(d), C.byref(P), _vp(u1.data_ptr()), _vp(u.data_ptr()),
                                         u.shape[1], _vp(out.data_ptr()), _stream(d)))
    return out


def coding_argmin(prob, search, u1, u0, want_l0=False):
    """One coarse-to-fine encoder update with u1 fixed.  Returns u0_out (and L0)."""
    torch = _torch()
    P, S = make_coding_problem(prob), make_search(search)
    _dev_f64(u1, P.n_y, "u1")
    _dev_f64(u0, P.n_x, "u0")
    out = torch.empty_like(u0)
    l0 = torch.empty_like(u0) if want_l0 else None
    d = _dev(u0)
    _check(_lib.ucp_coding_argmin(handle(d), C.byref(P), C.byref(S), _vp(u1.data_ptr()), _vp(u0.data_ptr()),
                                  _vp(out.data_ptr()), _vp(l0.data_ptr() if l0 is not None else 0),
                                  _stream(d)))
    return (out, l0) if want_l0 else out


def coding_update_u1(prob, u0):
    torch = _torch()
    P = make_coding_problem(prob)
    _dev_f64(u0, P.n_x, "u0")
    out = torch.empty(P.n_y, dtype=torch.float64, device=u0.device)
    d = _dev(u0)
    _check(_lib.ucp_coding_update_u1(handle(d), C.byref(P), _vp(u0.data_ptr()), _vp(out.data_ptr()),
                                     _stream(d)))
    return out


def coding_objective(prob, u0, u1):
    """J as a 1-element device tensor (FP64)."""
    torch = _torch()
    P = make_coding_problem(prob)
    _dev_f64(u0, P.n_x, "u0")
    _dev_f64(u1, P.n_y, "u1")
    out = torch.empty(1, dtype=torch.float64, device=u0.device)
    d = _dev(u0)
    _check(_lib.ucp_coding_objective(handle(d), C.byref(P), _vp(u0.data_ptr()), _vp(u1.data_ptr()),
                                     _vp(out.data_ptr()), _stream(d)))
    return out


def coding_solve(prob, search, iters, u0_init):
    """Returns (u0, u1, J_hist[iters + 1]) as device tensors."""
    torch = _torch()
    P, S = make_coding_problem(prob), make_search(search)
    _dev_f64(u0_init, P.n_x, "u0_init")
    dev = u0_init.device
    u0 = torch.empty(P.n_x, dtype=torch.float64, device=dev)
    u1 = torch.empty(P.n_y, dtype=torch.float64, device=dev)
    J = torch.empty(int(iters) + 1, dtype=torch.float64, device=dev)
    d = _dev(u0_init)
    _check(_lib.ucp_coding_solve(handle(d), C.byref(P), C.byref(S), int(iters), _vp(u0_init.data_ptr()),
                                 _vp(u0.data_ptr()), _vp(u1.data_ptr()), _vp(J.data_ptr()), _stream(d)))
    return u0, u1, J


# ------------------------------------ two-dimensional Witsenhausen (Section V-D)
# Vector fields are device tensors [2, n * n] (node (i1, i2) at i1 * n + i2).

def _dev_planes(t, n, name):
    _dev_f64(t, 2 * n, name)
    if t.dim() != 2 or t.shape[0] != 2:
        raise ValueError(f"{name} must be [2, {n}]")
    return t


def w2_marginal_cost(prob, u1, u):
    """L_0 [n_x^2, n_cand] for candidates u [2, n_x^2, n_cand]."""
    torch = _torch()
    P = make_problem(prob)
    _dev_planes(u1, P.n_y ** 2, "u1")
    _dev_f64(u, None, "u")
    if u.dim() != 3 or u.shape[0] != 2 or u.shape[1] != P.n_x ** 2:
        raise ValueError("u must be [2, n_x^2, n_cand]")
    out = torch.empty(u.shape[1], u.shape[2], dtype=torch.float64, device=u.device)
    d = _dev(u1)
    _check(_lib.ucp_w2_marginal_cost(handle(d), C.byref(P), _vp(u1.data_ptr()), _vp(u.data_ptr()), u.shape[2],
                                     _vp(out.data_ptr()), _stream(d)))
    return out


def w2_argmin(prob, search, u1, u0, want_l0=False):
    torch = _torch()
    P, S = make_problem(prob), make_search(search)
    _dev_planes(u1, P.n_y ** 2, "u1")
    _dev_planes(u0, P.n_x ** 2, "u0")
    out = torch.empty_like(u0)
    l0 = torch.empty(P.n_x ** 2, dtype=torch.float64, device=u0.device) if want_l0 else None
    d = _dev(u0)
    _check(_lib.ucp_w2_argmin(handle(d), C.byref(P), C.byref(S), _vp(u1.data_ptr()), _vp(u0.data_ptr()),
                              _vp(out.data_ptr()), _vp(l0.data_ptr() if l0 is not None else 0), _stream(d)))
    return (out, l0) if want_l0 else out


def w2_update_u1(prob, u0):
    torch = _torch()
    P = make_problem(prob)
    _dev_planes(u0, P.n_x ** 2, "u0")
    out = torch.empty(2, P.n_y ** 2, dtype=torch.float64, device=u0.device)
    d = _dev(u0)
    _check(_lib.ucp_w2_update_u1(handle(d), C.byref(P), _vp(u0.data_ptr()), _vp(out.data_ptr()), _stream(d)))
    return out


def w2_objective(prob, u0, u1):
    torch = _torch()
    P = make_problem(prob)
    _dev_planes(u0, P.n_x ** 2, "u0")
    _dev_planes(u1, P.n_y ** 2, "u1")
    out = torch.empty(1, dtype=torch.float64, device=u0.device)
    d = _dev(u0)
    _check(_lib.ucp_w2_objective(handle(d), C.byref(P), _vp(u0.data_ptr()), _vp(u1.data_ptr()),
                                 _vp(out.data_ptr()), _stream(d)))
    return out


def w2_solve(prob, search, iters, u0_init):
    """Returns (u0 [2, n_x^2], u1 [2, n_y^2], J_hist[iters + 1]) as device tensors."""
    torch = _torch()
    P, S = make_problem(prob), make_search(search)
    _dev_planes(u0_init, P.n_x ** 2, "u0_init")
    dev = u0_init.device
    u0 = torch.empty(2, P.n_x ** 2, dtype=torch.float64, device=dev)
    u1 = torch.empty(2, P.n_y ** 2, dtype=torch.float64, device=dev)
    J = torch.empty(int(iters) + 1, dtype=torch.float64, device=dev)
    d = _dev(u0_init)
    _check(_lib.ucp_w2_solve(handle(d), C.byref(P), C.byref(S), int(iters), _vp(u0_init.data_ptr()),
                             _vp(u0.data_ptr()), _vp(u1.data_ptr()), _vp(J.data_ptr()), _stream(d)))
    return u0, u1, J


# ------------------------------------------------------------------
# The paper's generic solver (Algorithm 1).

def alg1_local_u0(prob, tau, u1, u0):
    torch = _torch()
    P = make_problem(prob)
    _dev_f64(u1, P.n_y, "u1")
    _dev_f64(u0, P.n_x, "u0")
    out = torch.empty_like(u0)
    d = _dev(u0)
    _check(_lib.ucp_alg1_local_u0(handle(d), C.byref(P), float(tau), _vp(u1.data_ptr()), _vp(u0.data_ptr()),
                                  _vp(out.data_ptr()), _stream(d)))
    return out


def alg1_pe_u0(prob, u1, u0, r=2, tie=0.0):
    torch = _torch()
    P = make_problem(prob)
    _dev_f64(u1, P.n_y, "u1")
    _dev_f64(u0, P.n_x, "u0")
    out = torch.empty_like(u0)
    d = _dev(u0)
    _check(_lib.ucp_alg1_pe_u0(handle(d), C.byref(P), float(tie), int(r), _vp(u1.data_ptr()), _vp(u0.data_ptr()),
                               _vp(out.data_ptr()), _stream(d)))
    return out


def alg1_pe_u1(prob, u0, u1, r=2, tie=0.0):
    torch = _torch()
    P = make_problem(prob)
    _dev_f64(u0, P.n_x, "u0")
    _dev_f64(u1, P.n_y, "u1")
    out = torch.empty_like(u1)
    d = _dev(u0)
    _check(_lib.ucp_alg1_pe_u1(handle(d), C.byref(P), float(tie), int(r), _vp(u0.data_ptr()), _vp(u1.data_ptr()),
                               _vp(out.data_ptr()), _stream(d)))
    return out


def alg1_solve(prob, u0_init, u1_init, N=20, r=2, prec=1e-10, tau=0.1, tie=0.0, max_rounds=100):
    """Returns (u0, u1, J_log[1 + 2 rounds] as a device tensor, NL_log as a list)."""
    torch = _torch()
    P = make_problem(prob)
    _dev_f64(u0_init, P.n_x, "u0_init")
    _dev_f64(u1_init, P.n_y, "u1_init")
    a = Alg1Params()
    a.N, a.r, a.p, a.tau, a.tie_rel64, a.max_rounds = int(N), int(r), float(prec), float(tau), float(tie), \
        int(max_rounds)
    dev = u0_init.device
    u0 = torch.empty(P.n_x, dtype=torch.float64, device=dev)
    u1 = torch.empty(P.n_y, dtype=torch.float64, device=dev)
    J = torch.empty(1 + 2 * int(max_rounds), dtype=torch.float64, device=dev)
    NL = (C.c_int32 * int(max_rounds))()
    rounds = C.c_int32()
    d = _dev(u0_init)
    _check(_lib.ucp_alg1_solve(handle(d), C.byref(P), C.byref(a), _vp(u0_init.data_ptr()), _vp(u1_init.data_ptr()),
                               _vp(u0.data_ptr()), _vp(u1.data_ptr()), _vp(J.data_ptr()), NL, C.byref(rounds),
                               _stream(d)))
    n = rounds.value
    return u0, u1, J[:1 + 2 * n], list(NL[:n])


def peak_probe(kind, blocks=8192, iters=4096, device=0):
    """Lane-operations per second of one VALU operation: "fma32", "exp32" or
    "fma64" (diagnostic; fixes the peak of the roofline)."""
    k = {"fma32": 0, "exp32": 1, "fma64": 2}[kind]
    out = C.c_double()
    _check(_lib.ucp_peak_probe(int(device), k, int(blocks), int(iters), C.byref(out), _stream(device)))
    return out.value
