"""FP64 CPU oracle for the marginal-cost solver (Witsenhausen instance).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The product
path (``paper_1908_04489_amd``) never does, and this package imports nothing
from it.

The arithmetic lives in ``ucp_oracle.c`` (plain C, FP64, dense sums in index
order).  This module compiles it with gcc and exposes it through ctypes on
numpy arrays.  ``mp_oracle.py`` holds an independent arbitrary-precision
brute force for tiny grids.

Problem objects are duck-typed: any object with ``k`` (``lam`` for the
coding problem of Section V-B, the ``coding_*`` functions), ``comps`` (a sequence
of ``(weight, mean, sd)`` for the Gaussian-mixture prior of x0), ``x_lo``,
``x_hi``, ``n_x``, ``y_lo``, ``y_hi``, ``n_y`` and optionally ``noise_sd`` (the
standard deviation of the Gaussian noise, 1 by default).  Search objects need
``u_lo``, ``u_hi``, ``levels``, ``cands`` and may carry ``tie_rel64`` (the
relative tie band of the selection rule, 0 = 1e-12).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ucp_oracle.c")
_LIB = os.path.join(_HERE, "_ucp_oracle.so")
MAX_COMP = 8
TAU64 = 1e-12


class _Problem(C.Structure):
    _fields_ = [
        ("k", C.c_double),
        ("n_comp", C.c_int32),
        ("pad_", C.c_int32),
        ("w", C.c_double * MAX_COMP),
        ("mu", C.c_double * MAX_COMP),
        ("sd", C.c_double * MAX_COMP),
        ("x_lo", C.c_double),
        ("x_hi", C.c_double),
        ("n_x", C.c_int64),
        ("y_lo", C.c_double),
        ("y_hi", C.c_double),
        ("n_y", C.c_int64),
        ("noise_sd", C.c_double),
    ]


class _Search(C.Structure):
    _fields_ = [
        ("u_lo", C.c_double),
        ("u_hi", C.c_double),
        ("levels", C.c_int32),
        ("cands", C.c_int32),
        ("tie_rel64", C.c_double),
        ("band_rel32", C.c_double),
    ]


class _Alg1(C.Structure):
    _fields_ = [
        ("N", C.c_int32),
        ("r", C.c_int32),
        ("p", C.c_double),
        ("tau", C.c_double),
        ("tie_rel64", C.c_double),
        ("max_rounds", C.c_int32),
        ("pad_", C.c_int32),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/_ucp_oracle.so`` (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = [
            "gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
            "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm",
        ]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        P = C.POINTER
        dp = P(C.c_double)
        ip = P(C.c_int64)
        D = C.c_double
        L.orc_num_threads.restype = C.c_int
        L.orc_grid.argtypes = [C.c_double, C.c_double, C.c_int64, dp]
        L.orc_prior.argtypes = [P(_Problem), dp, dp]
        L.orc_B.argtypes = [P(_Problem), dp, C.c_double, C.c_double]
        L.orc_B.restype = C.c_double
        L.orc_marginal_cost.argtypes = [P(_Problem), dp, dp, C.c_int64, dp]
        L.orc_spacings.argtypes = [P(_Search), dp]
        L.orc_argmin.argtypes = [P(_Problem), P(_Search), dp, dp, ip, C.c_int64, dp, dp]
        L.orc_argmin_visits.argtypes = [P(_Problem), P(_Search), dp, dp, ip, C.c_int64, dp, dp]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_update_u1.argtypes = [P(_Problem), dp, ip, C.c_int64, dp]
        L.orc_B_derivs.argtypes = [P(_Problem), dp, D, D, dp, dp, dp]
        L.orc_alg1_local_u0.argtypes = [P(_Problem), D, dp, dp, ip, C.c_int64, dp]
        L.orc_alg1_local_u1.argtypes = [P(_Problem), dp, dp, ip, C.c_int64, dp]
        L.orc_alg1_pe_u0.argtypes = [P(_Problem), D, C.c_int32, dp, dp, ip, C.c_int64, dp]
        L.orc_alg1_pe_u1.argtypes = [P(_Problem), D, C.c_int32, dp, dp, ip, C.c_int64, dp]
        L.orc_alg1_allocate.argtypes = [C.c_int32, D, D, P(C.c_int32), P(C.c_int32)]
        L.orc_alg1_solve.argtypes = [P(_Problem), P(_Alg1), dp, dp, dp, dp, dp, P(C.c_int32)]
        L.orc_alg1_solve.restype = C.c_int32
        L.orc_objective.argtypes = [P(_Problem), dp, dp]
        L.orc_objective.restype = C.c_double
        L.orc_solve.argtypes = [P(_Problem), P(_Search), C.c_int32, dp, dp, dp, dp]
        L.orc_cd_B.argtypes = [P(_Problem), D, dp, D, D]
        L.orc_cd_B.restype = D
        L.orc_cd_marginal_cost.argtypes = [P(_Problem), D, dp, dp, C.c_int64, dp]
        L.orc_cd_argmin.argtypes = [P(_Problem), D, P(_Search), dp, dp, ip, C.c_int64, dp, dp]
        L.orc_cd_update_u1.argtypes = [P(_Problem), dp, ip, C.c_int64, dp]
        L.orc_cd_objective.argtypes = [P(_Problem), D, dp, dp]
        L.orc_cd_objective.restype = D
        L.orc_cd_solve.argtypes = [P(_Problem), D, P(_Search), C.c_int32, dp, dp, dp, dp]
        L.orc2_B.argtypes = [P(_Problem), dp, D, D, D, D]
        L.orc2_B.restype = D
        L.orc2_marginal_cost.argtypes = [P(_Problem), dp, dp, C.c_int64, dp]
        L.orc2_argmin.argtypes = [P(_Problem), P(_Search), dp, dp, ip, C.c_int64, dp, dp]
        L.orc2_update_u1.argtypes = [P(_Problem), dp, ip, C.c_int64, dp]
        L.orc2_objective.argtypes = [P(_Problem), dp, dp]
        L.orc2_objective.restype = D
        L.orc2_solve.argtypes = [P(_Problem), P(_Search), C.c_int32, dp, dp, dp, dp]
        _lib = L
    return _lib


def _prob(p) -> _Problem:
    comps = list(p.comps)
    if not 1 <= len(comps) <= MAX_COMP:
        raise ValueError("prior must have 1..8 components")
    s = _Problem()
    s.k = float(getattr(p, "k", 0.0))
    s.n_comp = len(comps)
    for c, (w, mu, sd) in enumerate(comps):
        s.w[c], s.mu[c], s.sd[c] = float(w), float(mu), float(sd)
    s.x_lo, s.x_hi, s.n_x = float(p.x_lo), float(p.x_hi), int(p.n_x)
    s.y_lo, s.y_hi, s.n_y = float(p.y_lo), float(p.y_hi), int(p.n_y)
    s.noise_sd = float(getattr(p, "noise_sd", 1.0))
    return s


def _search(s) -> _Search:
    r = _Search()
    r.u_lo, r.u_hi = float(s.u_lo), float(s.u_hi)
    r.levels, r.cands = int(s.levels), int(s.cands)
    r.tie_rel64 = float(getattr(s, "tie_rel64", 0.0))
    r.band_rel32 = float(getattr(s, "band_rel32", 0.0))
    return r


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.shape != (n,):
        raise ValueError(f"expected shape ({n},), got {a.shape}")
    return a


def num_threads() -> int:
    return int(lib().orc_num_threads())


def grid(lo: float, hi: float, n: int) -> np.ndarray:
    out = np.empty(int(n), np.float64)
    lib().orc_grid(float(lo), float(hi), int(n), _dp(out))
    return out


def prior(p):
    """(f, log f) at the x-grid nodes."""
    f = np.empty(int(p.n_x), np.float64)
    lf = np.empty(int(p.n_x), np.float64)
    lib().orc_prior(C.byref(_prob(p)), _dp(f), _dp(lf))
    return f, lf


def B(p, u1, x: float, u: float) -> float:
    """B(u; x) = L_0(u, x) / f(x) for one point and one candidate."""
    u1 = _f64(u1, int(p.n_y))
    return float(lib().orc_B(C.byref(_prob(p)), _dp(u1), float(x), float(u)))


def marginal_cost(p, u1, u) -> np.ndarray:
    """L_0 = f_i B(u; x_i) for candidates u of shape [n_x, n_cand]."""
    u1 = _f64(u1, int(p.n_y))
    u = np.ascontiguousarray(u, dtype=np.float64)
    if u.ndim != 2 or u.shape[0] != int(p.n_x):
        raise ValueError("u must be [n_x, n_cand]")
    out = np.empty_like(u)
    lib().orc_marginal_cost(C.byref(_prob(p)), _dp(u1), _dp(u), u.shape[1], _dp(out))
    return out


def spacings(s) -> np.ndarray:
    h = np.empty(int(s.levels), np.float64)
    lib().orc_spacings(C.byref(_search(s)), _dp(h))
    return h


def argmin(p, s, u1, u0_in, rows=None):
    """One coarse-to-fine u0 update.  Returns (u0_out, B_out) for the listed
    rows (all rows when ``rows`` is None)."""
    u1 = _f64(u1, int(p.n_y))
    u0_in = _f64(u0_in, int(p.n_x))
    if rows is None:
        n = int(p.n_x)
        rp = None
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        if rows.size and (rows.min() < 0 or rows.max() >= int(p.n_x)):
            raise ValueError("row index out of range")
        n = rows.size
        rp = rows.ctypes.data_as(C.POINTER(C.c_int64))
    u0o = np.empty(n, np.float64)
    Bo = np.empty(n, np.float64)
    lib().orc_argmin(C.byref(_prob(p)), C.byref(_search(s)), _dp(u1), _dp(u0_in),
                     rp, n, _dp(u0o), _dp(Bo))
    return u0o, Bo


def argmin_visits(p, s, u1, u0_in, rows):
    """orc_argmin on the listed rows, also returning every position whose B
    was evaluated: (u0_out [n], visits [n, levels * cands + 1])."""
    u1 = _f64(u1, int(p.n_y))
    u0_in = _f64(u0_in, int(p.n_x))
    n, r = _rows(rows, int(p.n_x))
    u0o = np.empty(n, np.float64)
    vis = np.empty((n, int(s.levels) * int(s.cands) + 1), np.float64)
    lib().orc_argmin_visits(C.byref(_prob(p)), C.byref(_search(s)), _dp(u1), _dp(u0_in),
                            r.ctypes.data_as(C.POINTER(C.c_int64)), n, _dp(u0o), _dp(vis))
    return u0o, vis


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's loops (0: the runtime's default)."""
    lib().orc_set_threads(int(n))


def update_u1(p, u0, rows=None) -> np.ndarray:
    u0 = _f64(u0, int(p.n_x))
    if rows is None:
        n, rp = int(p.n_y), None
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        if rows.size and (rows.min() < 0 or rows.max() >= int(p.n_y)):
            raise ValueError("row index out of range")
        n, rp = rows.size, rows.ctypes.data_as(C.POINTER(C.c_int64))
    out = np.empty(n, np.float64)
    lib().orc_update_u1(C.byref(_prob(p)), _dp(u0), rp, n, _dp(out))
    return out


def objective(p, u0, u1) -> float:
    u0 = _f64(u0, int(p.n_x))
    u1 = _f64(u1, int(p.n_y))
    return float(lib().orc_objective(C.byref(_prob(p)), _dp(u0), _dp(u1)))


def solve(p, s, iters: int, u0_init):
    """Returns (u0, u1, J_hist[iters + 1])."""
    u0_init = _f64(u0_init, int(p.n_x))
    u0 = np.empty(int(p.n_x), np.float64)
    u1 = np.empty(int(p.n_y), np.float64)
    J = np.empty(int(iters) + 1, np.float64)
    lib().orc_solve(C.byref(_prob(p)), C.byref(_search(s)), int(iters), _dp(u0_init),
                    _dp(u0), _dp(u1), _dp(J))
    return u0, u1, J


# ---------------------------------------------------------------------------
# Zero-delay source-channel coding (Section V-B): w ~ U(-1, 1), stage-0
# weight ``lam``; the problem object carries ``lam`` instead of ``k``.

def _rows(rows, n):
    if rows is None:
        return n, None
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    if rows.size and (rows.min() < 0 or rows.max() >= n):
        raise ValueError("row index out of range")
    return rows.size, rows


def coding_B(p, u1, x: float, u: float) -> float:
    u1 = _f64(u1, int(p.n_y))
    return float(lib().orc_cd_B(C.byref(_prob(p)), float(p.lam), _dp(u1), float(x), float(u)))


def coding_marginal_cost(p, u1, u) -> np.ndarray:
    u1 = _f64(u1, int(p.n_y))
    u = np.ascontiguousarray(u, dtype=np.float64)
    if u.ndim != 2 or u.shape[0] != int(p.n_x):
        raise ValueError("u must be [n_x, n_cand]")
    out = np.empty_like(u)
    lib().orc_cd_marginal_cost(C.byref(_prob(p)), float(p.lam), _dp(u1), _dp(u), u.shape[1], _dp(out))
    return out


def coding_argmin(p, s, u1, u0_in, rows=None):
    u1 = _f64(u1, int(p.n_y))
    u0_in = _f64(u0_in, int(p.n_x))
    n, r = _rows(rows, int(p.n_x))
    rp = r.ctypes.data_as(C.POINTER(C.c_int64)) if r is not None else None
    u0o = np.empty(n, np.float64)
    Bo = np.empty(n, np.float64)
    lib().orc_cd_argmin(C.byref(_prob(p)), float(p.lam), C.byref(_search(s)), _dp(u1), _dp(u0_in),
                        rp, n, _dp(u0o), _dp(Bo))
    return u0o, Bo


def coding_update_u1(p, u0, rows=None) -> np.ndarray:
    u0 = _f64(u0, int(p.n_x))
    n, r = _rows(rows, int(p.n_y))
    rp = r.ctypes.data_as(C.POINTER(C.c_int64)) if r is not None else None
    out = np.empty(n, np.float64)
    lib().orc_cd_update_u1(C.byref(_prob(p)), _dp(u0), rp, n, _dp(out))
    return out


def coding_objective(p, u0, u1) -> float:
    u0 = _f64(u0, int(p.n_x))
    u1 = _f64(u1, int(p.n_y))
    return float(lib().orc_cd_objective(C.byref(_prob(p)), float(p.lam), _dp(u0), _dp(u1)))


def coding_solve(p, s, iters: int, u0_init):
    """Returns (u0, u1, J_hist[iters + 1])."""
    u0_init = _f64(u0_init, int(p.n_x))
    u0 = np.empty(int(p.n_x), np.float64)
    u1 = np.empty(int(p.n_y), np.float64)
    J = np.empty(int(iters) + 1, np.float64)
    lib().orc_cd_solve(C.byref(_prob(p)), float(p.lam), C.byref(_search(s)), int(iters), _dp(u0_init),
                       _dp(u0), _dp(u1), _dp(J))
    return u0, u1, J


# ---------------------------------------------------------------------------
# Two-dimensional Witsenhausen (Section V-D): tensor grids, vector fields as
# arrays [2, n * n] (node (i1, i2) at i1 * n + i2).

def _planes(a, n, name):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != (2, n):
        raise ValueError(f"{name} must be [2, {n}]")
    return a


def w2_B(p, u1, x, u) -> float:
    u1 = _planes(u1, int(p.n_y) ** 2, "u1")
    return float(lib().orc2_B(C.byref(_prob(p)), _dp(u1), float(x[0]), float(x[1]), float(u[0]), float(u[1])))


def w2_marginal_cost(p, u1, u) -> np.ndarray:
    """u: [2, n_x^2, n_cand]; returns L_0 [n_x^2, n_cand]."""
    nn = int(p.n_x) ** 2
    u1 = _planes(u1, int(p.n_y) ** 2, "u1")
    u = np.ascontiguousarray(u, dtype=np.float64)
    if u.ndim != 3 or u.shape[:2] != (2, nn):
        raise ValueError("u must be [2, n_x^2, n_cand]")
    out = np.empty((nn, u.shape[2]), np.float64)
    lib().orc2_marginal_cost(C.byref(_prob(p)), _dp(u1), _dp(u), u.shape[2], _dp(out))
    return out


def w2_argmin(p, s, u1, u0_in, rows=None):
    nn = int(p.n_x) ** 2
    u1 = _planes(u1, int(p.n_y) ** 2, "u1")
    u0_in = _planes(u0_in, nn, "u0")
    n, r = _rows(rows, nn)
    rp = r.ctypes.data_as(C.POINTER(C.c_int64)) if r is not None else None
    u0o = np.empty((2, n), np.float64)
    Bo = np.empty(n, np.float64)
    lib().orc2_argmin(C.byref(_prob(p)), C.byref(_search(s)), _dp(u1), _dp(u0_in), rp, n, _dp(u0o), _dp(Bo))
    return u0o, Bo


def w2_update_u1(p, u0, rows=None) -> np.ndarray:
    nn = int(p.n_x) ** 2
    u0 = _planes(u0, nn, "u0")
    n, r = _rows(rows, int(p.n_y) ** 2)
    rp = r.ctypes.data_as(C.POINTER(C.c_int64)) if r is not None else None
    out = np.empty((2, n), np.float64)
    lib().orc2_update_u1(C.byref(_prob(p)), _dp(u0), rp, n, _dp(out))
    return out


def w2_objective(p, u0, u1) -> float:
    u0 = _planes(u0, int(p.n_x) ** 2, "u0")
    u1 = _planes(u1, int(p.n_y) ** 2, "u1")
    return float(lib().orc2_objective(C.byref(_prob(p)), _dp(u0), _dp(u1)))


def w2_solve(p, s, iters: int, u0_init):
    nn = int(p.n_x) ** 2
    u0_init = _planes(u0_init, nn, "u0_init")
    u0 = np.empty((2, nn), np.float64)
    u1 = np.empty((2, int(p.n_y) ** 2), np.float64)
    J = np.empty(int(iters) + 1, np.float64)
    lib().orc2_solve(C.byref(_prob(p)), C.byref(_search(s)), int(iters), _dp(u0_init), _dp(u0), _dp(u1), _dp(J))
    return u0, u1, J


# ---------------------------------------------------------------------------
# The paper's generic solver (Algorithm 1) on the Witsenhausen instance.

def B_derivs(p, u1, x: float, u: float):
    """(B, dB/du, d2B/du2) at one point."""
    u1 = _f64(u1, int(p.n_y))
    out = [C.c_double(), C.c_double(), C.c_double()]
    lib().orc_B_derivs(C.byref(_prob(p)), _dp(u1), float(x), float(u), *[C.byref(o) for o in out])
    return tuple(o.value for o in out)


def _rows_ptr(rows, n):
    n, r = _rows(rows, n)
    return n, (r.ctypes.data_as(C.POINTER(C.c_int64)) if r is not None else None)


def alg1_local_u0(p, tau, u1, u0, rows=None):
    u1, u0 = _f64(u1, int(p.n_y)), _f64(u0, int(p.n_x))
    n, rp = _rows_ptr(rows, int(p.n_x))
    out = np.empty(n, np.float64)
    lib().orc_alg1_local_u0(C.byref(_prob(p)), float(tau), _dp(u1), _dp(u0), rp, n, _dp(out))
    return out


def alg1_local_u1(p, u0, u1, rows=None):
    u0, u1 = _f64(u0, int(p.n_x)), _f64(u1, int(p.n_y))
    n, rp = _rows_ptr(rows, int(p.n_y))
    out = np.empty(n, np.float64)
    lib().orc_alg1_local_u1(C.byref(_prob(p)), _dp(u0), _dp(u1), rp, n, _dp(out))
    return out


def _radius(r):
    r = int(r)
    if not 1 <= r <= 31:
        raise ValueError("radius must be 1..31")
    return r


def alg1_pe_u0(p, u1, u0, r=2, tie=0.0, rows=None):
    u1, u0 = _f64(u1, int(p.n_y)), _f64(u0, int(p.n_x))
    n, rp = _rows_ptr(rows, int(p.n_x))
    out = np.empty(n, np.float64)
    lib().orc_alg1_pe_u0(C.byref(_prob(p)), float(tie or TAU64), _radius(r), _dp(u1), _dp(u0), rp, n, _dp(out))
    return out


def alg1_pe_u1(p, u0, u1, r=2, tie=0.0, rows=None):
    u0, u1 = _f64(u0, int(p.n_x)), _f64(u1, int(p.n_y))
    n, rp = _rows_ptr(rows, int(p.n_y))
    out = np.empty(n, np.float64)
    lib().orc_alg1_pe_u1(C.byref(_prob(p)), float(tie or TAU64), _radius(r), _dp(u0), _dp(u1), rp, n, _dp(out))
    return out


def alg1_allocate(N, IL, IP, NL_prev):
    nl, npp = C.c_int32(int(NL_prev)), C.c_int32()
    lib().orc_alg1_allocate(int(N), float(IL), float(IP), C.byref(nl), C.byref(npp))
    return nl.value, npp.value


def alg1_solve(p, u0_init, u1_init, N=20, r=2, prec=1e-10, tau=0.1, tie=0.0, max_rounds=100):
    """Returns (u0, u1, J_log[1 + 2 rounds], NL_log[rounds])."""
    u0_init, u1_init = _f64(u0_init, int(p.n_x)), _f64(u1_init, int(p.n_y))
    a = _Alg1()
    a.N, a.r, a.p, a.tau, a.tie_rel64, a.max_rounds = int(N), _radius(r), float(prec), float(tau), float(tie), \
        int(max_rounds)
    u0 = np.empty(int(p.n_x), np.float64)
    u1 = np.empty(int(p.n_y), np.float64)
    J = np.empty(1 + 2 * int(max_rounds), np.float64)
    NL = np.empty(max(1, int(max_rounds)), np.int32)
    rounds = lib().orc_alg1_solve(C.byref(_prob(p)), C.byref(a), _dp(u0_init), _dp(u1_init), _dp(u0), _dp(u1),
                                  _dp(J), NL.ctypes.data_as(C.POINTER(C.c_int32)))
    return u0, u1, J[:1 + 2 * rounds], NL[:rounds]
