"""Arbitrary-precision brute force of the discrete problem, for tiny grids.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  It restates the
discrete problem at 40 significant digits with mpmath so the FP64 C oracle
can be checked for rounding and indexing mistakes on grids of a few dozen
nodes.  It is written from the definitions (Section V-A objective,
Section III-A marginal cost, Section III-D step-function discretisation),
not from the C code.
"""
from __future__ import annotations

import mpmath as mp

DPS = 40
TAU = mp.mpf("1e-12")


def _nodes(lo, hi, n):
    lo, hi = mp.mpf(lo), mp.mpf(hi)
    return [lo + (hi - lo) * i / (n - 1) for i in range(n)]


def _prior(p, xs):
    out = []
    for x in xs:
        f = mp.mpf(0)
        for (w, mu, sd) in p.comps:
            w, mu, sd = mp.mpf(w), mp.mpf(mu), mp.mpf(sd)
            f += w * mp.npdf(x, mu, sd)
        out.append(f)
    return out


def _Bfun(p, ys, u1, x, u):
    dy = ys[1] - ys[0]
    z = x + u
    acc = mp.mpf(0)
    for y, v in zip(ys, u1):
        acc += mp.npdf(y - z) * (z - v) ** 2
    return mp.mpf(p.k) ** 2 * u ** 2 + dy * acc


def _select(cands, vals, inc, tau=TAU):
    m = min(vals)
    best = None
    for c, v in zip(cands, vals):
        if v <= m * (1 + tau):
            key = (abs(c - inc), c)
            if best is None or key < best[0]:
                best = (key, c, v)
    return best[1], best[2]


def _mpv(v):
    return v if isinstance(v, mp.mpf) else mp.mpf(float(v))


def u1_update(p, u0):
    with mp.workdps(DPS):
        xs = _nodes(p.x_lo, p.x_hi, p.n_x)
        ys = _nodes(p.y_lo, p.y_hi, p.n_y)
        f = _prior(p, xs)
        x1 = [x + mp.mpf(float(u)) for x, u in zip(xs, u0)]
        out = []
        for y in ys:
            num = mp.fsum(fi * mp.npdf(y - a) * a for fi, a in zip(f, x1))
            den = mp.fsum(fi * mp.npdf(y - a) for fi, a in zip(f, x1))
            out.append(num / den)
        return out


def objective(p, u0, u1):
    with mp.workdps(DPS):
        xs = _nodes(p.x_lo, p.x_hi, p.n_x)
        ys = _nodes(p.y_lo, p.y_hi, p.n_y)
        f = _prior(p, xs)
        dx = xs[1] - xs[0]
        dy = ys[1] - ys[0]
        k2 = mp.mpf(p.k) ** 2
        tot = mp.mpf(0)
        for x, fi, u in zip(xs, f, u0):
            u = mp.mpf(float(u))
            a = x + u
            inner = mp.fsum(mp.npdf(y - a) * (a - _mpv(v)) ** 2 for y, v in zip(ys, u1))
            tot += fi * (k2 * u ** 2 + dy * inner)
        return dx * tot


def argmin(p, s, u1, u0_in):
    """Coarse-to-fine search per point with FP64 candidate positions (the
    positions are inputs of the decision, so they are formed in binary64
    exactly as the discrete method defines them); costs at 40 digits."""
    import numpy as np

    with mp.workdps(DPS):
        xs = _nodes(p.x_lo, p.x_hi, p.n_x)
        ys = _nodes(p.y_lo, p.y_hi, p.n_y)
        u1m = [v if isinstance(v, mp.mpf) else mp.mpf(float(v)) for v in u1]
        K, L = int(s.cands), int(s.levels)
        t64 = float(getattr(s, "tie_rel64", 0.0))
        tau = mp.mpf(t64) if t64 > 0 else TAU
        h = [(float(s.u_hi) - float(s.u_lo)) / float(K - 1)]
        for _ in range(1, L):
            h.append(2.0 * h[-1] / float(K - 1))
        out = []
        for i in range(int(p.n_x)):
            # the FP64 grid node, so the decision sees the same x as FP64 code
            x64 = float(np.float64(p.x_lo) + np.float64(i) * ((np.float64(p.x_hi) - np.float64(p.x_lo)) / np.float64(p.n_x - 1)))
            x = mp.mpf(x64)
            inc = float(u0_in[i])
            cs = [float(np.float64(s.u_lo) + np.float64(q) * np.float64(h[0])) for q in range(K)]
            vs = [_Bfun(p, ys, u1m, x, mp.mpf(c)) for c in cs]
            c_best, v_best = _select([mp.mpf(c) for c in cs], vs, mp.mpf(inc), tau)
            c_best = float(c_best)
            for lvl in range(1, L):
                cs = []
                for q in range(K):
                    v = float((np.float64(c_best) - np.float64(h[lvl - 1])) + np.float64(q) * np.float64(h[lvl]))
                    cs.append(min(max(v, float(s.u_lo)), float(s.u_hi)))
                vs = [_Bfun(p, ys, u1m, x, mp.mpf(c)) for c in cs]
                cs.append(c_best)
                vs.append(v_best)
                cb, v_best = _select([mp.mpf(c) for c in cs], vs, mp.mpf(inc), tau)
                c_best = float(cb)
            v_inc = _Bfun(p, ys, u1m, x, mp.mpf(inc))
            cb, _ = _select([mp.mpf(c_best), mp.mpf(inc)], [v_best, v_inc], mp.mpf(inc), tau)
            out.append(float(cb))
        return out


def solve(p, s, iters, u0_init):
    """The solve loop written out from its definition: u1 is the closed-form
    second controller of the initial u0, J_0 = J(u0, u1); then each round
    updates u0 point by point with u1 held fixed, replaces u1 by the closed
    form of the new u0, and records J of the pair.  u1 stays at 40 digits
    between the steps; u0 is a set of binary64 candidate positions.
    Returns (u0 as floats, u1 as mpf, J_hist as mpf)."""
    with mp.workdps(DPS):
        u0 = [float(v) for v in u0_init]
        u1 = u1_update(p, u0)
        J = [objective(p, u0, u1)]
        for _ in range(int(iters)):
            u0 = argmin(p, s, u1, u0)
            u1 = u1_update(p, u0)
            J.append(objective(p, u0, u1))
        return u0, u1, J


# --- the generic solver's steps (Algorithm 1), at 40 digits ----------------

def _B_at(p, ys, u1m, x, u):
    return _Bfun(p, ys, u1m, x, u)


def alg1_local_u0(p, tau, u1, u0):
    """One local update of u0: u - B'/B'' where B'' > 0, else u - tau B', with
    B' and B'' from mpmath's numerical differentiation of the 40-digit B
    (independent of the closed-form derivatives)."""
    with mp.workdps(DPS):
        xs = _nodes(p.x_lo, p.x_hi, p.n_x)
        ys = _nodes(p.y_lo, p.y_hi, p.n_y)
        u1m = [_mpv(v) for v in u1]
        out = []
        for x, u in zip(xs, u0):
            u = mp.mpf(float(u))
            fn = lambda v: _B_at(p, ys, u1m, x, v)
            d1 = mp.diff(fn, u, 1)
            d2 = mp.diff(fn, u, 2)
            out.append(u - d1 / d2 if d2 > 0 else u - mp.mpf(tau) * d1)
        return out


def alg1_pe_u0(p, u1, u0, r):
    """Partial exhaustion of u0: each point takes, by the selection rule, the
    best of the values u0 holds at the nodes within r of it."""
    with mp.workdps(DPS):
        xs = _nodes(p.x_lo, p.x_hi, p.n_x)
        ys = _nodes(p.y_lo, p.y_hi, p.n_y)
        u1m = [_mpv(v) for v in u1]
        n = len(xs)
        out = []
        for i, x in enumerate(xs):
            cs = [mp.mpf(float(u0[k])) for k in range(max(0, i - r), min(n, i + r + 1))]
            vs = [_B_at(p, ys, u1m, x, c) for c in cs]
            c, _ = _select(cs, vs, mp.mpf(float(u0[i])))
            out.append(float(c))
        return out


def alg1_pe_u1(p, u0, u1, r):
    """Partial exhaustion of u1: each y node takes the best of the values u1
    holds at the nodes within r of it, by C_1(u, y) = dx sum f phi (x1 - u)^2."""
    with mp.workdps(DPS):
        xs = _nodes(p.x_lo, p.x_hi, p.n_x)
        ys = _nodes(p.y_lo, p.y_hi, p.n_y)
        f = _prior(p, xs)
        x1 = [x + mp.mpf(float(u)) for x, u in zip(xs, u0)]
        n = len(ys)
        out = []
        for j, y in enumerate(ys):
            w = [fi * mp.npdf(y - a) for fi, a in zip(f, x1)]
            cs = [mp.mpf(float(u1[k])) for k in range(max(0, j - r), min(n, j + r + 1))]
            vs = [mp.fsum(wi * (a - c) ** 2 for wi, a in zip(w, x1)) for c in cs]
            c, _ = _select(cs, vs, mp.mpf(float(u1[j])))
            out.append(float(c))
        return out
