"""Seeded synthetic workloads for the Witsenhausen marginal-cost solver.

This module only describes inputs: problem parameters, search settings,
iteration counts, initial controllers and request traces.  It holds none of
the solver's arithmetic, so both the FP64 oracle side (tests) and the GPU
side (tests, benchmark) can take their inputs from it.  Initial controllers
are functions evaluated at the grid nodes, which are placed by the same
linspace definition the discretisation uses (node i = lo + i * (hi - lo) /
(n - 1)).

The instance is the paper's (Section V-A): x0 ~ N(0, sigma^2), w ~ N(0, 1),
k and sigma as given; the paper's own runs use k = 0.2, sigma = 5
(Section IV).  No dataset is involved.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np


@dataclass
class Problem:
    k: float
    comps: Sequence[Tuple[float, float, float]]  # (weight, mean, sd) of the x0 prior
    x_lo: float
    x_hi: float
    n_x: int
    y_lo: float
    y_hi: float
    n_y: int
    noise_sd: float = 1.0  # standard deviation of the Gaussian noise w (Section V-A: 1)


@dataclass
class Search:
    u_lo: float
    u_hi: float
    levels: int
    cands: int
    tie_rel64: float = 0.0   # relative tie band of the selection rule (0: the default 1e-12)
    band_rel32: float = 0.0  # FP32 pre-selection band of the GPU path (0: its default)


@dataclass
class Case:
    name: str
    prob: Problem
    search: Search
    iters: int
    u0_init: np.ndarray = field(repr=False)
    sigma: float = 0.0


def nodes(lo: float, hi: float, n: int) -> np.ndarray:
    """Grid node positions (linspace definition, binary64)."""
    step = (float(hi) - float(lo)) / float(n - 1)
    return float(lo) + np.arange(int(n), dtype=np.float64) * step


def gaussian_problem(k: float, sigma: float, n: int, half: float) -> Problem:
    return Problem(k=k, comps=[(1.0, 0.0, sigma)], x_lo=-half, x_hi=half, n_x=n,
                   y_lo=-half, y_hi=half, n_y=n)


def init_sign(prob: Problem, sigma: float) -> np.ndarray:
    """u0(x) = sigma * sign(x) - x, with sign(0) = 0 (x1 in {-sigma, 0, sigma})."""
    x = nodes(prob.x_lo, prob.x_hi, prob.n_x)
    return sigma * np.sign(x) - x


def init_random_steps(prob: Problem, sigma: float, seed: int, steps: int = 8) -> np.ndarray:
    """Piecewise-constant u0 with `steps` pieces: breakpoints sorted
    uniform on [-3 sigma, 3 sigma], values uniform on [-sigma, sigma]."""
    rng = np.random.default_rng(seed)
    bp = np.sort(rng.uniform(-3 * sigma, 3 * sigma, steps - 1))
    vals = rng.uniform(-sigma, sigma, steps)
    x = nodes(prob.x_lo, prob.x_hi, prob.n_x)
    return vals[np.searchsorted(bp, x, side="right")]


def init_zero(prob: Problem) -> np.ndarray:
    return np.zeros(int(prob.n_x), np.float64)


def init_affine(prob: Problem, lam: float) -> np.ndarray:
    """u0(x) = (lam - 1) x, so x1 = lam * x."""
    return (lam - 1.0) * nodes(prob.x_lo, prob.x_hi, prob.n_x)


def ranges_for_sigma(sigma: float) -> Tuple[float, float]:
    """Grid half-width max(25, 5 sigma) and search half-width grid + 5;
    at sigma = 5 this is the [-25, 25] grid and [-30, 30] search."""
    half = max(25.0, 5.0 * sigma)
    return half, half + 5.0


# --- the five workload families -------------------------------------------

def small_case() -> Case:
    """k=0.2, sigma=5; 1001-node grids on [-25,25]; 3 levels x 21 candidates
    on [-30,30]; init sigma*sign(x)-x; 10 rounds."""
    p = gaussian_problem(0.2, 5.0, 1001, 25.0)
    return Case("wits-1001-3x21", p, Search(-30.0, 30.0, 3, 21), 10, init_sign(p, 5.0), 5.0)


def paper_res_case() -> Case:
    """As the small case at 20001 nodes; 5 levels x 16 candidates; 30 rounds."""
    p = gaussian_problem(0.2, 5.0, 20001, 25.0)
    return Case("wits-20001-5x16", p, Search(-30.0, 30.0, 5, 16), 30, init_sign(p, 5.0), 5.0)


def sweep_cases(n: int = 20001, ks=(0.05, 0.2, 0.5), sigmas=(1.0, 5.0, 10.0),
                seeds=range(9)) -> List[Case]:
    """Precision sweep: every (k, sigma, seed) with a random 8-step init."""
    out = []
    for k in ks:
        for sg in sigmas:
            half, uh = ranges_for_sigma(sg)
            p = gaussian_problem(k, sg, n, half)
            for sd in seeds:
                out.append(Case(f"sweep-k{k}-s{sg}-seed{sd}", p, Search(-uh, uh, 5, 16), 10,
                                init_random_steps(p, sg, sd), sg))
    return out


@dataclass
class Request:
    arrival: float  # seconds from the start of the trace
    case: Case


def serving_trace(n_req: int = 4096, rate: float = 100.0, seed: int = 0,
                  sizes=(1001, 4001, 8001, 20001), iters: int = 20) -> List[Request]:
    """Poisson arrivals at `rate` per second; k ~ logU[0.05, 0.5],
    sigma ~ logU[1, 10], grid size uniform over `sizes`; 3 x 21 search;
    init sigma*sign(x)-x."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n_req))
    ks = np.exp(rng.uniform(math.log(0.05), math.log(0.5), n_req))
    sg = np.exp(rng.uniform(math.log(1.0), math.log(10.0), n_req))
    nn = rng.choice(np.asarray(sizes), n_req)
    out = []
    for r in range(n_req):
        half, uh = ranges_for_sigma(float(sg[r]))
        p = gaussian_problem(float(ks[r]), float(sg[r]), int(nn[r]), half)
        c = Case(f"req{r}", p, Search(-uh, uh, 3, 21), iters, init_sign(p, float(sg[r])), float(sg[r]))
        out.append(Request(float(t[r]), c))
    return out


def mixture_case(s: int, n: int = 65536, levels: int = 4, cands: int = 32, iters: int = 3) -> Case:
    """Instance s of the large batched family: a 3-component Gaussian
    mixture prior (means U[-10,10], sds U[1,4], weights Dirichlet(1,1,1)),
    k=0.2, grids of n nodes on [-40,40], search 4 x 32 on [-30,30], u0 = 0."""
    rng = np.random.default_rng(s)
    mu = rng.uniform(-10.0, 10.0, 3)
    sd = rng.uniform(1.0, 4.0, 3)
    w = rng.dirichlet(np.ones(3))
    p = Problem(k=0.2, comps=[(float(w[c]), float(mu[c]), float(sd[c])) for c in range(3)],
                x_lo=-40.0, x_hi=40.0, n_x=n, y_lo=-40.0, y_hi=40.0, n_y=n)
    return Case(f"mix{s}-{n}", p, Search(-30.0, 30.0, levels, cands), iters, init_zero(p), 0.0)


def mixture_batch(n_inst: int = 64, n: int = 65536) -> List[Case]:
    return [mixture_case(s, n) for s in range(n_inst)]


# --- zero-delay source-channel coding (Section V-B) ------------------------
# x0 ~ N(0, 1), x1 = u0(x0) + w with w ~ U(-1, 1), stage-0 weight lam; the
# paper's figure uses lam = 2.

@dataclass
class CodingProblem:
    lam: float
    comps: Sequence[Tuple[float, float, float]]
    x_lo: float
    x_hi: float
    n_x: int
    y_lo: float
    y_hi: float
    n_y: int


@dataclass
class CodingCase:
    name: str
    prob: CodingProblem
    search: Search
    iters: int
    u0_init: np.ndarray = field(repr=False)


def coding_problem(n_x: int, n_y: int, lam: float = 2.0, comps=((1.0, 0.0, 1.0),)) -> CodingProblem:
    """x grid [-8, 8] (prior tail below 1e-14), y grid [-5, 5] (encoder
    range [-4, 4] plus the noise's reach)."""
    return CodingProblem(lam=lam, comps=list(comps), x_lo=-8.0, x_hi=8.0, n_x=n_x,
                         y_lo=-5.0, y_hi=5.0, n_y=n_y)


def coding_init(prob: CodingProblem, seed: int = 0, steps: int = 6) -> np.ndarray:
    """Piecewise-constant encoder: breakpoints sorted uniform on [-3, 3],
    levels sorted uniform on [-2.5, 2.5] (a monotone quantiser)."""
    rng = np.random.default_rng(seed)
    bp = np.sort(rng.uniform(-3.0, 3.0, steps - 1))
    vals = np.sort(rng.uniform(-2.5, 2.5, steps))
    x = nodes(prob.x_lo, prob.x_hi, prob.n_x)
    return vals[np.searchsorted(bp, x, side="right")]


def coding_small_case() -> CodingCase:
    """801 x-nodes, 1201 y-nodes (ragged against 256-wide tiles);
    3 levels x 9 candidates on [-4, 4]; 4 rounds."""
    p = coding_problem(801, 1201)
    return CodingCase("coding-801x1201-3x9", p, Search(-4.0, 4.0, 3, 9), 4, coding_init(p, 1))


def coding_paper_case(n: int = 20001, iters: int = 30) -> CodingCase:
    """lam = 2 (the paper's figure), 20001-node grids, the 5 x 16 search of
    the Witsenhausen runs on [-4, 4], 30 rounds."""
    p = coding_problem(n, n)
    return CodingCase(f"coding-{n}-5x16", p, Search(-4.0, 4.0, 5, 16), iters, coding_init(p, 0))


# --- two-dimensional Witsenhausen (Section V-D) -----------------------------
# x0 in R^2 with both coordinates drawn from the same prior, w ~ N(0, I_2),
# J = 1/2 E[k^2 |u0|^2 + |x2|^2]; the paper runs k = 0.2, sigma = 5 on
# 160 x 160 nodes.  Vector fields are arrays [2, n * n], node (i1, i2) at
# index i1 * n + i2.

def w2_problem(n: int, n_y: int = None, k: float = 0.2, sigma: float = 5.0, half: float = 25.0) -> Problem:
    """The 1-D problem whose tensor product is the 2-D grid."""
    return Problem(k=k, comps=[(1.0, 0.0, sigma)], x_lo=-half, x_hi=half, n_x=n, y_lo=-half, y_hi=half,
                   n_y=n_y or n)


def w2_separable(prob: Problem, g: np.ndarray) -> np.ndarray:
    """u0(x) = (g(x1), g(x2)) from a 1-D field g on the grid."""
    n = int(prob.n_x)
    return np.stack([np.repeat(g, n), np.tile(g, n)])


def w2_init(prob: Problem, seed: int = 0) -> np.ndarray:
    """A non-separable start: sigma sign(x_c) - x_c in each coordinate c,
    plus a seeded smooth coupling 0.5 sin(x_2 / 3) in the first coordinate."""
    n = int(prob.n_x)
    x = nodes(prob.x_lo, prob.x_hi, n)
    sigma = float(prob.comps[0][2])
    g = sigma * np.sign(x) - x
    u = w2_separable(prob, g)
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * math.pi)
    u[0] += 0.5 * np.sin(np.tile(x, n) / 3.0 + ph)
    return u


@dataclass
class W2Case:
    name: str
    prob: Problem
    search: Search
    iters: int
    u0_init: np.ndarray = field(repr=False)


def w2_small_case() -> W2Case:
    """21 x 21 x-nodes, 31 x 31 y-nodes on [-25, 25], 3 levels x 5 x 5
    candidates on [-30, 30], 3 rounds."""
    p = w2_problem(21, 31)
    return W2Case("w2-21x31-3x5", p, Search(-30.0, 30.0, 3, 5), 3, w2_init(p, 1))


def w2_paper_case(iters: int = 10) -> W2Case:
    """k = 0.2, sigma = 5, 160 x 160 nodes on [-25, 25] (the paper's sample
    count), 4 levels x 8 x 8 candidates on [-30, 30]."""
    p = w2_problem(160)
    return W2Case("w2-160-4x8x8", p, Search(-30.0, 30.0, 4, 8), iters, w2_init(p, 0))
