"""Benchmark of the MI355X marginal-cost solver.

Default (``--workload headline``): the largest single-GPU workload, 64
instances of 65536-node grids on [-40, 40] with seeded 3-component mixture
priors, k = 0.2, unit Gaussian noise, a 4 levels x 32 candidates search on
[-30, 30], u0 = 0, 3 rounds, FP32 terms with compensated sums, all in shared
launches.  One step is one batched solve of every instance: the prior, the
closed-form u1 of the initial controller, then every round of (the
coarse-to-fine u0 update over all levels - the marginal-cost sums, the
per-point selection with FP64 tie re-evaluation and the comparison with the
incumbent - the u0 advance, the u1 update and the FP64 objective), inputs
resident in HBM before the timed region.  The same line carries the
serving leg (continuous batching on the 4096-request Poisson trace at 0.8
and 0.5 of saturation, against one solve at a time run live on the same
arrivals), the roofline of the marginal-cost kernel from HIP events around
its launches, and the FP64 oracle's rate on the host (all threads and one).

The metric counts algorithmic marginal-cost terms: (point, candidate,
y node) triples with |y - x - u| <= 9 noise sds, counted on the device.
Prints one JSON line.  ``--workload paper`` times one 20001-node solve
(5 x 16, 30 rounds); the other workloads print lines of their own.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# ALU roofline of the marginal-cost kernel.  MI355X issues 128 FP32 VALU
# lane-operations per clock per CU without packed math (the published
# 157.3 TFLOP/s FP32 vector peak counts an FMA as two flops):
# 256 CUs x 128 x 2.4 GHz = 78.6e12 slots/s; v_exp_f32 issues at a quarter
# of that rate (4 slots).  The kernel factors the shifted Gaussian into a
# per-offset table value and a per-lane exponential, stages the differences
# around a per-block reference and folds the per-lane factor of the
# exponential into the difference, so one algorithmic term needs 3 FP32
# operations (scaled difference, weight, accumulate).  Blocks of 16 terms go
# in pairs that share one exponential: the first block takes 7 more slots
# (one exp2 = 4 and its argument, the block scale, the two-chain combine),
# the second 3 (its factor exp2(16 beta) times the first's, the scale, the
# combine) and the pair 5 (adding the two, 4 of compensation):
# 3 + (7 + 3 + 5)/32 = 3.46875 slots per term.  (Blocks whose
# positions spread wider than the reference form allows take two more
# operations per term; the count above is the smaller one.)
PEAK_SLOTS = 256 * 128 * 2.4e9
# Source-channel coding: the encoder search is FP64 work; MI355X's FP64
# vector peak is 78.6 TFLOP/s (an FMA counts two).  One B evaluation in the
# double-double box-window form takes about 144 FP64 flops: the two prefix
# lookups (44), the window sums (22), the expanded quadratic (42), the
# scaling (6) and the window's ends (30).
PEAK_FP64 = 78.6e12
CODING_FLOPS_PER_B = 144
# Two-dimensional Witsenhausen search: one windowed noise term is two
# differences, |e|^2 (two products and a sum), the weighted accumulate (an
# FMA) and the Gaussian recurrence (two products): 9 FP64 flops.
W2_FLOPS_PER_TERM = 9
SLOTS_PER_TERM = 3.46875


def kernel_source_hash():
    """Hash of the marginal-cost kernel's sources (the kernels and the
    shared header with their constants and layouts)."""
    import hashlib

    h = hashlib.sha256()
    for name in ("ucp_kernels.hip", "ucp_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1908_04489_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload_name):
    """HBM bytes per launch of the marginal-cost kernel from the committed
    rocprofv3 PMC summary (FETCH_SIZE and WRITE_SIZE, scaled by the same
    counters on a plain copy of known size), or None when the summary is
    missing or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"pmc-traffic_{workload_name}.md")
    return parse_traffic(path, kernel_source_hash())


def parse_traffic(path, src_hash):
    """The marginal-cost bytes per launch of a PMC traffic summary, if the
    summary was taken on the kernel source with hash `src_hash`."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ": " in line and line.startswith("- "):
            k, v = line[2:].split(": ", 1)  # keys may hold a colon ("sha256[:16]")
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel source sha256[:16]") != src_hash:
        return None
    try:
        return float(vals["marginal-cost kernel HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


def workload(name):
    import workloads as W

    if name == "paper":
        return W.paper_res_case()
    if name == "small":
        return W.small_case()
    raise SystemExit(f"unknown workload {name}")


def host_info():
    """CPU model and the logical CPUs this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "cpu_count": os.cpu_count()}


def alg_terms(p, rows, visits):
    """Algorithmic terms of the positions an update evaluated: for each
    (row i, position c), the y nodes within 9 noise sds of x_i + c, counted
    with the device counter's rule."""
    import numpy as np

    dx = (p.x_hi - p.x_lo) / (p.n_x - 1)
    dy = (p.y_hi - p.y_lo) / (p.n_y - 1)
    z = (p.x_lo + rows.astype(np.float64) * dx)[:, None] + visits
    lo = np.maximum(np.ceil((z - 9.0 - p.y_lo) * (1.0 / dy)), 0.0)
    hi = np.minimum(np.floor((z + 9.0 - p.y_lo) * (1.0 / dy)), p.n_y - 1.0)
    return float(np.sum(np.maximum(hi - lo + 1.0, 0.0)))


def cpu_baseline(cases, budget_s=10.0, one_core_s=6.0, seed=0):
    """The FP64 oracle, as it stands, on a bounded sample of the workload:
    one u0 update (every level and the incumbent) of randomly drawn rows of
    each listed instance, given the oracle's own u1 of the instance's
    initial controller, first on all the host's threads, then on one.  The
    work is counted from the positions the oracle evaluated, with the
    device counter's rule (nodes within 9 noise sds)."""
    import numpy as np

    import oracle

    rng = np.random.default_rng(seed)
    u1s = [oracle.update_u1(c.prob, c.u0_init) for c in cases]  # set-up, untimed
    c0 = cases[0]
    probe = np.sort(rng.choice(c0.prob.n_x, 32, replace=False))
    t0 = time.perf_counter()
    oracle.argmin_visits(c0.prob, c0.search, u1s[0], c0.u0_init, probe)
    per_row = (time.perf_counter() - t0) / len(probe)
    n = int(max(32, min(c0.prob.n_x, budget_s / len(cases) / max(per_row, 1e-9))))
    alg = dense = dt = 0.0
    for c, u1 in zip(cases, u1s):
        p, s = c.prob, c.search
        rows = np.sort(rng.choice(p.n_x, min(n, p.n_x), replace=False))
        t0 = time.perf_counter()
        _, vis = oracle.argmin_visits(p, s, u1, c.u0_init, rows)
        dt += time.perf_counter() - t0
        alg += alg_terms(p, rows, vis)
        dense += float(vis.size) * p.n_y
    threads = oracle.num_threads()
    # one core: fewer rows of the first instance
    n1 = int(max(8, min(c0.prob.n_x, one_core_s / max(per_row * threads, 1e-9))))
    rows1 = np.sort(rng.choice(c0.prob.n_x, n1, replace=False))
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        _, vis1 = oracle.argmin_visits(c0.prob, c0.search, u1s[0], c0.u0_init, rows1)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(0)
    alg1 = alg_terms(c0.prob, rows1, vis1)
    out = {"value": alg / dt, "unit": "terms/s", "cores": threads, "kind": "oracle",
           "sample": f"one u0 update of {n} random rows in each of {len(cases)} instance(s) "
                     f"({cases[0].search.levels}x{cases[0].search.cands} levels + incumbent, "
                     f"{vis.shape[1]} positions per row), {dt:.1f} s wall on {threads} threads; "
                     f"dense FP64 evaluation {dense / dt:.3e} terms/s",
           "one_core": {"value": alg1 / dt1, "unit": "terms/s", "cores": 1,
                        "sample": f"{n1} rows of {cases[0].name}, {dt1:.1f} s"}}
    out.update(host_info())
    return out


METRIC = "marginal-cost quadrature terms/s; served solves/s + p50/p99 at cost err\u22641e-6"


def batch_leg(a):
    """The 64-instance batch of 65536-node mixture-prior problems (4 x 32
    search, 3 rounds, u0 = 0) in shared launches: one step is one batched
    solve of every instance.  Returns the fields of the bench line."""
    import numpy as np
    import torch

    import paper_1908_04489_amd as U
    import workloads as W

    cases = W.mixture_batch(a.instances, n=65536)
    probs, srch = [c.prob for c in cases], [c.search for c in cases]
    iters = [c.iters for c in cases]
    u0s = [torch.as_tensor(c.u0_init).cuda() for c in cases]
    name = f"mixture-batch-{len(cases)}x65536-4x32"
    print(f"# {name}: {iters[0]} rounds, {a.prec}", file=sys.stderr, flush=True)
    for w in range(a.warmup):
        U.solve_batch(probs, srch, iters, u0s, a.prec)
        print(f"# warmup {w} done", file=sys.stderr, flush=True)
    st = torch.cuda.current_stream()
    torch.cuda.synchronize()
    U.profile(["marginal_cost"])  # HIP events around each marginal-cost launch of the timed steps
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(st)
    terms = evaluated = evals = 0
    for k in range(a.steps):
        out = U.solve_batch(probs, srch, iters, u0s, a.prec)
        t_, v_, e_ = U.last_counts()
        terms, evaluated, evals = terms + t_, evaluated + v_, evals + e_
        print(f"# step {k} done", file=sys.stderr, flush=True)
    ev1.record(st)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    mc_ms, mc_n = U.profile_read()["marginal_cost"]
    breakdown = kernel_breakdown(U, lambda: U.solve_batch(probs, srch, iters, u0s, a.prec))
    mc_avg_s = mc_ms / 1e3 / max(mc_n, 1)
    achieved = terms / max(mc_n, 1) * SLOTS_PER_TERM / mc_avg_s
    C = cases[0].search.levels * cases[0].search.cands + 1
    dense = float(len(cases)) * 65536.0 * C * 65536.0 * iters[0] * a.steps
    res = {"value": terms / (ms / 1e3), "unit": "terms/s", "ms_per_step": ms / a.steps,
           "config": {"workload": name, "instances": len(cases), "n_x": 65536, "n_y": 65536, "grid": [-40.0, 40.0],
                      "prior": "3-component Gaussian mixture per instance (seeded)", "k": 0.2, "levels": 4,
                      "cands": 32, "rounds": iters[0], "init": "u0 = 0", "prec": a.prec},
           "alg_terms_per_step": terms / a.steps, "evaluated_terms_per_step": evaluated / a.steps,
           "fp64_tie_evals_per_step": evals / a.steps, "dense_equiv_terms_per_s": dense / (ms / 1e3),
           "solves_per_s": len(cases) * a.steps / (ms / 1e3),
           "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS / 1e12, "unit": "Tslot/s",
                        "frac": achieved / PEAK_SLOTS, "traffic": measured_traffic(name),
                        "kernel": "k_mc32<FP32_KAHAN> (marginal-cost window sums)",
                        "per_unit": f"{SLOTS_PER_TERM} FP32 VALU slots per algorithmic term",
                        "kernel_avg_us": mc_avg_s * 1e6, "kernel_launches": mc_n,
                        "kernel_terms_per_s": terms / max(mc_n, 1) / mc_avg_s,
                        "kernel_dense_equiv_terms_per_s": dense / max(mc_n, 1) / mc_avg_s},
           "kernel_ms_per_step": breakdown}
    if not a.no_check:
        # the cost error bar: J of the final state of two instances against
        # the oracle's objective of the same state (FP64 both sides)
        import oracle

        errs = []
        for b in (0, len(cases) - 1):
            u0h, u1h = out[0][b].cpu().numpy(), out[1][b].cpu().numpy()
            Jo = oracle.objective(probs[b], u0h, u1h)
            errs.append(abs(out[2][b].cpu().numpy()[-1] - Jo) / Jo)
        res["J_final_rel_err_vs_oracle_objective"] = float(max(errs))
    return res, cases


def gt_leg(a, cases):
    """The same batch in the Gauss-transform arithmetic (UCP_FP64_GT): every
    marginal cost in FP64 from a per-node moment table of u1 instead of the
    window sums (decisions need no FP32 band).  Not the metric's method:
    reported beside it, with its own time and cost error."""
    import torch

    import paper_1908_04489_amd as U

    probs, srch = [c.prob for c in cases], [c.search for c in cases]
    iters = [c.iters for c in cases]
    u0s = [torch.as_tensor(c.u0_init).cuda() for c in cases]
    U.solve_batch(probs, srch, iters, u0s, "fp64_gt")  # warm-up
    st = torch.cuda.current_stream()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(st)
    for k in range(a.gt_steps):
        out = U.solve_batch(probs, srch, iters, u0s, "fp64_gt")
    ev1.record(st)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / a.gt_steps
    breakdown = kernel_breakdown(U, lambda: U.solve_batch(probs, srch, iters, u0s, "fp64_gt"))
    res = {"ms_per_step": ms, "solves_per_s": len(cases) * 1e3 / ms, "steps": a.gt_steps,
           "kernel_ms_per_step": breakdown}
    print(f"# fp64_gt: {ms:.1f} ms per step", file=sys.stderr, flush=True)
    if not a.no_check:
        import oracle

        errs = []
        for b in (0, len(cases) - 1):
            Jo = oracle.objective(probs[b], out[0][b].cpu().numpy(), out[1][b].cpu().numpy())
            errs.append(abs(out[2][b].cpu().numpy()[-1] - Jo) / Jo)
        res["J_final_rel_err_vs_oracle_objective"] = float(max(errs))
    return res


def serving_leg(a):
    """Continuous batching on the Poisson trace (4096 requests, seed 0) at
    0.8 and 0.5 of the server's saturated rate, against one solve at a time
    (ucp_solve, B = 1) run live, first come first served, on the same
    arrivals.  Returns the serving fields of the bench line."""
    import numpy as np
    import torch

    import paper_1908_04489_amd as U
    import workloads as W

    n = a.requests
    trace = W.serving_trace(n_req=n, rate=1.0, seed=0)  # unit rate: arrival times rescaled below
    unit_t = np.array([r.arrival for r in trace])

    def run_server(arrivals, max_slots, keep_out=None):
        srv = U.Server(max_slots=max_slots, prec=a.prec)
        t0 = time.perf_counter()
        nxt = 0
        done = {}
        live = []
        while len(done) < n:
            now = time.perf_counter() - t0
            while nxt < n and arrivals[nxt] <= now:
                c = trace[nxt].case
                live.append((srv.submit(c.prob, c.search, c.iters, c.u0_init), nxt))
                nxt += 1
            q, r, _ = srv.stats()
            if q + r == 0:
                if nxt < n:
                    time.sleep(max(0.0, min(0.01, arrivals[nxt] - now)))
                continue
            srv.step()
            t_now = time.perf_counter() - t0
            # admission is first come first served and at most max_slots
            # requests run at once, so only the first max_slots unfinished
            # requests (in submission order) can have finished in this step
            keep = []
            for tk, idx in live[:max_slots]:
                out = srv.poll(tk)
                if out is None:
                    keep.append((tk, idx))
                else:
                    done[idx] = t_now
                    if keep_out is not None:
                        keep_out[idx] = out
                    if len(done) % 1024 == 0:
                        print(f"# {len(done)}/{n} served", file=sys.stderr, flush=True)
            live = keep + live[max_slots:]
        srv.close()
        return np.array([done[i] for i in range(n)])

    # inputs of the one-at-a-time runs resident on the device beforehand
    u0_dev = [torch.as_tensor(r.case.u0_init).cuda() for r in trace]

    def run_fifo(arrivals, keep_out=None):
        """ucp_solve per request in arrival order; a request starts when it
        has arrived and the previous one has finished (ucp_solve returns
        when its work is done)."""
        t0 = time.perf_counter()
        end = np.empty(n)
        for i, r in enumerate(trace):
            wait = arrivals[i] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            c = r.case
            out = U.solve(c.prob, c.search, c.iters, u0_dev[i], a.prec)
            if keep_out is not None:
                keep_out.append(out)  # device tensors, compared after the timed runs
            end[i] = time.perf_counter() - t0
            if (i + 1) % 1024 == 0:
                print(f"# one at a time: {i + 1}/{n}", file=sys.stderr, flush=True)
        return end

    served, alone = {}, []
    fin = run_server(np.zeros(n), a.slots, served)  # saturated: every request queued at t = 0
    sat = n / fin.max()
    print(f"# server saturated: {sat:.1f} solves/s", file=sys.stderr, flush=True)
    fifo_sat = run_fifo(np.zeros(n), alone)
    sat1 = n / fifo_sat.max()
    print(f"# one at a time saturated: {sat1:.1f} solves/s", file=sys.stderr, flush=True)
    # every request served in the mix against the same request solved alone
    same = sum(all(np.array_equal(sv, t.cpu().numpy()) for sv, t in zip(served[i], alone[i])) for i in range(n))
    del served, alone
    print(f"# served results bitwise equal to the same request alone: {same}/{n}", file=sys.stderr, flush=True)
    rates = {}
    for frac in (0.8, 0.5):
        rate = frac * sat
        arr = unit_t / rate
        fin = run_server(arr, a.slots)
        lat = fin - arr
        end = run_fifo(arr)
        lat1 = end - arr
        rates[f"{frac}x"] = {
            "offered_per_s": rate,
            "server": {"solves_per_s": n / fin.max(), "p50_latency_s": float(np.percentile(lat, 50)),
                       "p99_latency_s": float(np.percentile(lat, 99))},
            "one_at_a_time": {"solves_per_s": n / end.max(), "p50_latency_s": float(np.percentile(lat1, 50)),
                              "p99_latency_s": float(np.percentile(lat1, 99))}}
        print(f"# {frac}x: server p99 {rates[f'{frac}x']['server']['p99_latency_s']:.3f} s, one at a time "
              f"p99 {rates[f'{frac}x']['one_at_a_time']['p99_latency_s']:.3f} s", file=sys.stderr, flush=True)
    return {"workload": f"serving-poisson-{n}", "requests": n, "sizes": [1001, 4001, 8001, 20001],
            "k": "logU[0.05, 0.5]", "sigma": "logU[1, 10]", "search": "3x21", "rounds": 20, "max_slots": a.slots,
            "prec": a.prec, "saturated_solves_per_s": sat, "one_at_a_time_saturated_solves_per_s": sat1,
            "rates": rates,
            "served_equal_alone": {"requests": n, "bitwise_equal": int(same),
                                   "compared": "u0, u1 and J of each request of the saturated server run "
                                               "against ucp_solve of the same request alone"}}


def bench_headline(a):
    """The bench line: the 64 x 65536 batch (the metric's terms/s), the
    served solves/s with p50/p99, the roofline of the marginal-cost kernel
    and the oracle's CPU baseline."""
    res, cases = batch_leg(a)
    line = {"metric": METRIC, "value": res.pop("value"), "unit": res.pop("unit"), "n_gpus": 1, "steps": a.steps,
            "warmup": a.warmup, "ms_per_step": res.pop("ms_per_step"), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic"}
    line.update(res)
    if a.gt_steps > 0:
        line["fp64_gt"] = gt_leg(a, cases)
    if not a.no_serving:
        line["serving"] = serving_leg(a)
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(cases[:4])
    print(json.dumps(line), flush=True)


def bench_serving(a):
    """The serving leg alone, as its own line."""
    srv = serving_leg(a)
    r = srv["rates"]["0.8x"]["server"]
    res = {"metric": "served solves/s", "value": r["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": 1,
           "warmup": 0, "ms_per_step": srv["requests"] / r["solves_per_s"] * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": srv["workload"]}, "serving": srv}
    print(json.dumps(res), flush=True)


def bench_sweep(a):
    """Precision study on 20001-node grids: k in {0.05, 0.2, 0.5}, sigma in
    {1, 5, 10}, seeds 0..8 (random 8-step initial u0), 3 rounds in each
    arithmetic.  Errors against the FP64 oracle on the same state:
    - J of the final state (oracle objective in full);
    - u1 on sampled y rows (oracle u1 of the same u0);
    - one more u0 update on sampled x rows (oracle argmin given the same u1
      and u0): fraction of differing decisions and their FP64 cost gap;
    - marginal cost at u0 on sampled rows (relative error).
    Prints one JSON line with per-precision maxima and medians."""
    import numpy as np
    import torch

    import oracle
    import paper_1908_04489_amd as U
    import workloads as W

    cases = W.sweep_cases(n=a.sweep_n, seeds=range(a.sweep_seeds))
    rng = np.random.default_rng(0)
    stats = {p: {"J_rel": [], "u1_abs": [], "L0_rel": [], "u0_diff_frac": [], "u0_gap": [], "ms": []}
             for p in ("fp32", "fp32_kahan", "fp64")}
    for ci, c in enumerate(cases):
        p, s = c.prob, c.search
        x = oracle.grid(p.x_lo, p.x_hi, p.n_x)
        rows = np.sort(rng.choice(p.n_x, a.sweep_rows, replace=False))
        yrows = np.sort(rng.choice(p.n_y, a.sweep_rows, replace=False))
        u0i = torch.as_tensor(c.u0_init).cuda()
        for prec in ("fp32", "fp32_kahan", "fp64"):
            t0 = time.perf_counter()
            u0g, u1g, Jg = U.solve(p, s, 3, u0i, prec)
            torch.cuda.synchronize()
            stats[prec]["ms"].append((time.perf_counter() - t0) * 1e3)
            u0 = u0g.cpu().numpy()
            u1 = u1g.cpu().numpy()
            Jo = oracle.objective(p, u0, u1)
            stats[prec]["J_rel"].append(abs(Jg.cpu().numpy()[-1] - Jo) / Jo)
            ref_u1 = oracle.update_u1(p, u0, rows=yrows)
            got_u1 = U.update_u1(p, u0g, prec).cpu().numpy()[yrows]
            f, _ = oracle.prior(p)
            stats[prec]["u1_abs"].append(float(np.max(np.abs(got_u1 - ref_u1))))
            L0g = U.marginal_cost(p, u1g, u0g[:, None].contiguous(), prec).cpu().numpy()[rows, 0]
            L0o = np.array([f[i] * oracle.B(p, u1, x[i], u0[i]) for i in rows])
            ok = L0o > 1e-300
            stats[prec]["L0_rel"].append(float(np.max(np.abs(L0g[ok] - L0o[ok]) / L0o[ok])) if ok.any() else 0.0)
            nxt = U.argmin_adaptive(p, s, u1g, u0g, prec).cpu().numpy()[rows]
            ref, Bref = oracle.argmin(p, s, u1, u0, rows=rows)
            d = np.nonzero(nxt != ref)[0]
            stats[prec]["u0_diff_frac"].append(len(d) / len(rows))
            gaps = [(oracle.B(p, u1, x[rows[r]], nxt[r]) - Bref[r]) / Bref[r] for r in d]
            stats[prec]["u0_gap"].append(float(max(gaps)) if gaps else 0.0)
        print(f"# {ci + 1}/{len(cases)} {c.name} J_rel " +
              " ".join(f"{k}={stats[k]['J_rel'][-1]:.1e}" for k in stats), file=sys.stderr, flush=True)
    summ = {}
    for k, v in stats.items():
        summ[k] = {m: {"max": float(np.max(x)), "median": float(np.median(x))} for m, x in v.items()}
    res = {"metric": "precision sweep: error vs FP64 oracle", "value": summ["fp32_kahan"]["J_rel"]["max"],
           "unit": "max relative J error (FP32 compensated)", "n_gpus": 1, "steps": len(cases), "warmup": 0,
           "ms_per_step": float(np.mean(stats["fp32_kahan"]["ms"])), "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"precision-sweep-{a.sweep_n}", "instances": len(cases), "rounds": 3,
                      "rows_sampled": a.sweep_rows},
           "by_precision": summ}
    print(json.dumps(res), flush=True)


def bench_coding(a):
    """Source-channel coding (Section V-B): lam = 2, 20001-node grids, the
    5 x 16 search, 30 rounds; one step is one whole solve, FP64."""
    import numpy as np
    import torch

    import paper_1908_04489_amd as U
    import workloads as W

    case = W.coding_paper_case()
    p, s = case.prob, case.search
    u0 = torch.as_tensor(case.u0_init).cuda()
    print(f"# workload {case.name}: n={p.n_x}, {s.levels}x{s.cands}, {case.iters} rounds, fp64", file=sys.stderr,
          flush=True)
    for w in range(a.warmup):
        U.coding_solve(p, s, case.iters, u0)
    st = torch.cuda.current_stream()
    torch.cuda.synchronize()
    U.profile(["marginal_cost"])  # HIP events around each encoder-search launch of the timed solves
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(st)
    for k in range(a.steps):
        out = U.coding_solve(p, s, case.iters, u0)
    ev1.record(st)
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / a.steps
    se_ms, se_n = U.profile_read()["marginal_cost"]
    breakdown = kernel_breakdown(U, lambda: U.coding_solve(p, s, case.iters, u0))
    se_avg_s = se_ms / 1e3 / max(se_n, 1)
    evals = p.n_x * (s.levels * s.cands + 1)  # B evaluations per search launch
    achieved = evals * CODING_FLOPS_PER_B / se_avg_s
    J = out[2].cpu().numpy()
    res = {"metric": "coding solves/s", "value": 1e3 / ms_step, "unit": "solves/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": case.name, "n_x": p.n_x, "n_y": p.n_y, "levels": s.levels, "cands": s.cands,
                      "rounds": case.iters, "lam": p.lam},
           "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                        "frac": achieved / PEAK_FP64, "traffic": None,
                        "kernel": "k_cd_search<16> (encoder search)",
                        "per_unit": f"{CODING_FLOPS_PER_B} FP64 flops per B evaluation, {evals} per launch",
                        "kernel_avg_us": se_avg_s * 1e6, "kernel_launches": se_n},
           "kernel_ms_per_step": {"search": breakdown["marginal_cost"], "prefix": breakdown["select"],
                                  "u1": breakdown["u1"], "objective": breakdown["objective"]},
           "J_final": float(J[-1])}
    if not a.no_check:
        import oracle

        Jo = oracle.coding_objective(p, out[0].cpu().numpy(), out[1].cpu().numpy())
        res["J_final_rel_err_vs_oracle_objective"] = abs(J[-1] - Jo) / Jo
    if not a.no_cpu:
        res["cpu_baseline"] = coding_cpu_baseline(case)
    print(json.dumps(res), flush=True)


def bench_w2(a):
    """Two-dimensional Witsenhausen (Section V-D): k = 0.2, sigma = 5,
    160 x 160 nodes, 4 levels x 8 x 8 candidates, 10 rounds; one step is
    one whole solve, FP64."""
    import numpy as np
    import torch

    import paper_1908_04489_amd as U
    import workloads as W

    case = W.w2_paper_case()
    p, s = case.prob, case.search
    u0 = torch.as_tensor(case.u0_init).cuda()
    print(f"# workload {case.name}: {p.n_x}^2 nodes, {s.levels}x{s.cands}^2, {case.iters} rounds, fp64",
          file=sys.stderr, flush=True)
    for w in range(a.warmup):
        U.w2_solve(p, s, case.iters, u0)
    st = torch.cuda.current_stream()
    torch.cuda.synchronize()
    U.profile(["marginal_cost"])  # HIP events around each search launch of the timed solves
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(st)
    for k in range(a.steps):
        out = U.w2_solve(p, s, case.iters, u0)
        print(f"# step {k} done", file=sys.stderr, flush=True)
    ev1.record(st)
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / a.steps
    se_ms, se_n = U.profile_read()["marginal_cost"]
    breakdown = kernel_breakdown(U, lambda: U.w2_solve(p, s, case.iters, u0))
    se_avg_s = se_ms / 1e3 / max(se_n, 1)
    terms = w2_search_terms(p, s, out[0].cpu().numpy())
    achieved = terms * W2_FLOPS_PER_TERM / se_avg_s
    J = out[2].cpu().numpy()
    res = {"metric": "2-D Witsenhausen solves/s", "value": 1e3 / ms_step, "unit": "solves/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": case.name, "n_x": p.n_x, "n_y": p.n_y, "levels": s.levels, "cands": s.cands,
                      "rounds": case.iters, "k": p.k, "sigma": 5.0},
           "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                        "frac": achieved / PEAK_FP64, "traffic": None, "kernel": "k_w2_search (2-D search)",
                        "per_unit": f"{W2_FLOPS_PER_TERM} FP64 flops per windowed term, {terms:.3e} per launch",
                        "kernel_avg_us": se_avg_s * 1e6, "kernel_launches": se_n},
           "kernel_ms_per_step": {"search": breakdown["marginal_cost"], "u1": breakdown["u1"],
                                  "objective": breakdown["objective"]},
           "J_final": float(J[-1]), "J_paper_context": 0.166719}
    if not a.no_cpu:
        res["cpu_baseline"] = w2_cpu_baseline(case)
    print(json.dumps(res), flush=True)


def bench_alg1(a):
    """The paper's generic solver (Algorithm 1): Witsenhausen k = 0.2, sigma =
    5, grids of a.alg1_n nodes on [-25, 25], both controllers initialised to
    the identity (Section III-D), N = 20 iterations per round, r = 2 nodes per
    direction, p = 1e-10 (Section IV), local-update gradient step 0.1; one
    step is one whole solve to termination (or the round cap), FP64."""
    import numpy as np
    import torch

    import paper_1908_04489_amd as U
    import workloads as W

    p = W.gaussian_problem(0.2, 5.0, a.alg1_n, 25.0)
    x = torch.as_tensor(W.nodes(p.x_lo, p.x_hi, p.n_x)).cuda()
    y = torch.as_tensor(W.nodes(p.y_lo, p.y_hi, p.n_y)).cuda()
    name = f"alg1-wits-{p.n_x}"
    print(f"# {name}: N = 20, r = 2, p = 1e-10, identity init", file=sys.stderr, flush=True)
    for w in range(a.warmup):
        U.alg1_solve(p, x, y, max_rounds=a.alg1_rounds)
    st = torch.cuda.current_stream()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(st)
    for k in range(a.steps):
        u0, u1, J, NL = U.alg1_solve(p, x, y, max_rounds=a.alg1_rounds)
        print(f"# step {k} done: {len(NL)} rounds, J = {J[-1].item():.9f}", file=sys.stderr, flush=True)
    ev1.record(st)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / a.steps
    Jh = J.cpu().numpy()
    res = {"metric": "generic-solver (Algorithm 1) solves/s", "value": 1e3 / ms, "unit": "solves/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": name, "n_x": p.n_x, "n_y": p.n_y, "k": 0.2, "sigma": 5.0, "N": 20, "r": 2,
                      "p": 1e-10, "tau": 0.1, "init": "identity", "max_rounds": a.alg1_rounds},
           "rounds": len(NL), "NL_per_round": NL, "J_initial": float(Jh[0]), "J_final": float(Jh[-1]),
           "J_paper_context": 0.166897}
    if not a.no_check:
        import oracle

        Jo = oracle.objective(p, u0.cpu().numpy(), u1.cpu().numpy())
        res["J_final_rel_err_vs_oracle_objective"] = abs(Jh[-1] - Jo) / Jo
    print(json.dumps(res), flush=True)


def w2_cpu_baseline(case):
    """The oracle's 2-D functions, as they stand, on a bounded sample of the
    same workload scaled to one whole solve: the search on evenly spaced
    points (sized to about 10 s), the decoder on evenly spaced y nodes, one
    full objective."""
    import numpy as np

    import oracle

    p, s = case.prob, case.search
    nn, m = p.n_x ** 2, p.n_y ** 2
    u1 = oracle.w2_update_u1(p, case.u0_init)
    rows = np.linspace(0, nn - 1, 16).astype(np.int64)
    t0 = time.perf_counter()
    oracle.w2_argmin(p, s, u1, case.u0_init, rows)
    n = int(min(nn, 16 * 10.0 / max(time.perf_counter() - t0, 1e-6)))
    rows = np.linspace(0, nn - 1, n).astype(np.int64)
    t0 = time.perf_counter()
    oracle.w2_argmin(p, s, u1, case.u0_init, rows)
    t_arg = (time.perf_counter() - t0) * nn / n
    t0 = time.perf_counter()
    oracle.w2_update_u1(p, case.u0_init)
    t_u1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.w2_objective(p, case.u0_init, u1)
    t_j = time.perf_counter() - t0
    solve_s = t_u1 + t_j + case.iters * (t_arg + t_u1 + t_j)
    return {"value": 1.0 / solve_s, "unit": "solves/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"search on {n} of {nn} points ({t_arg * n / nn:.1f} s), one full decoder and objective, "
                      f"scaled to {case.iters} rounds: {solve_s:.0f} s per solve"}


def w2_search_terms(p, s, u0):
    """Windowed noise terms one 2-D search launch sums: level 0 exactly (its
    candidates are the fixed grid), the later levels' and the incumbent's
    K^2 (levels - 1) + 1 candidates counted at the final controller (they
    sit within a few spacings of it)."""
    import numpy as np

    n, ny = p.n_x, p.n_y
    dy = (p.y_hi - p.y_lo) / (ny - 1)
    wn = max(1, min(int(np.floor(10.0 / dy)), ny))
    x = p.x_lo + np.arange(n) * ((p.x_hi - p.x_lo) / (n - 1))

    def width(z):
        c = np.clip(np.rint((z - p.y_lo) / dy), 0, ny - 1)
        return np.minimum(ny - 1, c + wn) - np.maximum(0, c - wn) + 1

    h0 = (s.u_hi - s.u_lo) / (s.cands - 1)
    c0 = s.u_lo + np.arange(s.cands) * h0
    w0 = width(x[:, None] + c0[None, :]).sum(axis=1)  # per coordinate value, summed over candidates
    level0 = float(np.outer(w0, w0).sum())
    wa = width(np.repeat(x, n) + u0[0])
    wb = width(np.tile(x, n) + u0[1])
    later = float((wa * wb).sum()) * (s.cands ** 2 * (s.levels - 1) + 1)
    return level0 + later


def coding_cpu_baseline(case):
    """The oracle's coding functions, as they stand, on a bounded sample of
    the same workload, scaled to one whole solve: an encoder update on evenly
    spaced rows, one full decoder and one full objective."""
    import numpy as np

    import oracle

    p, s = case.prob, case.search
    u1 = oracle.coding_update_u1(p, case.u0_init)
    # probe, then size the encoder sample to about 10 s
    rows = np.linspace(0, p.n_x - 1, 256).astype(np.int64)
    t0 = time.perf_counter()
    oracle.coding_argmin(p, s, u1, case.u0_init, rows)
    n = int(min(p.n_x, 256 * 10.0 / max(time.perf_counter() - t0, 1e-6)))
    rows = np.linspace(0, p.n_x - 1, n).astype(np.int64)
    t0 = time.perf_counter()
    oracle.coding_argmin(p, s, u1, case.u0_init, rows)
    t_arg = (time.perf_counter() - t0) * p.n_x / len(rows)
    t0 = time.perf_counter()
    oracle.coding_update_u1(p, case.u0_init)
    t_u1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.coding_objective(p, case.u0_init, u1)
    t_j = time.perf_counter() - t0
    solve_s = t_u1 + t_j + case.iters * (t_arg + t_u1 + t_j)
    return {"value": 1.0 / solve_s, "unit": "solves/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"encoder update on {len(rows)} of {p.n_x} rows ({t_arg * len(rows) / p.n_x:.1f} s), one "
                      f"full decoder and objective, scaled to {case.iters} rounds: {solve_s:.1f} s per solve"}


def kernel_breakdown(U, step):
    """Milliseconds per kind of kernel in one extra, untimed step with every
    launch bracketed by HIP events (the events themselves add a few
    microseconds per launch, which is why the timed steps time only the
    marginal-cost kernel)."""
    import torch

    torch.cuda.synchronize()
    U.profile(True)
    step()
    torch.cuda.synchronize()
    prof = U.profile_read()
    U.profile(None)
    return {k: v[0] for k, v in prof.items()}


def peak_probe(a):
    """Issue rates of FP32 FMA, the FP32 base-2 exponential and FP64 FMA on
    this GPU (every wave slot busy, 8 independent chains per lane), against
    the published figures: 256 CUs x 128 FP32 lanes x 2.4 GHz = 78.6e12 FP32
    lane-operations/s without packed math, and the FP64 vector rate, half
    of that.  The exponential's cost in FMA slots is the ratio of the two
    FP32 rates."""
    import paper_1908_04489_amd as U

    out = {}
    for kind in ("fma32", "exp32", "fma64"):
        out[kind] = U.peak_probe(kind)
        print(f"# {kind}: {out[kind]:.3e} lane-ops/s", file=sys.stderr, flush=True)
    res = {"metric": "VALU issue rate", "value": out["fma32"], "unit": "lane-ops/s", "n_gpus": 1, "steps": 1,
           "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic", "config": {"workload": "peak-probe", "blocks": 8192, "iters": 4096,
                                                           "chains": 8},
           "fma32_lane_ops_per_s": out["fma32"], "exp32_lane_ops_per_s": out["exp32"],
           "fma64_lane_ops_per_s": out["fma64"], "fma32_frac_of_published": out["fma32"] / PEAK_SLOTS,
           "fma64_frac_of_published": out["fma64"] / (PEAK_SLOTS / 2), "exp32_slots": out["fma32"] / out["exp32"]}
    print(json.dumps(res), flush=True)


def copy_calibration():
    """Plain device-to-device copies of a known size (3 x 256 MiB), run under
    rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE to scale those counters to bytes."""
    import torch

    x = torch.empty(64 << 20, dtype=torch.float32, device="cuda").uniform_()
    for _ in range(3):
        x.clone()
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": 3 * (256 << 20)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="headline",
                    help="headline (64 x 65536 batch + serving + CPU baseline), paper (one 20001-node solve), "
                         "small, batch, serving, sweep, coding, w2, alg1, peak-probe, copy-calibration")
    ap.add_argument("--prec", default="fp32_kahan")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-check", action="store_true", help="skip the FP64 oracle check of the final J")
    ap.add_argument("--no-serving", action="store_true", help="headline: skip the serving leg")
    ap.add_argument("--gt-steps", type=int, default=3,
                    help="headline: timed steps of the same batch in the Gauss-transform arithmetic (0: skip)")
    ap.add_argument("--requests", type=int, default=4096, help="serving: requests taken from the trace")
    ap.add_argument("--slots", type=int, default=64, help="serving: concurrent solves")
    ap.add_argument("--instances", type=int, default=64, help="batch: instances per launch")
    ap.add_argument("--sweep-n", type=int, default=20001, help="sweep: grid nodes")
    ap.add_argument("--sweep-seeds", type=int, default=9, help="sweep: seeds per (k, sigma)")
    ap.add_argument("--sweep-rows", type=int, default=48, help="sweep: sampled rows per check")
    ap.add_argument("--alg1-n", type=int, default=20001, help="alg1: grid nodes")
    ap.add_argument("--alg1-rounds", type=int, default=200, help="alg1: cap on rounds")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (the solver shards over x0 "
              "rows by design, but only the single-GPU kernel is built and measured).", file=sys.stderr)
        sys.exit(2)

    if a.workload == "headline":
        return bench_headline(a)
    if a.workload == "batch":
        a.no_serving = True
        return bench_headline(a)
    if a.workload == "serving":
        return bench_serving(a)
    if a.workload == "sweep":
        return bench_sweep(a)
    if a.workload == "coding":
        return bench_coding(a)
    if a.workload == "w2":
        return bench_w2(a)
    if a.workload == "peak-probe":
        return peak_probe(a)
    if a.workload == "alg1":
        return bench_alg1(a)
    if a.workload == "copy-calibration":
        return copy_calibration()

    import numpy as np
    import torch

    import paper_1908_04489_amd as U

    case = workload(a.workload)
    p, s = case.prob, case.search
    u0 = torch.as_tensor(case.u0_init).cuda()
    print(f"# workload {case.name}: n={p.n_x}, {s.levels}x{s.cands}, {case.iters} rounds, {a.prec}", file=sys.stderr,
          flush=True)
    for w in range(a.warmup):
        U.solve(p, s, case.iters, u0, a.prec)
        print(f"# warmup {w} done", file=sys.stderr, flush=True)
    st = torch.cuda.current_stream()
    torch.cuda.synchronize()
    U.profile(["marginal_cost"])  # HIP events around each marginal-cost launch of the timed solves
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(st)
    terms = evaluated = evals = 0
    for k in range(a.steps):
        out = U.solve(p, s, case.iters, u0, a.prec)
        t_, v_, e_ = U.last_counts()
        terms += t_
        evaluated += v_
        evals += e_
    ev1.record(st)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    ms_step = ms / a.steps
    mc_ms, mc_n = U.profile_read()["marginal_cost"]
    breakdown = kernel_breakdown(U, lambda: U.solve(p, s, case.iters, u0, a.prec))
    mc_avg_s = mc_ms / 1e3 / max(mc_n, 1)
    achieved = terms / max(mc_n, 1) * SLOTS_PER_TERM / mc_avg_s
    value = terms / (ms / 1e3)
    C = s.levels * s.cands + 1
    dense = float(p.n_x) * C * p.n_y * case.iters
    res = {
        "metric": "marginal-cost quadrature terms/s",
        "value": value,
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": case.name, "n_x": p.n_x, "n_y": p.n_y, "levels": s.levels, "cands": s.cands,
                   "rounds": case.iters, "k": p.k, "sigma": case.sigma, "prec": a.prec},
        "alg_terms_per_step": terms / a.steps,
        "evaluated_terms_per_step": evaluated / a.steps,
        "fp64_tie_evals_per_step": evals / a.steps,
        "dense_equiv_terms_per_s": dense / (ms_step / 1e3),
        "solves_per_s": 1e3 / ms_step,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS / 1e12,
                     "unit": "Tslot/s", "frac": achieved / PEAK_SLOTS, "traffic": measured_traffic(case.name),
                     "kernel": "k_mc32<FP32_KAHAN> (marginal-cost window sums)",
                     "per_unit": f"{SLOTS_PER_TERM} FP32 VALU slots per algorithmic term",
                     "kernel_avg_us": mc_avg_s * 1e6, "kernel_launches": mc_n,
                     "kernel_terms_per_s": terms / max(mc_n, 1) / mc_avg_s},
        "kernel_ms_per_step": breakdown,
    }
    J = out[2].cpu().numpy()
    res["J_final"] = float(J[-1])
    if not a.no_check:
        import oracle

        Jo = oracle.objective(p, out[0].cpu().numpy(), out[1].cpu().numpy())
        res["J_final_rel_err_vs_oracle_objective"] = abs(J[-1] - Jo) / Jo
    if not a.no_cpu:
        res["cpu_baseline"] = cpu_baseline([case])
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
