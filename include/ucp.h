/*
 * ucp.h - C ABI of the MI355X marginal-cost solver for Witsenhausen's
 * counterexample (Tseng, "A Generic Solver for Unconstrained Control
 * Problems with Integral Functional Objectives").
 *
 * The problem (Section V-A): x0 ~ prior f (the paper's N(0, sigma^2), or a
 * Gaussian mixture), y0 = x0, x1 = x0 + u0(y0), y1 = x1 + w with
 * w ~ N(0, 1), x2 = x1 - u1(y1), minimise J = E[k^2 u0(y0)^2 + x2^2].
 * Controllers are step functions on linearly spaced grids (Section III-D,
 * "Initialization"); integrals are rectangle-rule sums over the grid nodes.
 *
 * Conventions for every call below:
 *  - Array arguments are DEVICE pointers (memory on the handle's GPU),
 *    FP64, contiguous, owned by the caller.  The library never frees or
 *    keeps them past the call's stream work.  The library owns only the
 *    workspace held inside the handle.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls enqueue work on it and return without synchronising, except
 *    where stated; results are valid once the stream has reached them.
 *  - Return value: UCP_OK (0) or a negative error code; on error nothing was
 *    enqueued and ucp_last_error() returns a message (thread-local).
 *  - A handle is not thread-safe: use one handle per host thread.  Calls on
 *    one handle must share one stream or be ordered by the caller, because
 *    they share the handle's workspace.
 */
#ifndef UCP_H_
#define UCP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define UCP_MAX_COMP 8
#define UCP_MAX_LEVELS 16
#define UCP_MAX_CANDS 63

enum {
  UCP_OK = 0,
  UCP_EINVAL = -1,     /* invalid argument (null pointer, bad size or parameter) */
  UCP_ENOMEM = -2,     /* device allocation failed / over the memory budget */
  UCP_EHIP = -3,       /* a HIP runtime call failed (no device, launch failure) */
  UCP_EAGAIN = -4,     /* server: not admitted yet / result not ready */
  UCP_ENONFINITE = -5, /* a solve produced non-finite values (e.g. NaN input) */
  UCP_ENOTFOUND = -6   /* server: unknown or already collected ticket */
};

/* Arithmetic of the bulk marginal-cost and u1 sums. */
typedef enum {
  UCP_FP32 = 0,       /* FP32 terms, plain FP32 accumulation */
  UCP_FP32_KAHAN = 1, /* FP32 terms, compensated (Kahan) accumulation */
  UCP_FP64 = 2,       /* FP64 throughout */
  UCP_FP64_GT = 3     /* FP64 marginal costs from a Gauss transform of u1 (below) */
} ucp_prec;

/* The moment table (Gauss transform of u1).  The marginal cost depends on
 * (u, x0) only through z = x0 + u (besides k^2 u^2), and about any centre c,
 * with delta = z - c, d = delta / s and t_j = (y_j - c) / s,
 *   dy sum_j phi_s(y_j - z)(z - u1_j)^2
 *     = dy/(s sqrt(2 pi)) e^{-d^2/2} sum_n d^n / n!
 *       [A2_n + 2 delta A1_n + delta^2 A0_n](c),
 *   A_a,n(c) = sum_j e^{-t_j^2/2} t_j^n (c - u1_j)^a
 * (the Gaussian's shift expanded in powers of d).  After each u1 update
 * one FP64 pass over the window (11 noise sds) of each centre tabulates A
 * for n <= 12; the centres are every m-th y node, m the largest stride
 * with m dy / s <= 0.05 for which the series' truncation bound x^13 / 13! /
 * (1 - x / 14), x = (m dy / 2s) (window in noise sds), is below 1e-17 (m =
 * 40 on a 65536-node grid over [-40, 40] with s = 1), from 11 noise sds
 * before the grid to 11 past it.  Every position then costs O(12); one
 * farther outside has no grid node within its window and a noise sum of
 * 0.  The table differs from
 * the dense sum by the truncation, the window's tail and rounding (about
 * 1e-16 of the cost at the centre; measured within 1e-14 of the dense sum).
 *
 * UCP_FP64_GT evaluates every marginal cost from the table and decides on
 * those FP64 values; its u1 update and objective are those of UCP_FP64.
 * Grids with dy / noise_sd > 0.05 are refused (UCP_EINVAL); so is
 * ucp_argmin_adaptive_noalloc in this mode.
 * In the FP32 modes the searches (solves, ucp_argmin_adaptive, the server)
 * take the FP64 values that decide FP32 near-ties from the table where
 * dy / noise_sd <= 0.05, and from FP64 window sums otherwise; L_0 of a
 * winner that needed no FP64 value comes from a window sum. */

/* Problem instance: weight k of the stage-1 cost, the prior of x0 as a
 * mixture of n_comp Gaussians (weights w summing to 1, means mu, standard
 * deviations sd > 0), the x0 grid (n_x nodes on [x_lo, x_hi]) and the y1
 * grid (n_y nodes on [y_lo, y_hi]), 2 <= n_x, n_y <= 2^24, and the
 * standard deviation noise_sd of the Gaussian noise w (Section V-A fixes 1;
 * 0 also selects 1; otherwise 1e-6 <= noise_sd <= 1e6).  Node i of a grid
 * is lo + i * ((hi - lo) / (n - 1)) in binary64.  Every window below is
 * measured in noise standard deviations. */
typedef struct ucp_problem {
  double k;
  int32_t n_comp;
  int32_t pad_;
  double w[UCP_MAX_COMP];
  double mu[UCP_MAX_COMP];
  double sd[UCP_MAX_COMP];
  double x_lo, x_hi;
  int64_t n_x;
  double y_lo, y_hi;
  int64_t n_y;
  double noise_sd;
} ucp_problem;

/* Coarse-to-fine search of argmin_u L_0(u, x0) per point: level 0 takes
 * `cands` equally spaced candidates on [u_lo, u_hi] (spacing
 * h0 = (u_hi - u_lo) / (cands - 1)); level l takes `cands` equally spaced
 * candidates on [c* - h_{l-1}, c* + h_{l-1}] clamped to [u_lo, u_hi]
 * (h_l = 2 h_{l-1} / (cands - 1)), c* being the best so far, which stays in
 * the comparison; the incumbent u0(x0) is compared last and kept on ties.
 *
 * tie_rel64: relative tie band of the selection rule (FP64 values within
 * m (1 + tie_rel64) of the minimum m are ties); 0 selects 1e-12.  Finite,
 * 0 <= tie_rel64 <= 1e-3.
 * band_rel32: relative part tau of the FP32 pre-selection band of the FP32
 * modes, B32 <= m32 (1 + tau + tie_rel64) + 6e-7 sqrt(m32); 0 selects
 * 5e-7 with compensated sums and 5e-6 with plain sums, the widths that
 * keep the FP64 minimum in the band (a narrower band is faster and may
 * drop it).  Finite, 0 <= band_rel32 <= 1e-2.  Ignored in FP64 mode.
 * A zero-initialised record's two fields select the defaults. */
typedef struct ucp_search {
  double u_lo, u_hi;
  int32_t levels; /* 1 .. UCP_MAX_LEVELS */
  int32_t cands;  /* 2 .. UCP_MAX_CANDS */
  double tie_rel64;
  double band_rel32;
} ucp_search;

typedef struct ucp_handle ucp_handle;

/* Library version string. */
const char* ucp_version(void);

/* Message of the last error on the calling thread ("" if none). */
const char* ucp_last_error(void);

/* Create a handle on HIP device `device`.  Allocates no device memory yet;
 * the workspace grows on first use, never beyond `hbm_budget` bytes
 * (0 = no limit): a call whose workspace would exceed it fails with
 * UCP_ENOMEM and enqueues nothing.  Errors: UCP_EINVAL (null out, no such
 * device), UCP_EHIP (no HIP device). */
int ucp_create(ucp_handle** out, int device, size_t hbm_budget);

/* Release the handle and its workspace (synchronises the device first).
 * NULL is a no-op. */
void ucp_destroy(ucp_handle* h);

/* Marginal cost of the first controller (Section III-A, definition of C_m
 * applied to the Section V-A objective):
 *   L0_out[i*n_cand + c] = f(x_i) * ( k^2 u^2
 *        + dy * sum_j phi(y_j - x_i - u) (x_i + u - u1[j])^2 ),
 *   u = u[i*n_cand + c], phi the N(0, noise_sd^2) density.
 * u1: [n_y]; u: [n_x * n_cand] row-major per point; L0_out: [n_x * n_cand].
 * The sum runs over the nodes within 9 (FP32 modes) or 11 (FP64) noise
 * standard deviations of the node nearest x_i + u, scaled by the Gaussian
 * at that node (max-shift).  The omitted tail is below
 * 2 phi(W)/W max_j (x_i + u - u1[j])^2 for a window of W sds: 2.6e-19 of
 * that square at W = 9 (far below the FP32 sums' rounding), 3.9e-28 at
 * W = 11 (below 1e-16 of the FP64 result wherever it exceeds 4e-12 of
 * that square).
 * Errors: UCP_EINVAL for null pointers, n_cand < 1, invalid problem. */
int ucp_marginal_cost(ucp_handle* h, const ucp_problem* prob, ucp_prec prec,
                      const double* u1, const double* u, int64_t n_cand,
                      double* L0_out, void* stream);

/* One pointwise improvement of u0 (Corollary 1 with the update rule of
 * Section III-B, all points in parallel as in Section IV-A): for every x_i
 * the coarse-to-fine search of ucp_search over u of
 * B(u; x_i) = L_0(u, x_i) / f(x_i), with u1 held fixed.
 * Selection at every level and at the final comparison with the incumbent:
 * the candidates within the relative band tie_rel64 (default 1e-12) of the
 * minimum (in FP64) are ties, the one nearest u0_in[i] wins, then the
 * smaller u.  In the FP32 modes the minimum and band are first found in
 * FP32 - the band is B <= m (1 + tau + tie_rel64) + 6e-7 sqrt(m), tau =
 * band_rel32 (default 5e-7 with compensated sums and 5e-6 with plain sums)
 * - and the band members are re-evaluated in FP64 (window of 11 sds)
 * before the rule is applied.
 * u1: [n_y]; u0_in, u0_out: [n_x] (may alias); L0_out: [n_x] or NULL - if
 * given, receives f(x_i) * B(u0_out[i]; x_i) evaluated in FP64.
 * Errors: UCP_EINVAL (null pointers, invalid problem or search). */
int ucp_argmin_adaptive(ucp_handle* h, const ucp_problem* prob, const ucp_search* search,
                        ucp_prec prec, const double* u1, const double* u0_in,
                        double* u0_out, double* L0_out, void* stream);

/* ucp_argmin_adaptive for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops and harnesses that forbid
 * hipMalloc): the same update, kernels and results, with the workspace
 * taken from a fixed 64 MiB device array that the library holds on each
 * GPU it runs on until the process ends, instead of the handle's
 * workspace.  The call allocates nothing (no hipMalloc, hipFree, pinned
 * host memory or library routine that allocates) and issues no
 * hipMemsetAsync; the caller passes every input and output as for
 * ucp_argmin_adaptive (u0_in and u0_out may alias).  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams,
 * other handles or threads) race and must be ordered by the caller.
 * Errors: as ucp_argmin_adaptive, and UCP_EINVAL when the problem needs
 * more scratch than the array holds (64 MiB: the 20001-node grid with
 * 5 x 16 candidates needs 14.2 MiB, the 65536-node grid with 4 x 32 needs
 * 36.8 MiB; the need grows with n_x (cands + 1) times the window segments). */
int ucp_argmin_adaptive_noalloc(ucp_handle* h, const ucp_problem* prob, const ucp_search* search,
                                ucp_prec prec, const double* u1, const double* u0_in,
                                double* u0_out, double* L0_out, void* stream);

/* Second controller by its closed form, the conditional mean
 * u1(y_j) = sum_i x1_i f_i phi(y_j - x1_i) / sum_i f_i phi(y_j - x1_i),
 * x1_i = x_i + u0[i], the exact minimiser of the discrete marginal cost
 * C_1 (the closed form the paper credits to the earlier solver, Section
 * IV-B).  Weights are max-shifted per y_j.  The logits are FP64; in the FP32
 * modes each weight is the FP32 exponential of its FP64 logit, in FP64 mode
 * the FP64 one.  On grids of at least 16384 y nodes spaced at most 0.05
 * noise sds, three of every four consecutive nodes take their weights as
 * the previous node's times an FP64 ratio per x node, exp2(-log2(e) dy
 * (y_c - x1_i) / s^2) (a common factor per node cancels in the ratio), so
 * one exponential serves four nodes.  Numerator and denominator are FP64 sums in every mode
 * (the two FP32 modes give the same u1): u1 feeds every later marginal
 * cost, and an FP32 numerator would move it by ~1e-7 |x1|, far beyond the
 * FP64 tie band of the decisions that follow.
 * u0: [n_x]; u1_out: [n_y].  Errors: UCP_EINVAL. */
int ucp_update_u1(ucp_handle* h, const ucp_problem* prob, ucp_prec prec,
                  const double* u0, double* u1_out, void* stream);

/* Objective of Section V-A by the rectangle rule, in FP64:
 * J = dx * sum_i f_i [k^2 u0_i^2 + dy * sum_j phi(y_j - x1_i)(x1_i - u1_j)^2].
 * u0: [n_x]; u1: [n_y]; J_out: one double on the device.
 * Errors: UCP_EINVAL. */
int ucp_objective(ucp_handle* h, const ucp_problem* prob, const double* u0,
                  const double* u1, double* J_out, void* stream);

/* The solve loop: u1 <- closed form of u0_init, J_hist[0] = J; then
 * `iters` rounds of (ucp_argmin_adaptive on u0, ucp_update_u1), with
 * J_hist[t] taken after round t.  This is the per-controller loop of
 * Algorithm 1 with the two controllers visited in order, run for a fixed
 * number of rounds; every step stays on the device.  It is ucp_solve_batch
 * with B = 1 and, like it, synchronises the stream before returning (it
 * reads the work counters and the non-finite flag).
 * u0_init, u0_out: [n_x]; u1_out: [n_y]; J_hist: [iters + 1].
 * Errors: UCP_EINVAL (iters < 0, invalid inputs), UCP_ENONFINITE. */
int ucp_solve(ucp_handle* h, const ucp_problem* prob, const ucp_search* search, ucp_prec prec,
              int32_t iters, const double* u0_init, double* u0_out, double* u1_out,
              double* J_hist, void* stream);

/* Work counters of the last ucp_solve / ucp_solve_batch on this handle
 * (any pointer may be NULL): `terms` = algorithmic marginal-cost terms,
 * the (point, candidate, y node) triples with |y_j - x_i - u| <= 9 over
 * every level and round (the work the method needs); `evaluated` = the
 * terms the FP32 kernels actually summed (windows around the nearest node,
 * which for x_i + u outside the y grid still cover the nodes near its
 * edge); `fp64_evals` = FP64 re-evaluations of FP32 tie-band members.
 * Errors: UCP_EINVAL. */
int ucp_last_counts(ucp_handle* h, uint64_t* terms, uint64_t* evaluated, uint64_t* fp64_evals);

/* Kernel timing: ucp_solve / ucp_solve_batch record a pair of HIP events on
 * the caller's stream around each launch of every kind selected in the
 * profiling mask: the marginal-cost kernel (UCP_PROF_MC), the selection
 * kernels (UCP_PROF_SELECT), the u1 kernels (UCP_PROF_U1) and the
 * objective kernels (UCP_PROF_J); totals accumulate until the mask is set
 * again.  ucp_profile(h, mask) sets the mask (bit 1 << kind per kind, 0 =
 * off, UCP_PROF_ALL = every kind) and resets the totals; ucp_profile_read
 * returns the total milliseconds and the launch count of one kind.  Each
 * timed launch costs a few microseconds of stream time for its events, so
 * time only the kinds needed.  Errors: UCP_EINVAL (unknown kind bits). */
#define UCP_PROF_MC 0
#define UCP_PROF_SELECT 1
#define UCP_PROF_U1 2
#define UCP_PROF_J 3
#define UCP_PROF_KINDS 4
#define UCP_PROF_ALL 15
int ucp_profile(ucp_handle* h, int enable);
int ucp_profile_read(ucp_handle* h, int kind, double* total_ms, int64_t* launches);

/* Diagnostic, not part of the solver: the issue rate of one VALU operation
 * the kernels are built from - kind 0 FP32 FMA, 1 the FP32 base-2
 * exponential, 2 FP64 FMA - as lane-operations per second, with `blocks`
 * blocks of 256 lanes each running 8 independent chains of `iters`
 * operations (a second, timed launch after a warm-up) on HIP device
 * `device`.  Allocates a small
 * device buffer and synchronises `stream`.  This fixes the VALU peak the
 * marginal-cost kernel's roofline is quoted against.
 * Errors: UCP_EINVAL, UCP_ENOMEM, UCP_EHIP. */
int ucp_peak_probe(int device, int kind, int32_t blocks, int32_t iters, double* lane_ops_per_s, void* stream);

/* B independent solves advanced together: every kernel launch covers all
 * instances still running (one flat work list per launch), each instance
 * with its own problem, search and iteration count.  Per-instance results
 * are bitwise identical to ucp_solve on that instance alone.
 * All pointer arrays have B entries (host arrays of device pointers).
 * Errors: UCP_EINVAL.  Synchronises the stream before returning. */
int ucp_solve_batch(ucp_handle* h, int32_t B, const ucp_problem* probs,
                    const ucp_search* searches, ucp_prec prec, const int32_t* iters,
                    const double* const* u0_init, double* const* u0_out,
                    double* const* u1_out, double* const* J_hist, void* stream);

/* ---- The paper's generic solver (Algorithm 1, Sections III-B to III-D) --
 * Both controllers are improved by the paper's own methods instead of the
 * coarse-to-fine search and the closed form: local updates (a modified
 * Newton step on each point's marginal cost) and partial exhaustion (each
 * point takes the best of the values its controller holds at the grid
 * nodes within r of it, the domain-ball set of Eq. (2)), the N iterations
 * of each round shared between the two by their last improvements, until
 * a round improves J by at most p.  Everything is FP64; the windows are
 * those of the FP64 sums above (11 noise sds).  Readings where the paper is
 * silent: the local update of u0 works on B = L_0 / f (the Newton step is
 * the same; the gradient step u - tau B' does not vanish where f
 * underflows); a phase's improvement is |J before - J after|; partial
 * exhaustion compares candidates by the selection rule of the search
 * (relative tie band, nearest to the point's own value, then the smaller
 * u), every point of a controller from the same previous array; the local
 * update of u1 is the Newton step of the quadratic C_1, i.e. exactly the
 * closed form ucp_update_u1 computes in FP64 mode. */
typedef struct ucp_alg1_params {
  int32_t N;          /* iterations per round, >= 2 (the paper: 20) */
  int32_t r;          /* partial-exhaustion radius in grid nodes: 1 or 2 (the paper: 2) */
  double p;           /* precision: stop once a round's two improvements sum to <= p (the paper: 1e-10) */
  double tau;         /* gradient step where the curvature is not positive, > 0 */
  double tie_rel64;   /* relative tie band of partial exhaustion; 0 selects 1e-12 */
  int32_t max_rounds; /* cap on rounds, >= 1 */
  int32_t pad_;
} ucp_alg1_params;

/* One local update of u0 (Section III-D, Local Update): for every x_i, with
 * u = u0_in[i] and B'(u), B''(u) the first two derivatives of
 * B(u; x_i) = L_0(u, x_i) / f(x_i) (Gaussian-weighted moments over the
 * window), u0_out[i] = u - B'/B'' where B'' > 0, else u - tau B'.
 * u1: [n_y]; u0_in, u0_out: [n_x] (may alias).  Errors: UCP_EINVAL. */
int ucp_alg1_local_u0(ucp_handle* h, const ucp_problem* prob, double tau, const double* u1,
                      const double* u0_in, double* u0_out, void* stream);

/* One partial exhaustion of u0 (Section III-D, Partial Exhaustion, and
 * Eq. (2)): u0_out[i] = the best, by B(.; x_i) and the selection rule, of
 * u0_in at the nodes i - r .. i + r of the grid.  u0_in, u0_out may alias.
 * Errors: UCP_EINVAL (also r not 1 or 2). */
int ucp_alg1_pe_u0(ucp_handle* h, const ucp_problem* prob, double tie_rel64, int32_t r, const double* u1,
                   const double* u0_in, double* u0_out, void* stream);

/* One partial exhaustion of u1: u1_out[j] = the best of u1_in at the nodes
 * j - r .. j + r by C_1(u, y_j) = dx sum_i f_i phi(y_j - x1_i)(x1_i - u)^2
 * (x1 = x + u0), with the weights max-shifted per y_j (a positive factor
 * per node, which changes neither the order nor the relative band).
 * u1_in, u1_out may alias.  Errors: UCP_EINVAL. */
int ucp_alg1_pe_u1(ucp_handle* h, const ucp_problem* prob, double tie_rel64, int32_t r, const double* u0,
                   const double* u1_in, double* u1_out, void* stream);

/* Algorithm 1 from (u0_init, u1_init) (the paper initialises both to the
 * identity): J_log (device, [1 + 2 max_rounds]) receives J initially and
 * after each phase (local updates, then partial exhaustion) of each round;
 * NL_log (HOST, [max_rounds], or NULL) the local-update iterations of each
 * round; *rounds_out (HOST) the rounds run.  Reads J back after every
 * phase and synchronises the stream before returning.
 * Errors: UCP_EINVAL, UCP_ENONFINITE. */
int ucp_alg1_solve(ucp_handle* h, const ucp_problem* prob, const ucp_alg1_params* params,
                   const double* u0_init, const double* u1_init, double* u0_out, double* u1_out,
                   double* J_log, int32_t* NL_log, int32_t* rounds_out, void* stream);

/* ---- Zero-delay source-channel coding (Section V-B) --------------------
 * x0 ~ prior f (the paper's N(0, 1), or a Gaussian mixture), y0 = x0,
 * x1 = u0(y0) + w with w ~ U(-1, 1), y1 = x1; minimise
 * J = E[lam u0(y0)^2 + (u1(y1) - x0)^2] (the paper's figure: lam = 2).
 * The same grids, rectangle rule, conventions and error codes as above; the
 * noise density is p_w(t) = 1/2 for |t| <= 1 (end points included) and 0
 * otherwise, the test evaluated in binary64 as fabs(y_j - v) <= 1 with
 * y_j = y_lo + j * dy.  Everything is FP64. */
typedef struct ucp_coding_problem {
  double lam; /* weight of the encoder's power, finite and >= 0 */
  int32_t n_comp;
  int32_t pad_;
  double w[UCP_MAX_COMP];
  double mu[UCP_MAX_COMP];
  double sd[UCP_MAX_COMP];
  double x_lo, x_hi;
  int64_t n_x;
  double y_lo, y_hi;
  int64_t n_y;
} ucp_coding_problem;

/* Marginal cost of the encoder (Section III-A, C_0 of the coding
 * objective):
 *   L0_out[i*n_cand + c] = f(x_i) * ( lam u^2
 *        + dy * sum_j p_w(y_j - u) (u1[j] - x_i)^2 ),  u = u[i*n_cand + c].
 * The window sum is taken from double-double prefix sums of u1 and u1^2
 * over the nodes with |y_j - u| <= 1 (exact window membership).
 * u1: [n_y]; u: [n_x * n_cand]; L0_out: [n_x * n_cand].
 * Errors: UCP_EINVAL (null pointers, n_cand outside 1..4096, invalid
 * problem). */
int ucp_coding_marginal_cost(ucp_handle* h, const ucp_coding_problem* prob, const double* u1,
                             const double* u, int64_t n_cand, double* L0_out, void* stream);

/* One pointwise improvement of u0 with u1 fixed: the coarse-to-fine search
 * and the selection rule of ucp_argmin_adaptive (relative tie band
 * tie_rel64, default 1e-12,
 * nearest to u0_in[i], then the smaller u; the incumbent compared last),
 * every B evaluated in FP64 as in ucp_coding_marginal_cost.
 * u1: [n_y]; u0_in, u0_out: [n_x] (may alias); L0_out: [n_x] or NULL
 * (receives f(x_i) B(u0_out[i]; x_i)).  Errors: UCP_EINVAL. */
int ucp_coding_argmin(ucp_handle* h, const ucp_coding_problem* prob, const ucp_search* search,
                      const double* u1, const double* u0_in, double* u0_out, double* L0_out,
                      void* stream);

/* Decoder by its closed form, the conditional mean
 * u1(y_j) = sum_i f_i p_w(y_j - u0_i) x_i / sum_i f_i p_w(y_j - u0_i),
 * and u1(y_j) = 0 where no x node has |y_j - u0_i| <= 1 (no probability
 * reaches y_j).  u0: [n_x]; u1_out: [n_y].  Errors: UCP_EINVAL. */
int ucp_coding_update_u1(ucp_handle* h, const ucp_coding_problem* prob, const double* u0,
                         double* u1_out, void* stream);

/* Objective of Section V-B by the rectangle rule, in FP64:
 * J = dx * sum_i f_i [lam u0_i^2 + dy * sum_j p_w(y_j - u0_i)(u1_j - x_i)^2].
 * u0: [n_x]; u1: [n_y]; J_out: one double on the device.  Errors: UCP_EINVAL. */
int ucp_coding_objective(ucp_handle* h, const ucp_coding_problem* prob, const double* u0,
                         const double* u1, double* J_out, void* stream);

/* The solve loop of ucp_solve for the coding problem: u1 <- closed form of
 * u0_init, J_hist[0] = J, then `iters` rounds of (ucp_coding_argmin,
 * ucp_coding_update_u1) with J_hist[t] after round t.  Under ucp_profile
 * the launches are timed with the kinds UCP_PROF_MC (the u0 search),
 * UCP_PROF_SELECT (the prefix sums), UCP_PROF_U1 and UCP_PROF_J, and the
 * call synchronises the stream before returning; otherwise it does not.
 * u0_init, u0_out: [n_x] (may alias); u1_out: [n_y]; J_hist: [iters + 1].
 * Errors: UCP_EINVAL. */
int ucp_coding_solve(ucp_handle* h, const ucp_coding_problem* prob, const ucp_search* search,
                     int32_t iters, const double* u0_init, double* u0_out, double* u1_out,
                     double* J_hist, void* stream);

/* ---- Two-dimensional Witsenhausen counterexample (Section V-D) ---------
 * x0 in R^2 with both coordinates independent draws of the prior of
 * `prob`, x1 = x0 + u0(x0), y1 = x1 + w with w ~ N(0, I_2),
 * x2 = x1 - u1(y1); minimise J = 1/2 E[k^2 |u0|^2 + |x2|^2] (the paper:
 * k = 0.2, sigma = 5 on 160 x 160 nodes).  The grids are tensor products:
 * x node (i1, i2) at index i1 * n_x + i2, y node (j1, j2) at j1 * n_y + j2,
 * at most 4096 nodes per coordinate, prob->noise_sd 0 or 1 (the noise is
 * N(0, I_2)); rectangle rule with weights dx^2 and
 * dy^2.  Vector fields are two planes: [2][n_x^2] for u0, [2][n_y^2] for
 * u1 (first coordinates, then second).  FP64 throughout.  The noise sums
 * run over the floor(10 / dy) nodes on either side of the node nearest
 * x + u in each coordinate, at least 10 - 1.5 dy noise standard deviations
 * (omitted weight below 1e-18 relative for dy <= 1). */

/* L0_out[i*n_cand + c] = f(x_i1) f(x_i2) B(u; x_i) with
 * B = 1/2 [k^2 |u|^2 + dy^2 sum_j phi(y_j1 - z1) phi(y_j2 - z2) |z - u1(y_j)|^2],
 * z = x_i + u, u = (u[i*n_cand + c], u[n_x^2 * n_cand + i*n_cand + c]).
 * u1: [2][n_y^2]; u: [2][n_x^2][n_cand]; L0_out: [n_x^2][n_cand].
 * Errors: UCP_EINVAL (null pointers, n_cand outside 1..4096, invalid or too
 * large problem). */
int ucp_w2_marginal_cost(ucp_handle* h, const ucp_problem* prob, const double* u1, const double* u,
                         int64_t n_cand, double* L0_out, void* stream);

/* One pointwise improvement of u0 with u1 fixed: the coarse-to-fine search
 * over the K x K tensor grid of candidates per level (K = cands <= 8;
 * level 0 on [u_lo, u_hi]^2, level l on c* -/+ h_{l-1} in each coordinate,
 * clamped; the best so far carried; spacings as in ucp_search), then the
 * incumbent.  Selection: the candidates within the relative band tie_rel64
 * (default 1e-12) of the minimum are ties; the nearest to u0_in (squared distance) wins, then
 * the smaller first coordinate, then the smaller second, then the earlier
 * candidate (index q1 * K + q2, the best so far last).
 * u0_in, u0_out: [2][n_x^2] (may alias); L0_out: [n_x^2] or NULL.
 * Errors: UCP_EINVAL (also cands > 8). */
int ucp_w2_argmin(ucp_handle* h, const ucp_problem* prob, const ucp_search* search, const double* u1,
                  const double* u0_in, double* u0_out, double* L0_out, void* stream);

/* u1(y_j) = E[x1 | y1 = y_j] = sum_i f_i phi2(y_j - x1_i) x1_i / sum_i f_i phi2(y_j - x1_i),
 * x1_i = x_i + u0_i, phi2 the N(0, I_2) density; the weights are
 * max-shifted (log f(x_i1) + log f(x_i2) - |y_j - x1_i|^2 / 2).
 * u0: [2][n_x^2]; u1_out: [2][n_y^2].  Errors: UCP_EINVAL. */
int ucp_w2_update_u1(ucp_handle* h, const ucp_problem* prob, const double* u0, double* u1_out,
                     void* stream);

/* J = dx^2 sum_i f(x_i1) f(x_i2) B(u0_i; x_i), in FP64.
 * u0: [2][n_x^2]; u1: [2][n_y^2]; J_out: one double.  Errors: UCP_EINVAL. */
int ucp_w2_objective(ucp_handle* h, const ucp_problem* prob, const double* u0, const double* u1,
                     double* J_out, void* stream);

/* The solve loop of ucp_solve in 2-D (u1 from u0_init, J_hist[0], then
 * `iters` rounds of ucp_w2_argmin and ucp_w2_update_u1 with J after each).
 * Profiling kinds as for ucp_coding_solve (UCP_PROF_MC = the search).
 * u0_init, u0_out: [2][n_x^2] (may alias); u1_out: [2][n_y^2];
 * J_hist: [iters + 1].  Errors: UCP_EINVAL. */
int ucp_w2_solve(ucp_handle* h, const ucp_problem* prob, const ucp_search* search, int32_t iters,
                 const double* u0_init, double* u0_out, double* u1_out, double* J_hist, void* stream);

/* ---- Continuous-batching server --------------------------------------
 * Requests (HOST arrays) are admitted while the number of running solves is
 * below `max_slots` and their device footprint fits in `hbm_budget` bytes;
 * each call to ucp_server_step() admits what fits, runs one round
 * (u0 update + u1 update + objective) for every running solve in shared
 * launches, and retires the finished ones (results copied to host).
 * Results are bitwise identical to ucp_solve of the same request alone. */
typedef struct ucp_server ucp_server;

/* Device bytes one solve of this problem and search needs (state and
 * partial sums) at precision `prec` for `iters` rounds: the footprint the
 * server's admission test uses.  Errors: UCP_EINVAL. */
int ucp_footprint(const ucp_problem* prob, const ucp_search* search, ucp_prec prec, int32_t iters,
                  size_t* bytes);

/* Create a server on `device`.  hbm_budget = 0 means no memory limit. */
int ucp_server_create(ucp_server** out, int device, size_t hbm_budget, int32_t max_slots, ucp_prec prec);
void ucp_server_destroy(ucp_server* s);

/* Queue a request; u0_init is a host array [n_x], copied at submission.
 * Returns a ticket (> 0).  Errors: UCP_EINVAL, UCP_ENOMEM (a request that
 * can never fit the budget). */
int ucp_server_submit(ucp_server* s, const ucp_problem* prob, const ucp_search* search,
                      int32_t iters, const double* u0_init, int64_t* ticket);

/* Admit, run one round for all running solves, retire finished ones.
 * *n_running (may be NULL) receives the number of solves still running.
 * Synchronises the server's stream. */
int ucp_server_step(ucp_server* s, int32_t* n_running);

/* Collect a finished request: u0_out [n_x], u1_out [n_y], J_hist [iters+1]
 * are HOST arrays (any may be NULL).  UCP_EAGAIN while queued or running,
 * UCP_ENOTFOUND for an unknown ticket, UCP_ENONFINITE if the solve produced
 * non-finite values (its outputs are still copied). */
int ucp_server_poll(ucp_server* s, int64_t ticket, double* u0_out, double* u1_out, double* J_hist);

/* Cancel a queued or running request (its slot is freed at once). */
int ucp_server_cancel(ucp_server* s, int64_t ticket);

/* Counts: queued, running, finished-but-uncollected. */
int ucp_server_stats(ucp_server* s, int32_t* queued, int32_t* running, int32_t* done);

#ifdef __cplusplus
}
#endif
#endif /* UCP_H_ */
