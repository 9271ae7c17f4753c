// HIP kernels (gfx950) of the marginal-cost solver for Witsenhausen's
// counterexample.
//
// Every kernel takes a flat list of work units over a batch of independent
// instances (Launch: device instance table + prefix sums of units per
// instance); a block finds its instance by binary search over the prefix
// sums.  A single solve is the batch of one.  Nothing here depends on which
// other instances share a launch, so each instance's results are the same
// alone and in a batch.
//
// Kernels (all per Section IV-A: the points of one controller are
// independent, the two controllers are updated one after the other):
//   k_prior        prior density f and log f at the x nodes (FP64)
//   k_mc32<P>      marginal-cost window sums for one level of the search,
//                  FP32 terms, plain (P=0) or compensated (P=1) sums
//   k_mc64         the same in FP64 (precision-study mode)
//   k_gt_table     moment table of the noise sum (a Gauss transform of u1,
//                  Section III-A on the Section V-A cost), after each u1
//                  update
//   k_mc_gt        marginal costs from the table (UCP_FP64_GT)
//   k_select<P,T>  per point: level minimum, FP32 tie band, FP64 values of
//                  the band members (from the table, T, or FP64 window
//                  sums; queued and evaluated within the block), selection
//                  rule, next bracket, and after the last level the
//                  comparison with the incumbent
//   k_u1_stats/k_u1_partial<P>/k_u1_combine   closed-form second controller
//   k_j_rows/k_j_reduce            objective in FP64, fixed-order reduction
//   k_a1_*         the generic solver's steps (Section III-B to III-D)
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <climits>
#include <cmath>

#include "ucp_internal.h"

namespace ucp {

// ----------------------------------------------------------------- helpers

__device__ __forceinline__ int find_inst(const int32_t* __restrict__ pre, int n, int u) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= u) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int wave_min_i(int v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wave_min_d(double v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
// Reductions over a wave whose 64 lanes are all active, through DPP lane
// moves (no LDS traffic): quad swaps and row mirrors reduce each row of 16,
// two row broadcasts fold the rows into lane 63, whose value is returned to
// every lane (the sum's order is fixed, so its bits are reproducible).
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_mov(int v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_mov_d(double v) {
  const int lo = dpp_mov<CTRL, ROWS>(__double2loint(v));
  const int hi = dpp_mov<CTRL, ROWS>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wred_sum_d(double v) {
  v += dpp_mov_d<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov_d<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_mov_d<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_mov_d<0x140, 0xF>(v);  // row_mirror
  v += dpp_mov_d<0x142, 0xA>(v);  // row_bcast:15 into rows 1, 3
  v += dpp_mov_d<0x143, 0xC>(v);  // row_bcast:31 into rows 2, 3
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                          __builtin_amdgcn_readlane(__double2loint(v), 63));
}

// Sum over a group of W lanes (the whole wave, or an aligned half): DPP for
// a whole wave, a butterfly within the half otherwise.
template <int W>
__device__ __forceinline__ double grp_sum_d(double v) {
  if constexpr (W == kWave) {
    return wred_sum_d(v);
  } else {
    for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
  }
}

__device__ __forceinline__ double clampd(double v, double lo, double hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// Candidate q of `level` at point i: level 0 is the global grid over
// [u_lo, u_hi] (q == cands is the incumbent); level l spans the neighbour
// bracket of the best so far, clamped to the range.  Plain binary64
// arithmetic, no contraction (the library is built with -ffp-contract=off).
__device__ __forceinline__ double cand_pos(const Inst& I, int level, int q, int i) {
  if (level < 0) return I.u0[(size_t)i * I.cands + q];  // explicit candidates
  if (level == 0) {
    if (q == I.cands) return I.u0[i];
    return I.u_lo + (double)q * I.h[0];
  }
  return clampd((I.cbest[i] - I.h[level - 1]) + (double)q * I.h[level], I.u_lo, I.u_hi);
}

// Nearest y node to z (clamped to the grid; NaN maps to node 0).
__device__ __forceinline__ int nearest_node(const Inst& I, double z) {
  double jf = rint((z - I.y_lo) * I.inv_dy);
  jf = fmin(fmax(jf, 0.0), (double)(I.n_y - 1));
  return (int)jf;
}

// Centre of the FP32 window of z: the nearest node of the grid extended
// past its ends (a position beyond the grid keeps its own window, clipped
// to the grid, and one more than nw32 nodes out has none), held within
// [-nw32 - 1, n_y + nw32]; NaN maps to node 0.
__device__ __forceinline__ int window_centre32(const Inst& I, double z) {
  double jf = rint((z - I.y_lo) * I.inv_dy);
  jf = fmin(fmax(jf, -(double)I.nw32 - 1.0), (double)(I.n_y + I.nw32));
  return isnan(jf) ? 0 : (int)jf;
}

// FP64 window sum for one position z, spread over a group of W lanes (a
// wave, or in the selection kernels possibly an aligned half of one):
// returns dy/sqrt(2 pi) * sum_j phi(y_j - z) (z - u1_j)^2 over the nodes
// within kWin64 of the node nearest z.  The Gaussian is max-shifted to that
// node, g_k = exp(-(t_k^2 - delta^2)/2) = exp(-d (d + 2 delta)/2) with
// d = k dy, and the shift exp(-delta^2/2) is applied once at the end.
// Lane l takes k = klo + l + W m; along m the Gaussian obeys the exact
// recurrence g_{k+W} = g_k r_k, r_{k+W} = r_k q with
// r_k = exp(-W dy t_k - (W dy)^2 / 2) and q = exp(-(W dy)^2), so two
// multiplies replace an exp; both are recomputed by exp every I.rs64 steps
// (at most kReseed), which bounds the relative error of any weight by
// ~kReseed^2/2 ulp (5.7e-14).  (All distances here are in noise sds.)  A
// pass over the union of several positions' windows starts far from some of
// them, where a seed beyond 37.6 sds underflows; reseeds at most 24 sds
// apart (I.rs64 W dy <= 24, steps of W nodes) give every position an exact
// seed more than 11 sds out, before its window begins; r's exponent is
// capped so a far seed cannot overflow it.  Every lane has a node in the first floor(n/W)
// steps: they run without masks in groups of kPrefetch, the loads of group
// g + 1 issued before group g is summed (two register buffers); only the
// last step can be partial.  Even steps go to one accumulator and odd steps
// to another.
constexpr int kReseed = 32;
constexpr int kPrefetch = 4;
static_assert(kReseed % kPrefetch == 0, "reseeds fall on group boundaries");
constexpr double kRMaxExp = 700.0;  // cap of r's exponent (exp(700) is finite)
typedef const __attribute__((address_space(1))) double* glb_dptr;

struct B64Walk {
  double g, r;  // weight of the lane's next node and its ratio
};

template <int W>
__device__ __forceinline__ void b64_reseed(B64Walk& w, int klo, int lane, int m, double dy, double delta, double D) {
  const double d = (double)(klo + lane + W * m) * dy;
  w.g = exp(-0.5 * d * (d + 2.0 * delta));
  w.r = exp(fmin(-D * (d + delta) - 0.5 * D * D, kRMaxExp));
}

// Sum one group of kPrefetch steps starting at step m (m a multiple of
// kPrefetch, reseeded by the caller when due); reseeds inside the group when
// the instance reseeds more often than every kPrefetch steps.
template <int W>
__device__ __forceinline__ void b64_group(const double* uv, double z, double q, B64Walk& w, double& s0, double& s1,
                                          int m, int rs, int klo, int lane, double dy, double delta, double D) {
#pragma unroll
  for (int mm = 0; mm < kPrefetch; mm += 2) {
    if (rs < kPrefetch && mm > 0 && ((m + mm) & (rs - 1)) == 0) b64_reseed<W>(w, klo, lane, m + mm, dy, delta, D);
    const double e0 = z - uv[mm];
    s0 = fma(w.g * e0, e0, s0);
    w.g *= w.r;
    w.r *= q;
    if (rs == 1) b64_reseed<W>(w, klo, lane, m + mm + 1, dy, delta, D);
    const double e1 = z - uv[mm + 1];
    s1 = fma(w.g * e1, e1, s1);
    w.g *= w.r;
    w.r *= q;
  }
}

template <int W = kWave>
__device__ double b64_wave(const Inst& I, double z, int lane) {
  const int jr = nearest_node(I, z);
  // offsets in noise sds: delta and the spacing times 1 / noise_sd
  const double delta = ((I.y_lo + (double)jr * I.dy) - z) * I.isw;
  // 0 <= jr <= n_y - 1, so klo <= 0 <= khi and the window is never empty
  const int klo = max(-I.nw64, -jr), khi = min(I.nw64, I.n_y - 1 - jr);
  const int n = khi - klo + 1;
  const double dy = I.dy * I.isw, D = (double)W * dy;
  const double q = exp(-D * D);
  glb_dptr u1 = (glb_dptr)(I.u1 + jr + klo + lane);  // this lane's node of step m: u1[W m]
  double s0 = 0.0, s1 = 0.0;
  const int steps = (n + W - 1) / W;
  const int groups = (n / W) / kPrefetch;  // unmasked groups
  const int rs = I.rs64;                   // steps between reseeds (a power of two)
  B64Walk w;
  double ua[kPrefetch], ub[kPrefetch];
  if (groups > 0) {
#pragma unroll
    for (int mm = 0; mm < kPrefetch; ++mm) ua[mm] = u1[W * mm];
  }
  int gi = 0;
  for (; gi + 2 <= groups; gi += 2) {
    const int m = gi * kPrefetch;
#pragma unroll
    for (int mm = 0; mm < kPrefetch; ++mm) ub[mm] = u1[W * (m + kPrefetch + mm)];
    if ((m & (rs - 1)) == 0) b64_reseed<W>(w, klo, lane, m, dy, delta, D);
    b64_group<W>(ua, z, q, w, s0, s1, m, rs, klo, lane, dy, delta, D);
    // the group after next, or (past the end, unused) the last one: in range
    const int mn = min(m + 2 * kPrefetch, (groups - 1) * kPrefetch);
#pragma unroll
    for (int mm = 0; mm < kPrefetch; ++mm) ua[mm] = u1[W * (mn + mm)];
    if (((m + kPrefetch) & (rs - 1)) == 0) b64_reseed<W>(w, klo, lane, m + kPrefetch, dy, delta, D);
    b64_group<W>(ub, z, q, w, s0, s1, m + kPrefetch, rs, klo, lane, dy, delta, D);
  }
  if (gi < groups) {  // one group left, already loaded
    const int m = gi * kPrefetch;
    if ((m & (rs - 1)) == 0) b64_reseed<W>(w, klo, lane, m, dy, delta, D);
    b64_group<W>(ua, z, q, w, s0, s1, m, rs, klo, lane, dy, delta, D);
  }
  for (int m = groups * kPrefetch; m < steps; ++m) {  // the rest, the last step possibly partial
    if ((m & (rs - 1)) == 0) b64_reseed<W>(w, klo, lane, m, dy, delta, D);
    double e = 0.0;
    if (lane + W * m < n) e = z - u1[W * m];
    if (m & 1) s1 = fma(w.g * e, e, s1);
    else s0 = fma(w.g * e, e, s0);
    w.g *= w.r;
    w.r *= q;
  }
  const double s = grp_sum_d<W>(s0 + s1);
  return I.phi_scale * exp(-0.5 * delta * delta) * s;
}

// FP64 window sums for R positions z_q sharing one pass over the union of
// their windows (the positions of one point's queued candidates lie within
// a small bracket): each lane's u1 load serves all R sums.  Per position the
// same shifted Gaussian and reseeded recurrence as b64_wave, relative to its
// own nearest node; nodes of the union beyond a position's own window add
// weights below exp(-60) (terms of the dense sum all the same).  The union
// may start far from a position (the objective's rows, a winner and a
// distant incumbent): its weights there underflow, and the reseed interval
// (I.rs64) restores them before its peak.  One accumulator per position.
template <int R, int W = kWave>
__device__ void b64_multi(const Inst& I, const double* z, int lane, double* out) {
  int jr[R];
  double delta[R];
  int jlo = INT_MAX, jhi = INT_MIN;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    jr[q] = nearest_node(I, z[q]);
    delta[q] = ((I.y_lo + (double)jr[q] * I.dy) - z[q]) * I.isw;  // in noise sds
    jlo = min(jlo, max(0, jr[q] - I.nw64));
    jhi = max(jhi, min(I.n_y - 1, jr[q] + I.nw64));
  }
  const int n = jhi - jlo + 1;
  const double dy = I.dy * I.isw, D = (double)W * dy;
  const double qf = exp(-D * D);
  glb_dptr u1 = (glb_dptr)(I.u1 + jlo + lane);  // this lane's node of step m: u1[W m]
  double g[R], r[R], s[R];
#pragma unroll
  for (int q = 0; q < R; ++q) s[q] = 0.0;
  auto reseed = [&](int m) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const double d = (double)(jlo + lane + W * m - jr[q]) * dy;
      g[q] = exp(-0.5 * d * (d + 2.0 * delta[q]));
      r[q] = exp(fmin(-D * (d + delta[q]) - 0.5 * D * D, kRMaxExp));
    }
  };
  const int rs = I.rs64;  // steps between reseeds (a power of two)
  auto group = [&](const double* uv, int m) {
#pragma unroll
    for (int mm = 0; mm < kPrefetch; ++mm) {
      if (rs < kPrefetch && mm > 0 && ((m + mm) & (rs - 1)) == 0) reseed(m + mm);
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const double e = z[q] - uv[mm];
        s[q] = fma(g[q] * e, e, s[q]);
        g[q] *= r[q];
        r[q] *= qf;
      }
    }
  };
  const int steps = (n + W - 1) / W;
  const int groups = (n / W) / kPrefetch;  // unmasked groups
  double ua[kPrefetch], ub[kPrefetch];
  if (groups > 0) {
#pragma unroll
    for (int mm = 0; mm < kPrefetch; ++mm) ua[mm] = u1[W * mm];
  }
  int gi = 0;
  for (; gi + 2 <= groups; gi += 2) {
    const int m = gi * kPrefetch;
#pragma unroll
    for (int mm = 0; mm < kPrefetch; ++mm) ub[mm] = u1[W * (m + kPrefetch + mm)];
    if ((m & (rs - 1)) == 0) reseed(m);
    group(ua, m);
    const int mn = min(m + 2 * kPrefetch, (groups - 1) * kPrefetch);
#pragma unroll
    for (int mm = 0; mm < kPrefetch; ++mm) ua[mm] = u1[W * (mn + mm)];
    if (((m + kPrefetch) & (rs - 1)) == 0) reseed(m + kPrefetch);
    group(ub, m + kPrefetch);
  }
  if (gi < groups) {
    const int m = gi * kPrefetch;
    if ((m & (rs - 1)) == 0) reseed(m);
    group(ua, m);
  }
  for (int m = groups * kPrefetch; m < steps; ++m) {
    if ((m & (rs - 1)) == 0) reseed(m);
    const bool in = lane + W * m < n;
    const double u = in ? u1[W * m] : 0.0;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const double e = in ? z[q] - u : 0.0;
      s[q] = fma(g[q] * e, e, s[q]);
      g[q] *= r[q];
      r[q] *= qf;
    }
  }
#pragma unroll
  for (int q = 0; q < R; ++q) out[q] = I.phi_scale * exp(-0.5 * delta[q] * delta[q]) * grp_sum_d<W>(s[q]);
}

// Algorithmic terms of one (point, candidate): the y nodes within kWin32
// noise sds (I.win32 = kWin32 noise_sd) of z (the work the method needs for FP64-level accuracy; the
// kernels may evaluate a few more).  Summed per wave, one atomic per wave.
__device__ __forceinline__ void count_terms(const Inst& I, double z, bool act, int lane) {
  long long n = 0;
  if (act && I.terms) {
    double lo = ceil((z - I.win32 - I.y_lo) * I.inv_dy);
    double hi = floor((z + I.win32 - I.y_lo) * I.inv_dy);
    lo = fmax(lo, 0.0);
    hi = fmin(hi, (double)(I.n_y - 1));
    if (hi >= lo) n = (long long)(hi - lo) + 1;
  }
  for (int o = kWave / 2; o > 0; o >>= 1) n += __shfl_xor(n, o);
  if (lane == 0 && n > 0 && I.terms)
    atomicAdd(I.terms + kCountTerms + (blockIdx.x & (kCountSlots - 1)) * kCountStride, (unsigned long long)n);
}

// ------------------------------------------------------------------ prior

int32_t units_prior(const Inst& I) { return (I.n_x + 255) / 256; }

__global__ __launch_bounds__(256) void k_prior(Launch L) {
  const int u = blockIdx.x;
  const int b = find_inst(L.pre, L.n_inst, u);
  const Inst& I = L.insts[b];
  const int i = (u - L.pre[b]) * 256 + threadIdx.x;
  if (i >= I.n_x) return;
  const double x = I.x_lo + (double)i * I.dx;
  const double r2pi = 2.5066282746310005024157652848110;  // sqrt(2 pi)
  double sum = 0.0, lmax = -INFINITY;
  double lc[kMaxComp];
  for (int c = 0; c < I.n_comp; ++c) {
    double d = (x - I.mu[c]) / I.sd[c];
    sum += I.w[c] * exp(-0.5 * d * d) / (I.sd[c] * r2pi);
    lc[c] = log(I.w[c]) - log(I.sd[c]) - log(r2pi) - 0.5 * d * d;
    lmax = fmax(lmax, lc[c]);
  }
  double acc = 0.0;
  for (int c = 0; c < I.n_comp; ++c) acc += exp(lc[c] - lmax);
  I.f[i] = sum;
  I.logf[i] = lmax + log(acc);
}

// Offset table of the marginal-cost kernel: G_k = exp(-(k dy / s)^2 / 2) =
// exp2(-(k alpha dy)^2) for |k| <= nw32 (s the noise sd, alpha =
// sqrt(log2(e)/2) / s), rounded once from FP64.
__global__ __launch_bounds__(256) void k_gtab(Launch L) {
  const int u = blockIdx.x;
  const int b = find_inst(L.pre, L.n_inst, u);
  const Inst& I = L.insts[b];
  const int k = (u - L.pre[b]) * 256 + (int)threadIdx.x - I.nw32;
  if (k > I.nw32 + kGtabPad) return;  // padded past the window for the last block's reads
  const double d = (double)k * I.dy * I.isw;
  I.gtab[k + I.nw32] = (float)exp(-0.5 * d * d);
}

int32_t units_gtab(const Inst& I) { return (2 * I.nw32 + 1 + kGtabPad + 255) / 256; }

hipError_t launch_prior(const Launch& L, hipStream_t st) {
  if (L.total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_prior, dim3(L.total), dim3(256), 0, st, L);
  return hipGetLastError();
}

hipError_t launch_gtab(const Launch& L, hipStream_t st) {
  if (L.total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gtab, dim3(L.total), dim3(256), 0, st, L);
  return hipGetLastError();
}

// ---------------------------------------------------- marginal cost, FP32
//
// Work unit = (tile of 256 consecutive points, candidate q, window segment).
// Lane = point.  For point i and candidate c: z = x_i + c, jr = nearest y
// node, delta = y_jr - z, and with t_k = y_{jr+k} - z = k dy + delta the unit
// sums, over its segment of the window |k| <= nw32,
//   sum_k exp(-(t_k^2 - delta^2)/2) (z - u1_{jr+k})^2.
// In scaled units (alpha^2 = log2(e)/2) the shifted Gaussian factors as
//   exp(-(t_k^2 - delta^2)/2) = G_k * E_k,
//   G_k = exp2(-(k alpha dy)^2)          (the same for every lane: a table),
//   E_k = exp2(beta k), beta = -2 alpha^2 dy delta (one constant per lane).
// Every lane of a wave is at the same window offset k, so G_k is one scalar
// load; E_k costs one v_exp_f32 per block of kMcUnroll offsets times the
// per-lane constants exp2(beta m), m < kMcUnroll.  The difference
// alpha (z - u1) comes from a staged array in one of two forms (see mc_e).
// After the shift every weight is <= 1, so FP32 neither overflows nor
// underflows where terms matter.  The block stages the nodes it touches in
// LDS (falls back to global loads of the residual form when its node range
// exceeds kMcLds, e.g. across a jump of the controller).

int32_t units_mc(const Inst& I, int level) {
  if (level >= 0 && level >= I.levels) return 0;
  const int tiles = (I.n_x + kMcBlock - 1) / kMcBlock;
  const int kq = level == 0 ? I.cands + 1 : I.cands;  // level < 0: explicit candidates
  return tiles * kq * I.segs;
}

typedef const __attribute__((address_space(3))) float* lds_cptr;
typedef const __attribute__((address_space(1))) float* glb_cptr;
typedef const __attribute__((address_space(4))) float* cst_cptr;  // read through the scalar cache

__device__ __forceinline__ void kahan_add(float x, float& acc, float& comp) {
  const float y = x - comp;
  const float t = acc + y;
  comp = (t - acc) - y;
  acc = t;
}

constexpr int kMcUnroll = 16;
static_assert(kGtabPad >= kMcUnroll, "the offset table covers the last block's reads");

// Per-lane constants of one unit.
struct McLane {
  float aDy;             // alpha dy
  float Dl;              // residual form: alpha delta; reference form: a = alpha (z - z_c)
  float beta;            // -2 alpha^2 dy delta
  float F16;             // exp2(beta kMcUnroll): the factor from one block's E_k to the next's
  float R[kMcUnroll];    // residual form: exp2(beta m); reference form: exp2(beta m / 2)
  float Dm[kMcUnroll];   // residual form: Dl + m alpha dy; reference form: exp2(beta m / 2) a
};

// The scaled difference e = alpha (z - u1_j) of node j = jr + k, from the
// staged value s_j, in one of two forms:
//  - residual form (REF = false): s_j = alpha (y_j - u1_j), e = s_j - T_k
//    with T_k = alpha (y_j - z) = alpha (delta + k dy);
//  - reference form (REF = true): s_j = alpha (z_c - u1_j) around one z_c per
//    block, e = s_j + a with a = alpha (z - z_c).  Used when every z of the
//    block lies within kMcRefHalf of z_c, where its rounding error (<= ulp
//    of |a| <= 2.1 and of |e|) is no larger than the residual form's (<= ulp
//    of alpha |y_j - z|, a few units over the weighted nodes).  In the unrolled
//    blocks the term's factor R_m = exp2(beta m) is folded into the
//    difference: R_m e^2 = e'^2 with e' = fma(sqrt R_m, s_j, sqrt R_m a), so
//    a term costs one fma, one multiply and one fma.
template <bool REF>
__device__ __forceinline__ float mc_e(float sj, float kf, float Dm, const McLane& c) {
  return REF ? sj + c.Dl : sj - fmaf(kf, c.aDy, Dm);
}

// Offsets k in [k0, k1] (wave-uniform bounds, every lane in range): blocks of
// kMcUnroll terms summed plainly in two chains, each block sum added with
// compensation (KAHAN) or plainly.  Two register buffers alternate: the
// staged values (LDS) and table values (scalar loads) of block b + 1 are
// requested once block b's have been consumed into its first partial
// products, so their latency overlaps the rest of block b.  (LDS and scalar
// loads share one wait counter: loads issued any earlier would be waited
// for together with block b's.)
struct McBlk {
  float g[kMcUnroll];  // table values G_{k+m}
  float v[kMcUnroll];  // staged values s_{jr+k+m}
};

template <typename P, typename Q>
__device__ __forceinline__ void mc_load(McBlk& B, P v, Q G, int k) {
#pragma unroll
  for (int m = 0; m < kMcUnroll; ++m) {
    B.g[m] = G[k + m];
    B.v[m] = v[k + m];
  }
}

// First half of a block: the differences (consumes the staged values; the
// table values stay in scalar registers until the second half).  Reference
// form: e'_m = sqrt(R_m) e_m.
template <bool REF>
__device__ __forceinline__ void mc_first(const McBlk& B, float kf, const McLane& c, float* e) {
#pragma unroll
  for (int m = 0; m < kMcUnroll; ++m)
    e[m] = REF ? fmaf(c.R[m], B.v[m], c.Dm[m]) : mc_e<false>(B.v[m], kf, c.Dm[m], c);
}

// Second half: the weights g_m R_m and the block sum times E_k = exp2(beta k)
// (E_{k+m} = E_k R_m).  mc_block_sum returns the block's sum times a given
// E_k, not yet added; mc_second computes E_k and adds the sum.
template <bool REF>
__device__ __forceinline__ float mc_block_sum(const McBlk& B, const float* e, float E0, const McLane& c) {
  float b0 = 0.0f, b1 = 0.0f;
#pragma unroll
  for (int m = 0; m < kMcUnroll; m += 2) {
    if (REF) {
      b0 = fmaf(B.g[m] * e[m], e[m], b0);
      b1 = fmaf(B.g[m + 1] * e[m + 1], e[m + 1], b1);
    } else {
      b0 = fmaf((B.g[m] * c.R[m]) * e[m], e[m], b0);
      b1 = fmaf((B.g[m + 1] * c.R[m + 1]) * e[m + 1], e[m + 1], b1);
    }
  }
  return E0 * (b0 + b1);
}

template <bool KAHAN, bool REF>
__device__ __forceinline__ void mc_second(const McBlk& B, const float* e, float kf, const McLane& c, float& acc,
                                          float& comp) {
  // |beta| <= kMcBetaMax for every lane that reaches the blocked loops, so
  // in a block holding a term of the lane's window beta k <= 79 at most; a
  // masked block before the window can have beta k beyond FP32 range, and
  // the cap keeps its zero sum from meeting an infinite factor
  const float E0 = __builtin_amdgcn_exp2f(fminf(c.beta * kf, 126.0f));
  float b0 = 0.0f, b1 = 0.0f;
#pragma unroll
  for (int m = 0; m < kMcUnroll; m += 2) {
    if (REF) {  // R_m is inside e'
      b0 = fmaf(B.g[m] * e[m], e[m], b0);
      b1 = fmaf(B.g[m + 1] * e[m + 1], e[m + 1], b1);
    } else {
      b0 = fmaf((B.g[m] * c.R[m]) * e[m], e[m], b0);
      b1 = fmaf((B.g[m + 1] * c.R[m + 1]) * e[m + 1], e[m + 1], b1);
    }
  }
  if (KAHAN) kahan_add(E0 * (b0 + b1), acc, comp);
  else acc = fmaf(E0, b0 + b1, acc);
}

// One term outside the unrolled blocks.
template <bool KAHAN, bool REF, typename P, typename Q>
__device__ __forceinline__ void mc_one(P v, Q G, int k, const McLane& c, float& acc, float& comp) {
  const float kf = (float)k;
  const float g = G[k] * __builtin_amdgcn_exp2f(c.beta * kf);
  const float e = mc_e<REF>(v[k], kf, c.Dl, c);
  if (KAHAN) kahan_add((g * e) * e, acc, comp);
  else acc = fmaf(g * e, e, acc);
}

// PAD: v and G hold kMcUnroll readable entries past k1 (the padded LDS
// stage and offset table), so the last pair's look-ahead load needs no
// clamp; the values it reads past k1 are never used.
template <bool KAHAN, bool REF, bool PAD, typename P, typename Q>
__device__ __forceinline__ void mc_bulk(P v, Q G, int k0, int k1, const McLane& c, float& acc,
                                        float& comp) {
  constexpr int U = kMcUnroll;
  int k = k0;
  McBlk A, B;
  float e[U];
  if (k + U - 1 <= k1) mc_load(A, v, G, k);
  for (; k + 2 * U - 1 <= k1; k += 2 * U) {
    mc_first<REF>(A, (float)k, c, e);
    __builtin_amdgcn_sched_barrier(0);
    mc_load(B, v, G, k + U);
    __builtin_amdgcn_sched_barrier(0);
    // E_k of the pair's first block; the second's is E_k exp2(16 beta)
    // (every offset here lies in every lane's window, where beta k <= 79,
    // so neither factor overflows and no cap is needed)
    const float Ea = __builtin_amdgcn_exp2f(c.beta * (float)k);
    const float sa = mc_block_sum<REF>(A, e, Ea, c);
    mc_first<REF>(B, (float)(k + U), c, e);
    __builtin_amdgcn_sched_barrier(0);
    // the next block; past the end (unused) the padding, or else the last
    // full block, so every read stays in range
    mc_load(A, v, G, PAD ? k + 2 * U : min(k + 2 * U, k1 - U + 1));
    __builtin_amdgcn_sched_barrier(0);
    const float sb = mc_block_sum<REF>(B, e, Ea * c.F16, c);
    if (KAHAN) kahan_add(sa + sb, acc, comp);  // one compensated add per pair of blocks
    else acc += sa + sb;
  }
  if (k + U - 1 <= k1) {  // one block left, already loaded into A
    mc_first<REF>(A, (float)k, c, e);
    mc_second<KAHAN, REF>(A, e, (float)k, c, acc, comp);
    k += U;
  }
  for (; k <= k1; ++k) mc_one<KAHAN, REF>(v, G, k, c, acc, comp);
}

// Offsets k in [k0, k1] restricted to the lane's own range [klo, khi].
template <bool KAHAN, bool REF, typename P, typename Q>
__device__ __forceinline__ void mc_masked(P v, Q G, int k0, int k1, int klo, int khi, const McLane& c,
                                          float& acc, float& comp) {
  for (int k = k0; k <= k1; ++k)
    if (k >= klo && k <= khi) mc_one<KAHAN, REF>(v, G, k, c, acc, comp);
}

// The lane's window [klo, khi] (empty when klo > khi): the range common to
// every non-empty lane of the wave runs unmasked, the ragged ends masked.
template <bool KAHAN, bool REF, typename P, typename Q>
__device__ __forceinline__ void mc_lane(P v, Q G, int klo, int khi, const McLane& c, float& acc,
                                        float& comp) {
  const bool empty = klo > khi;
  const int kc_lo = __builtin_amdgcn_readfirstlane(wave_max_i(empty ? INT_MIN : klo));
  const int kc_hi = __builtin_amdgcn_readfirstlane(wave_min_i(empty ? INT_MAX : khi));
  const int ku_lo = __builtin_amdgcn_readfirstlane(wave_min_i(empty ? INT_MAX : klo));
  const int ku_hi = __builtin_amdgcn_readfirstlane(wave_max_i(empty ? INT_MIN : khi));
  if (ku_lo > ku_hi || empty) return;
  if (kc_lo > kc_hi) {
    mc_masked<KAHAN, REF>(v, G, ku_lo, ku_hi, klo, khi, c, acc, comp);
    return;
  }
  mc_masked<KAHAN, REF>(v, G, ku_lo, kc_lo - 1, klo, khi, c, acc, comp);
  mc_bulk<KAHAN, REF, false>(v, G, kc_lo, kc_hi, c, acc, comp);
  mc_masked<KAHAN, REF>(v, G, kc_hi + 1, ku_hi, klo, khi, c, acc, comp);
}

// One block of kMcUnroll offsets from k, each term kept only where the
// offset lies in the lane's [lo, hi] (the others are zeroed through their
// difference).  Reads k .. k + kMcUnroll - 1, which may run past the
// window: the staged array and the offset table are padded for that.
template <bool KAHAN, bool REF, typename P, typename Q>
__device__ __forceinline__ void mc_block_masked(P v, Q G, int k, int lo, int hi, const McLane& c, float& acc,
                                                float& comp) {
  McBlk B;
  mc_load(B, v, G, k);
  float e[kMcUnroll];
  mc_first<REF>(B, (float)k, c, e);
#pragma unroll
  for (int m = 0; m < kMcUnroll; ++m)
    if (!(k + m >= lo && k + m <= hi)) e[m] = 0.0f;
  mc_second<KAHAN, REF>(B, e, (float)k, c, acc, comp);
}

// Offsets [a, b] in masked blocks; the lane keeps [max(a, klo), min(b, khi)].
template <bool KAHAN, bool REF, typename P, typename Q>
__device__ __forceinline__ void mc_region_masked(P v, Q G, int a, int b, int klo, int khi, const McLane& c,
                                                 float& acc, float& comp) {
  const int lo = max(a, klo), hi = min(b, khi);
  for (int k = a; k <= b; k += kMcUnroll) mc_block_masked<KAHAN, REF>(v, G, k, lo, hi, c, acc, comp);
}

// The lane's window [klo, khi] from a staged, padded array: the offsets
// common to every non-empty lane of the wave ([kc_lo, kc_hi]) run in the
// unrolled loop, its last partial block and the ragged ends of the wave's
// union [ku_lo, ku_hi] in masked blocks (the ragged ends are long where a
// wave straddles a jump of the controller next to the grid's edge).
template <bool KAHAN, bool REF, typename P, typename Q>
__device__ __forceinline__ void mc_lane_padded(P v, Q G, int klo, int khi, int kc_lo, int kc_hi, int ku_lo,
                                               int ku_hi, const McLane& c, float& acc, float& comp) {
  // a lane with an empty window takes no part (its node range is not staged)
  if (ku_lo > ku_hi || klo > khi) return;
  if (kc_lo > kc_hi) {
    mc_region_masked<KAHAN, REF>(v, G, ku_lo, ku_hi, klo, khi, c, acc, comp);
    return;
  }
  mc_region_masked<KAHAN, REF>(v, G, ku_lo, kc_lo - 1, klo, khi, c, acc, comp);
  const int nfull = (kc_hi - kc_lo + 1) / kMcUnroll * kMcUnroll;
  if (nfull) mc_bulk<KAHAN, REF, true>(v, G, kc_lo, kc_lo + nfull - 1, c, acc, comp);
  mc_region_masked<KAHAN, REF>(v, G, kc_lo + nfull, kc_hi, klo, khi, c, acc, comp);
  mc_region_masked<KAHAN, REF>(v, G, kc_hi + 1, ku_hi, klo, khi, c, acc, comp);
}

template <int PREC>
__global__ __launch_bounds__(kMcBlock) void k_mc32(Launch L, int level) {
  constexpr bool KAHAN = PREC == UCP_FP32_KAHAN;
  constexpr int NW = kMcBlock / kWave;
  __shared__ float sv[kMcLds];
  __shared__ int sred[2][NW];
  __shared__ double szr[2][NW];
  const int u = blockIdx.x;
  const int b = find_inst(L.pre, L.n_inst, u);
  const Inst& I = L.insts[b];
  int local = u - L.pre[b];
  const int S = I.segs;
  const int kq = level < 0 ? I.cands : (level == 0 ? I.cands + 1 : I.cands);
  // window segment slowest: blocks dispatched together read the same part
  // of the offset table, which then stays in the scalar cache
  const int per_seg = ((I.n_x + kMcBlock - 1) / kMcBlock) * kq;
  // middle segments first and the window's two end segments last: the end
  // segments lose the most to the grid's edges, so the last units of the
  // launch are the shorter ones and the launch drains sooner
  const int sidx = local / per_seg;
  const int WS = I.wsegs;
  const int so = min(sidx, WS - 1);
  const int seg = (WS - 1) / 2 + ((so & 1) ? (so + 1) / 2 : -(so / 2));
  // units past the window segments are the two halves of the last one
  const int half = S > WS && sidx >= WS - 1 ? sidx - (WS - 1) : -1;
  local %= per_seg;
  const int q = local % kq;
  const int tile = local / kq;
  const int i = tile * kMcBlock + (int)threadIdx.x;
  const bool act = i < I.n_x;
  const int ii = act ? i : I.n_x - 1;

  const double c = cand_pos(I, level, q, ii);
  const double x = I.x_lo + (double)ii * I.dx;
  const double z = x + c;
  // the window's centre: past the grid's ends the nearest node of the
  // extended grid, so the window holds only nodes within nw32 of z
  const int jr = window_centre32(I, z);
  const double delta = (I.y_lo + (double)jr * I.dy) - z;
  const int nw = I.nw32;
  const int seglen = (2 * nw + 1 + WS - 1) / WS;
  int s_lo = -nw + seg * seglen;
  int s_hi = min(nw, s_lo + seglen - 1);
  if (half >= 0) {
    const int mid = s_lo + (s_hi - s_lo + 1) / 2;
    if (half == 0) s_hi = mid - 1;
    else s_lo = mid;
  }
  int klo = max(s_lo, -jr), khi = min(s_hi, I.n_y - 1 - jr);
  if (!act) { klo = 1; khi = 0; }
  const double beta = -2.0 * I.a2 * I.dy * delta;
  // Lanes whose weights change by more than 2^kMcBetaMax from node to node
  // (very coarse y grids, or positions far outside the y grid) sum their
  // window term by term below with exact weights; the blocked loops see
  // them as empty, so the per-lane factors exp2(beta m) stay within range.
  const bool bigb = fabs(beta) > kMcBetaMax && klo <= khi;
  const int wlo = bigb ? 1 : klo, whi = bigb ? 0 : khi;

  // the wave's common and union offset ranges, and the node range it reads
  // (staged in LDS with kMcUnroll nodes of padding past the union, for the
  // unrolled loop's look-ahead; zero beyond the grid), plus the z range of
  // the block
  const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const bool ne = wlo <= whi;
  const int kc_lo = __builtin_amdgcn_readfirstlane(wave_max_i(ne ? wlo : INT_MIN));
  const int kc_hi = __builtin_amdgcn_readfirstlane(wave_min_i(ne ? whi : INT_MAX));
  const int ku_lo = __builtin_amdgcn_readfirstlane(wave_min_i(ne ? wlo : INT_MAX));
  const int ku_hi = __builtin_amdgcn_readfirstlane(wave_max_i(ne ? whi : INT_MIN));
  const int jmin = wave_min_i(ne ? jr : INT_MAX);
  const int jmax = wave_max_i(ne ? jr : INT_MIN);
  const bool wne = ku_lo <= ku_hi;  // some lane of the wave has offsets
  const double zlo = wave_min_d(ne ? z : INFINITY);
  const double zhi = -wave_min_d(ne ? -z : INFINITY);
  if (lane == 0) {
    sred[0][wid] = wne ? jmin + ku_lo : INT_MAX;
    sred[1][wid] = wne ? jmax + ku_hi + kMcUnroll : INT_MIN;
    szr[0][wid] = zlo;
    szr[1][wid] = zhi;
  }
  __syncthreads();
  int blo = INT_MAX, bhi = INT_MIN;
  double bzlo = INFINITY, bzhi = -INFINITY;
  for (int w = 0; w < NW; ++w) {
    blo = min(blo, sred[0][w]);
    bhi = max(bhi, sred[1][w]);
    bzlo = fmin(bzlo, szr[0][w]);
    bzhi = fmax(bzhi, szr[1][w]);
  }
  if (sidx == 0) {
    count_terms(I, z, act, lane);
    // terms this unit's (point, candidate) evaluates over all its segments
    long long ev = act ? (long long)max(0, min(nw, I.n_y - 1 - jr) - max(-nw, -jr) + 1) : 0;
    for (int o = kWave / 2; o > 0; o >>= 1) ev += __shfl_xor(ev, o);
    if (lane == 0 && ev > 0 && I.terms)
      atomicAdd(I.terms + kCountEvalTerms + (blockIdx.x & (kCountSlots - 1)) * kCountStride, (unsigned long long)ev);
  }
  const double alpha = I.alpha;
  const bool staged = bhi >= blo && bhi - blo + 1 <= kMcLds;
  const bool ref = staged && bzhi - bzlo <= 2.0 * kMcRefHalf * I.sw;
  const double zc = 0.5 * (bzlo + bzhi);  // block-uniform
  {
    // fields in registers and global-space pointers: the instance is read
    // through a generic pointer, which the LDS stores below could alias, so
    // it would be reloaded (three dependent loads) on every iteration
    const int ny = I.n_y;
    const glb_dptr u1g = (glb_dptr)I.u1;
    const glb_cptr vg = (glb_cptr)I.v;
    // four nodes per thread per step, their loads issued together (indices
    // clamped into the grid, so every load is in bounds; nodes beyond the
    // grid are stored as zero)
    constexpr int SU = 4;
    if (ref) {
      for (int j0 = blo + (int)threadIdx.x; j0 <= bhi; j0 += SU * kMcBlock) {
        double uv[SU];
#pragma unroll
        for (int t = 0; t < SU; ++t) uv[t] = u1g[min(max(j0 + t * kMcBlock, 0), ny - 1)];
#pragma unroll
        for (int t = 0; t < SU; ++t) {
          const int j = j0 + t * kMcBlock;
          if (j <= bhi) sv[j - blo] = j >= 0 && j < ny ? (float)(alpha * (zc - uv[t])) : 0.0f;
        }
      }
    } else if (staged) {
      for (int j0 = blo + (int)threadIdx.x; j0 <= bhi; j0 += SU * kMcBlock) {
        float vv[SU];
#pragma unroll
        for (int t = 0; t < SU; ++t) vv[t] = vg[min(max(j0 + t * kMcBlock, 0), ny - 1)];
#pragma unroll
        for (int t = 0; t < SU; ++t) {
          const int j = j0 + t * kMcBlock;
          if (j <= bhi) sv[j - blo] = j >= 0 && j < ny ? vv[t] : 0.0f;
        }
      }
    }
  }
  __syncthreads();

  McLane cl;
  cl.aDy = (float)(alpha * I.dy);
  cl.Dl = ref ? (float)(alpha * (z - zc)) : (float)(alpha * delta);
  cl.beta = (float)beta;
  cl.F16 = __builtin_amdgcn_exp2f((float)(beta * kMcUnroll));
#pragma unroll
  for (int m = 0; m < kMcUnroll; ++m) {
    if (ref) {
      cl.R[m] = __builtin_amdgcn_exp2f((float)(0.5 * beta * m));
      cl.Dm[m] = cl.R[m] * cl.Dl;
    } else {
      cl.R[m] = __builtin_amdgcn_exp2f((float)(beta * m));
      cl.Dm[m] = (float)(alpha * (delta + m * I.dy));
    }
  }

  float acc = 0.0f, comp = 0.0f;
  // the offset table is read at wave-uniform offsets: scalar loads
  cst_cptr G = (cst_cptr)(I.gtab + nw);
  if (ref) {
    lds_cptr v = (lds_cptr)(sv + (jr - blo));
    mc_lane_padded<KAHAN, true>(v, G, wlo, whi, kc_lo, kc_hi, ku_lo, ku_hi, cl, acc, comp);
  } else if (staged) {
    lds_cptr v = (lds_cptr)(sv + (jr - blo));
    mc_lane_padded<KAHAN, false>(v, G, wlo, whi, kc_lo, kc_hi, ku_lo, ku_hi, cl, acc, comp);
  } else {
    glb_cptr v = (glb_cptr)(I.v + jr);
    mc_lane<KAHAN, false>(v, G, wlo, whi, cl, acc, comp);
  }
  if (bigb) {  // term by term, residual form from global memory, exact weights
    glb_cptr vg = (glb_cptr)(I.v + jr);
    glb_cptr Gg = (glb_cptr)(I.gtab + nw);
    const float Dr = (float)(alpha * delta);
    for (int k = klo; k <= khi; ++k) {
      const float kf = (float)k;
      const float g = Gg[k] * __builtin_amdgcn_exp2f(cl.beta * kf);
      const float e = vg[k] - fmaf(kf, cl.aDy, Dr);
      if (KAHAN) kahan_add((g * e) * e, acc, comp);
      else acc = fmaf(g * e, e, acc);
    }
  }
  // tiles of 8 points [slot][segment][point] (part_idx): the wave's 64
  // consecutive points write 8 whole lines
  if (act) I.part[part_idx(I, i, q, sidx)] = KAHAN ? (double)acc - (double)comp : (double)acc;
}

// FP64 marginal cost (precision-study mode): lane = point, window kWin64,
// the same shifted Gaussian as b64_wave, walked node by node with the exact
// recurrence g_{k+1} = g_k r_k, r_{k+1} = r_k exp(-dy^2),
// r_k = exp(-dy t_k - dy^2/2), reseeded by exp every kReseed nodes.
// One lane's FP64 window sum for position z, node by node: returns
// sum_k exp(-(t_k^2 - delta^2)/2) (z - u1_{jr+k})^2 over |k| <= nw64, the
// scale dy/(s sqrt(2 pi)) exp(-delta^2/2) left to the caller (jr the
// nearest node, delta = (y_jr - z)/s).
__device__ double lane_sum64(const Inst& I, double z, int jr, double delta) {
  const int klo = max(-I.nw64, -jr), khi = min(I.nw64, I.n_y - 1 - jr);
  const double dy = I.dy * I.isw, qd = exp(-dy * dy);
  const double* __restrict__ u1 = I.u1 + jr;
  double s0 = 0.0, s1 = 0.0;
  for (int k0 = klo; k0 <= khi; k0 += kReseed) {
    const double d = (double)k0 * dy;
    double g = exp(-0.5 * d * (d + 2.0 * delta));
    double r = exp(fmin(-dy * (d + delta) - 0.5 * dy * dy, kRMaxExp));
    const int k1 = min(khi, k0 + kReseed - 1);
    int k = k0;
    for (; k + 1 <= k1; k += 2) {
      const double e0 = z - u1[k];
      s0 = fma(g * e0, e0, s0);
      g *= r;
      r *= qd;
      const double e1 = z - u1[k + 1];
      s1 = fma(g * e1, e1, s1);
      g *= r;
      r *= qd;
    }
    if (k <= k1) {
      const double e0 = z - u1[k];
      s0 = fma(g * e0, e0, s0);
    }
  }
  return s0 + s1;
}

__global__ __launch_bounds__(kMcBlock) void k_mc64(Launch L, int level) {
  const int u = blockIdx.x;
  const int b = find_inst(L.pre, L.n_inst, u);
  const Inst& I = L.insts[b];
  int local = u - L.pre[b];
  const int kq = level < 0 ? I.cands : (level == 0 ? I.cands + 1 : I.cands);
  const int q = local % kq;
  const int tile = local / kq;
  const int i = tile * kMcBlock + (int)threadIdx.x;
  const bool act = i < I.n_x;
  const double c = cand_pos(I, level, q, act ? i : I.n_x - 1);
  const double z = (I.x_lo + (double)(act ? i : I.n_x - 1) * I.dx) + c;
  count_terms(I, z, act, (int)threadIdx.x % kWave);
  if (!act) return;
  const int jr = nearest_node(I, z);
  const double delta = ((I.y_lo + (double)jr * I.dy) - z) * I.isw;  // in noise sds
  I.part[part_idx(I, i, q, 0)] = lane_sum64(I, z, jr, delta);
}

// ------------------------------------------- Gauss-transform arithmetic
//
// For z within d = (z - c) / s of a centre c (delta = z - c, t_j =
// (y_j - c) / s):
//   sum_j exp(-(y_j - z)^2 / (2 s^2)) (z - u1_j)^2
//     = e^{-d^2/2} sum_n d^n / n! [A2_n + 2 delta A1_n + delta^2 A0_n],
//   A_a,n = sum_j e^{-t_j^2/2} t_j^n (c - u1_j)^a,
// since exp(t d) = sum_n (t d)^n / n! and z - u1_j = (c - u1_j) + delta.
// The table holds A_a,n (n <= kGtN) for the centres c = y_lo + k dy, k =
// r gts - gto (row r), over the grid nodes within nw64 of k; the centres run
// from nw64 nodes before the grid to nw64 past it (the sums still run over
// grid nodes only), so every z whose window holds a grid node lies within
// half a row spacing of a centre, and any other z has a noise sum of 0.
// k_gt_table fills it after each u1 update: one wave per row over its
// window, the Gaussian by the reseeded recurrence of the FP64 sums (delta
// = 0 at a centre).  gt_noise_sum then costs O(kGtN) per position.

int32_t units_gt(const Inst& I) { return I.gts ? (I.gtr + 3) / 4 : 0; }

__global__ __launch_bounds__(256) void k_gt_table(Launch L) {
  const int u = blockIdx.x;
  const int b = find_inst(L.pre, L.n_inst, u);
  const Inst& I = L.insts[b];
  const int lane = (int)threadIdx.x % kWave;
  const int r = (u - L.pre[b]) * 4 + (int)threadIdx.x / kWave;
  if (r >= I.gtr) return;  // whole waves
  const int k = r * I.gts - I.gto;  // the row's centre node (may lie off the grid)
  const int klo = max(-I.nw64, -k), khi = min(I.nw64, I.n_y - 1 - k);
  const int n = max(0, khi - klo + 1);  // 0 for a centre whose window misses the grid
  const double dy = I.dy * I.isw, D = (double)kWave * dy;
  const double q = exp(-D * D);
  const double yk = I.y_lo + (double)k * I.dy;
  const int rs = I.rs64;
  glb_dptr u1 = (glb_dptr)(I.u1 + max(0, k + klo) + lane);  // k + klo >= 0 whenever n > 0
  double A0[kGtN + 1], A1[kGtN + 1], A2[kGtN + 1];
#pragma unroll
  for (int m = 0; m <= kGtN; ++m) A0[m] = A1[m] = A2[m] = 0.0;
  B64Walk w;
  const int steps = (n + kWave - 1) / kWave;
  // u1 loads of the next kGtGroup steps are issued before the current
  // group is consumed: a small table has about one wave per SIMD, which
  // would otherwise wait out each step's load
  constexpr int kGtGroup = 8;
  double nx[kGtGroup];
#pragma unroll
  for (int e = 0; e < kGtGroup; ++e) nx[e] = lane + kWave * e < n ? (double)u1[kWave * e] : 0.0;
  for (int m0 = 0; m0 < steps; m0 += kGtGroup) {
    double uv[kGtGroup];
#pragma unroll
    for (int e = 0; e < kGtGroup; ++e) {
      uv[e] = nx[e];
      const int mn = m0 + kGtGroup + e;
      nx[e] = lane + kWave * mn < n ? (double)u1[kWave * mn] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < kGtGroup; ++e) {
      const int m = m0 + e;
      if (m < steps) {
        if ((m & (rs - 1)) == 0) b64_reseed<kWave>(w, klo, lane, m, dy, 0.0, D);
        if (lane + kWave * m < n) {
          const double t = (double)(klo + lane + kWave * m) * dy;
          const double v = yk - uv[e];
          const double v2 = v * v;
          double p = w.g;
#pragma unroll
          for (int o = 0; o <= kGtN; ++o) {
            A0[o] += p;
            A1[o] = fma(p, v, A1[o]);
            A2[o] = fma(p, v2, A2[o]);
            p *= t;
          }
        }
        w.g *= w.r;
        w.r *= q;
      }
    }
  }
  double* row = I.gt + (size_t)r * 3 * (kGtN + 1);
#pragma unroll
  for (int o = 0; o <= kGtN; ++o) {
    const double s0 = grp_sum_d<kWave>(A0[o]), s1 = grp_sum_d<kWave>(A1[o]), s2 = grp_sum_d<kWave>(A2[o]);
    if (lane == 0) {
      row[o] = s0;
      row[(kGtN + 1) + o] = s1;
      row[2 * (kGtN + 1) + o] = s2;
    }
  }
}

hipError_t launch_gt_table(const Launch& L, hipStream_t st) {
  if (L.total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gt_table, dim3(L.total), dim3(256), 0, st, L);
  return hipGetLastError();
}

// 1 / n for the series' Horner steps.
__constant__ double kGtInv[kGtN + 2] = {0.0,       1.0,       1.0 / 2,  1.0 / 3,  1.0 / 4,  1.0 / 5,  1.0 / 6,
                                        1.0 / 7,   1.0 / 8,   1.0 / 9,  1.0 / 10, 1.0 / 11, 1.0 / 12, 1.0 / 13};
static_assert(kGtN == 12, "kGtInv holds 1/n for n <= kGtN + 1");

// The noise part of B at z, dy/(s sqrt(2 pi)) sum_j exp(-(y_j - z)^2 /
// (2 s^2)) (z - u1_j)^2 over the grid nodes within the window, per lane,
// from the moment table: the row whose centre is nearest z (within half a
// row spacing), or 0 where no row is that near (no grid node within the
// window).  LEAN keeps the series loop rolled (three row loads per order
// instead of all 3 (kGtN + 1) at once), for callers whose registers are
// scarce.
template <bool LEAN = false>
__device__ __forceinline__ double gt_noise_sum(const Inst& I, double z) {
  const double span = (double)I.gts * I.dy;
  const double rr = rint((z - I.y_lo) / span) + (double)(I.gto / I.gts);
  if (!(rr >= 0.0 && rr <= (double)(I.gtr - 1))) return 0.0;
  const int r = (int)rr;
  const double del = z - (I.y_lo + (double)(r * I.gts - I.gto) * I.dy);
  const double* row = I.gt + (size_t)r * 3 * (kGtN + 1);
  const double d = del * I.isw;
  double acc = 0.0;
  if (LEAN) {
#pragma unroll 1
    for (int o = kGtN; o >= 0; --o) {
      const double C = fma(del, fma(del, row[o], 2.0 * row[(kGtN + 1) + o]), row[2 * (kGtN + 1) + o]);
      acc = fma(acc, d * kGtInv[o + 1], C);
    }
  } else {
#pragma unroll
    for (int o = kGtN; o >= 0; --o) {
      const double C = fma(del, fma(del, row[o], 2.0 * row[(kGtN + 1) + o]), row[2 * (kGtN + 1) + o]);
      acc = fma(acc, d * kGtInv[o + 1], C);
    }
  }
  return I.phi_scale * exp(-0.5 * d * d) * acc;
}

// Marginal cost from the table (UCP_FP64_GT): lane = point, as k_mc64.
// Stores B itself.
__global__ __launch_bounds__(kMcBlock) void k_mc_gt(Launch L, int level) {
  const int u = blockIdx.x;
  const int b = find_inst(L.pre, L.n_inst, u);
  const Inst& I = L.insts[b];
  int local = u - L.pre[b];
  const int kq = level < 0 ? I.cands : (level == 0 ? I.cands + 1 : I.cands);
  const int q = local % kq;
  const int tile = local / kq;
  const int i = tile * kMcBlock + (int)threadIdx.x;
  const bool act = i < I.n_x;
  const double c = cand_pos(I, level, q, act ? i : I.n_x - 1);
  const double z = (I.x_lo + (double)(act ? i : I.n_x - 1) * I.dx) + c;
  count_terms(I, z, act, (int)threadIdx.x % kWave);
  if (!act) return;
  I.part[part_idx(I, i, q, 0)] = I.k2 * c * c + gt_noise_sum(I, z);
}

hipError_t launch_mc(const Launch& L, int level, int prec, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (L.total == 0) return hipSuccess;
  if (prec == UCP_FP64)
    hipExtLaunchKernelGGL(k_mc64, dim3(L.total), dim3(kMcBlock), 0, st, e0, e1, 0, L, level);
  else if (prec == UCP_FP64_GT)
    hipExtLaunchKernelGGL(k_mc_gt, dim3(L.total), dim3(kMcBlock), 0, st, e0, e1, 0, L, level);
  else if (prec == UCP_FP32_KAHAN)
    hipExtLaunchKernelGGL(k_mc32<UCP_FP32_KAHAN>, dim3(L.total), dim3(kMcBlock), 0, st, e0, e1, 0, L, level);
  else
    hipExtLaunchKernelGGL(k_mc32<UCP_FP32>, dim3(L.total), dim3(kMcBlock), 0, st, e0, e1, 0, L, level);
  return hipGetLastError();
}

// B from the partial sums of candidate lane q: k^2 c^2 + dy/(s sqrt(2 pi))
// exp(-(delta/s)^2/2) * sum (the FP32 sums carry the factor alpha^2).
__device__ __forceinline__ double b_from_parts(const Inst& I, int i, int q, int S,
                                               double c, int prec) {
  const double z = (I.x_lo + (double)i * I.dx) + c;
  // the node the kernel's sums are taken around (FP32: the window centre of
  // k_mc32, which may lie past the grid's ends; FP64: the nearest grid node)
  const int jr = prec == UCP_FP64 ? nearest_node(I, z) : window_centre32(I, z);
  const double delta = ((I.y_lo + (double)jr * I.dy) - z) * I.isw;  // in noise sds
  const double* p = I.part + part_idx(I, i, q, 0);  // segment g at p[g * kPartTile]
  if (prec == UCP_FP64_GT) return p[0];  // B itself
  double s = 0.0;
  for (int g = 0; g < S; ++g) s += p[(size_t)g * kPartTile];
  if (prec != UCP_FP64) s = s / I.a2;
  return I.k2 * c * c + I.phi_scale * exp(-0.5 * delta * delta) * s;
}

// L_0 = f B for explicit candidates (ucp_marginal_cost).
__global__ __launch_bounds__(256) void k_mc_finish(Launch L, double* out, int prec) {
  const int u = blockIdx.x;
  const int b = find_inst(L.pre, L.n_inst, u);
  const Inst& I = L.insts[b];
  const long idx = (long)(u - L.pre[b]) * 256 + threadIdx.x;
  if (idx >= (long)I.n_x * I.cands) return;
  const int i = (int)(idx / I.cands), q = (int)(idx % I.cands);
  const double c = I.u0[idx];
  const int S = I.segs;
  out[idx] = I.f[i] * b_from_parts(I, i, q, S, c, prec);
}

// ------------------------------------------------------------- selection
//
// One kernel per level (k_select), one block per kSelWaves * 64 / W
// points.  A point is handled by a group of W lanes: a wave (W = 64), or,
// where the level's set and the incumbent fit in 32 lanes (cands + 2 <= 32),
// an aligned half-wave (W = 32, two points per wave).  Lane q of the group
// holds candidate q of the level (lane `cands` the best so far, or at level
// 0 the incumbent, whose FP32-path B is kept for the final comparison).
// FP32 minimum and tie band; a one-member band (and the FP64 arithmetics)
// decides at once, otherwise the members without an FP64 value queue their
// positions in the block, which evaluates their FP64 values (from the
// moment table, or FP64 window sums where the instance has none) and then
// decides.  On the last level a decided point runs the comparison with the
// incumbent the same way.  Every cross-lane step of a group (minimum, ballot, shuffle)
// reads lanes of its own group only, and every branch depends on values
// uniform over the group, so the two groups of a wave may take different
// paths.  W is a function of the instance alone.

__device__ __forceinline__ int pad_chunk(int n) { return (n + kEvalChunk - 1) / kEvalChunk * kEvalChunk; }

int32_t units_select(const Inst& I) {
  const int pts = kSelWaves * (kWave / sel_width(I));  // points per block
  return (I.n_x + pts - 1) / pts;
}

template <int W>
__device__ __forceinline__ int grp_base() {
  return W == kWave ? 0 : ((int)threadIdx.x % kWave) / W * W;
}
template <int W>
__device__ __forceinline__ unsigned long long grp_ballot(bool p) {
  const unsigned long long b = __ballot(p);
  if constexpr (W == kWave) return b;
  else return (b >> grp_base<W>()) & ((1ull << W) - 1ull);
}
template <int W, typename T>
__device__ __forceinline__ T grp_shfl(T v, int l) {
  return __shfl(v, grp_base<W>() + l);
}
template <int W>
__device__ __forceinline__ double grp_min_d(double v) {
  for (int o = W / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}

// The selection rule on FP64 values among the lanes with `member`: ties
// within tau64 of the minimum, the one nearest the incumbent wins, then the
// smaller u, then the lower lane.  Returns the group lane (0 if there is
// none).
template <int W>
__device__ int tie_rule(bool member, double c, double Bf, double uinc, int lane, double tau64) {
  const double big = INFINITY;
  const double m = grp_min_d<W>(member ? Bf : big);
  const bool band = member && Bf <= m * (1.0 + tau64);
  double k1 = band ? fabs(c - uinc) : big;
  double k2 = band ? c : big;
  int k3 = band ? lane : INT_MAX;
  for (int o = W / 2; o > 0; o >>= 1) {
    const double o1 = __shfl_xor(k1, o), o2 = __shfl_xor(k2, o);
    const int o3 = __shfl_xor(k3, o);
    const bool take = (o1 < k1) || (o1 == k1 && (o2 < k2 || (o2 == k2 && o3 < k3)));
    if (take) { k1 = o1; k2 = o2; k3 = o3; }
  }
  return k3 == INT_MAX ? 0 : k3;
}

// FP32 tie band over the lanes with `in_set`: B32 <= m (1 + tau) + kappa
// sqrt(m), tau covering the relative error of the weights and the sum and
// kappa sqrt(m) the rounding of z - u1 (|dB| grows like sqrt(B)).  Returns
// the member mask over the group (0 when no candidate is finite).
template <int W>
__device__ unsigned long long band32(bool in_set, double B32, double tau) {
  const bool fin = in_set && isfinite(B32);
  const double m32 = grp_min_d<W>(fin ? B32 : INFINITY);
  if (!(m32 < INFINITY)) return 0ull;
  return grp_ballot<W>(fin && B32 <= m32 * (1.0 + tau) + kKappa32 * sqrt(m32));
}

// This lane's candidate of the level: position, FP32-path B and (FP64 mode,
// or the carried best) its FP64 B.
// The arithmetics whose marginal costs are FP64 values (decided directly by
// the rule, with no FP32 band).
template <int PREC>
constexpr bool F64 = PREC == UCP_FP64 || PREC == UCP_FP64_GT;

template <int PREC>
__device__ void level_view(const Inst& I, int level, int i, int lane, double& c, double& B32, double& B64,
                           bool& in_set) {
  const int K = I.cands;
  const int kq = level == 0 ? K + 1 : K;
  c = 0.0;
  B32 = INFINITY;
  B64 = NAN;
  if (lane < kq) {
    c = cand_pos(I, level, lane, i);
    B32 = b_from_parts(I, i, lane, I.segs, c, PREC);
    if (F64<PREC>) B64 = B32;
  }
  if (level > 0 && lane == K) {
    c = I.cbest[i];
    B32 = I.b32best[i];
    B64 = I.b64best[i];
  }
  in_set = level == 0 ? lane < K : lane <= K;
}

__device__ __forceinline__ void count_evals(const Inst& I, int n) {
  if (n && I.terms)
    atomicAdd(I.terms + kCountEvals + (blockIdx.x & (kCountSlots - 1)) * kCountStride, (unsigned long long)n);
}

// Points whose decision needs FP64 values queue them in their block:
// kind 1 = the level's band members (lane q), kind 2 = the comparison of
// the level's winner (lane 0) with the incumbent (lane 1), kind 3 = on the
// last level, the band members and (lane cands + 1) the incumbent, whose
// sum the comparison that follows may need.
struct Queued {
  unsigned long long todo;  // group lanes whose sum is needed
  int kind;                 // 0: nothing queued
  double c;                 // this lane's position
};

// The FP64 value of the incumbent where a lane of the set sits at its
// position with a known FP64 value (the carried best often does), else NaN.
template <int W>
__device__ __forceinline__ double inc_from_set(bool in_set, double c, double B64, double uinc) {
  const unsigned long long m = grp_ballot<W>(in_set && c == uinc && !isnan(B64));
  return m ? grp_shfl<W>(B64, __ffsll((long long)m) - 1) : NAN;
}

// Whether the FP32 band of the pair {b0, b1} (as band32 forms it) holds both.
__device__ __forceinline__ bool pair_band_both(double b0, double b1, double tau) {
  if (!isfinite(b0) || !isfinite(b1)) return false;
  const double m = fmin(b0, b1);
  const double lim = m * (1.0 + tau) + kKappa32 * sqrt(m);
  return b0 <= lim && b1 <= lim;
}

template <int W, bool T>
__device__ void finish_point(const Inst& I, int i, double res, double Bres, double x, int lane, int want_l0) {
  if (want_l0 && isnan(Bres)) {
    if constexpr (T) Bres = I.k2 * res * res + gt_noise_sum<true>(I, x + res);
    else Bres = I.k2 * res * res + b64_wave<W>(I, x + res, lane);
  }
  if (lane == 0) {
    I.u0_next[i] = res;
    if (!isfinite(res)) atomicOr(I.flags, 1);
    if (want_l0) I.L0_out[i] = I.f[i] * Bres;
  }
}

// Comparison of the level's winner (cw, B32w, B64w) with the incumbent
// (B64i its FP64 value where known).  In the band phase (inline_eval =
// false) a two-member band is queued (returned in Q); in the resolve phase
// missing FP64 sums are evaluated in place.
template <int PREC, int W, bool T>
__device__ void accept(const Inst& I, int i, double x, double uinc, double cw, double B32w, double B64w, double B64i,
                       int lane, bool inline_eval, int want_l0, int& n_eval, Queued& Q) {
  if (cw == uinc) {
    finish_point<W, T>(I, i, uinc, B64w, x, lane, want_l0);
    return;
  }
  const double B32i = I.b32inc[i];
  const bool in2 = lane < 2;
  const double c2 = lane == 0 ? cw : uinc;
  const double b32 = lane == 0 ? B32w : B32i;
  double b64 = lane == 0 ? B64w : (F64<PREC> ? B32i : B64i);
  if (F64<PREC>) {
    const bool fin = in2 && isfinite(b32);
    const int w = tie_rule<W>(fin, c2, b32, uinc, lane, I.tau64);
    if (grp_ballot<W>(fin) == 0ull && lane == 0) atomicOr(I.flags, 1);
    finish_point<W, T>(I, i, grp_shfl<W>(c2, w), grp_shfl<W>(b64, w), x, lane, want_l0);
    return;
  }
  const unsigned long long mask = band32<W>(in2, b32, I.tau32);
  if (mask == 0ull) {
    if (lane == 0) atomicOr(I.flags, 1);
    finish_point<W, T>(I, i, uinc, NAN, x, lane, want_l0);
    return;
  }
  if (__popcll(mask) == 1) {
    const int w = __ffsll((long long)mask) - 1;
    finish_point<W, T>(I, i, grp_shfl<W>(c2, w), grp_shfl<W>(b64, w), x, lane, want_l0);
    return;
  }
  const unsigned long long todo = grp_ballot<W>(in2 && isnan(b64));
  if (!inline_eval && todo) {
    Q.todo = todo;
    Q.kind = 2;
    Q.c = c2;
    return;
  }
  if constexpr (T) {  // each lane its own value from the moment table
    if ((todo >> lane) & 1ull) b64 = I.k2 * c2 * c2 + gt_noise_sum<true>(I, x + c2);
    n_eval += __popcll(todo);
  } else if (todo == 3ull) {  // both: one pass over their windows
    const double c0 = grp_shfl<W>(c2, 0), c1 = grp_shfl<W>(c2, 1);
    const double z[2] = {x + c0, x + c1};
    double v[2];
    b64_multi<2, W>(I, z, lane, v);
    if (lane == 0) b64 = I.k2 * c0 * c0 + v[0];
    if (lane == 1) b64 = I.k2 * c1 * c1 + v[1];
    n_eval += 2;
  } else if (todo) {
    const int L = __ffsll((long long)todo) - 1;
    const double cl = grp_shfl<W>(c2, L);
    const double v = I.k2 * cl * cl + b64_wave<W>(I, x + cl, lane);
    if (lane == L) b64 = v;
    ++n_eval;
  }
  const int w = tie_rule<W>(in2, c2, b64, uinc, lane, I.tau64);
  finish_point<W, T>(I, i, grp_shfl<W>(c2, w), grp_shfl<W>(b64, w), x, lane, want_l0);
}

// Band phase for one point: decide it, or return in Q the FP64 sums it
// needs; the lane's view of the level (c, B32, B64, in_set) is returned for
// the resolve phase.
template <int PREC, int W, bool T>
__device__ void band_point(const Inst& I, int level, int i, int lane, int want_l0, int& n_eval, Queued& Q,
                           double& c, double& B32, double& B64, bool& in_set) {
  const int K = I.cands;
  const double uinc = I.u0[i];
  const double x = I.x_lo + (double)i * I.dx;
  level_view<PREC>(I, level, i, lane, c, B32, B64, in_set);
  if (level == 0 && lane == K) I.b32inc[i] = B32;
  int w;
  if (F64<PREC>) {
    const bool fin = in_set && isfinite(B32);
    if (grp_ballot<W>(fin) == 0ull && lane == 0) atomicOr(I.flags, 1);
    w = tie_rule<W>(fin, c, B32, uinc, lane, I.tau64);
  } else {
    const unsigned long long mask = band32<W>(in_set, B32, I.tau32);
    if (mask == 0ull) {
      if (lane == 0) atomicOr(I.flags, 1);
      w = 0;
    } else if (__popcll(mask) == 1) {
      w = __ffsll((long long)mask) - 1;
    } else {
      const bool member = (mask >> lane) & 1ull;
      const unsigned long long todo = grp_ballot<W>(member && isnan(B64));
      if (todo) {  // FP64 sums needed: the resolve phase decides
        Q.todo = todo;
        Q.kind = 1;
        Q.c = c;
        // last level: if the incumbent could share the FP32 band of the
        // winner, whichever member wins, its sum is queued too, so the
        // comparison in the resolve phase evaluates nothing itself.  (An
        // incumbent that is itself a member, as the carried best, gets its
        // FP64 value as a member.)
        if (level == I.levels - 1 && K + 1 < W && !grp_ballot<W>(member && c == uinc)) {
          const double b32i = I.b32inc[i];
          if (grp_ballot<W>(member && pair_band_both(B32, b32i, I.tau32))) {
            Q.todo |= 1ull << (K + 1);
            Q.kind = 3;
            if (lane == K + 1) Q.c = uinc;
          }
        }
        return;
      }
      w = tie_rule<W>(member, c, B64, uinc, lane, I.tau64);
    }
  }
  const double cw = grp_shfl<W>(c, w), B32w = grp_shfl<W>(B32, w), B64w = grp_shfl<W>(B64, w);
  if (lane == 0) {
    I.cbest[i] = cw;
    I.b32best[i] = B32w;
    I.b64best[i] = B64w;
  }
  if (level == I.levels - 1) {
    const double B64i = inc_from_set<W>(in_set, c, B64, uinc);
    accept<PREC, W, T>(I, i, x, uinc, cw, B32w, B64w, B64i, lane, false, want_l0, n_eval, Q);
  }
}

// Resolve phase for a point that queued FP64 sums; `qv` is this lane's
// queued sum (NaN where the lane queued none).
template <int PREC, int W, bool T>
__device__ void resolve_point(const Inst& I, int level, int i, int lane, int want_l0, int& n_eval, int kind,
                              double qv, double c, double B32, double B64, bool in_set) {
  const double uinc = I.u0[i];
  const double x = I.x_lo + (double)i * I.dx;
  if (kind != 2) {
    const unsigned long long mask = band32<W>(in_set, B32, I.tau32);
    const bool member = (mask >> lane) & 1ull;
    if (member && isnan(B64)) B64 = qv;
    const int w = tie_rule<W>(member, c, B64, uinc, lane, I.tau64);
    const double cw = grp_shfl<W>(c, w), B32w = grp_shfl<W>(B32, w), B64w = grp_shfl<W>(B64, w);
    if (lane == 0) {
      I.cbest[i] = cw;
      I.b32best[i] = B32w;
      I.b64best[i] = B64w;
    }
    if (level == I.levels - 1) {
      Queued Q;
      double B64i = inc_from_set<W>(in_set, c, B64, uinc);
      if (kind == 3 && isnan(B64i)) B64i = grp_shfl<W>(qv, I.cands + 1);
      accept<PREC, W, T>(I, i, x, uinc, cw, B32w, B64w, B64i, lane, true, want_l0, n_eval, Q);
    }
  } else {
    // the queued incumbent comparison: lane 0 the winner, lane 1 the incumbent
    const double cw = I.cbest[i], B64w = I.b64best[i];
    const bool in2 = lane < 2;
    const double c2 = lane == 0 ? cw : uinc;
    const double b32 = lane == 0 ? I.b32best[i] : I.b32inc[i];
    const double b64 = lane == 0 ? (isnan(B64w) ? qv : B64w) : qv;
    const unsigned long long mask = band32<W>(in2, b32, I.tau32);
    const bool member = (mask >> lane) & 1ull;
    const int w = tie_rule<W>(member, c2, b64, uinc, lane, I.tau64);
    finish_point<W, T>(I, i, grp_shfl<W>(c2, w), grp_shfl<W>(b64, w), x, lane, want_l0);
  }
}

// A queued FP64 value of the block: point and position (i < 0 pads).
struct SelItem {
  int32_t i;
  double c;
};

// Largest number of queue entries of one point: cands + 2 lanes, padded to
// whole chunks.
constexpr int kSelCapMax = (UCP_MAX_CANDS + 2 + kEvalChunk - 1) / kEvalChunk * kEvalChunk;

// One selection block (kSelWaves waves, G points per wave):
//  1. band: every group decides its point or queues the FP64 sums it needs
//     in the block's queue (a point's entries padded to whole chunks of
//     kEvalChunk, so the positions that share one pass depend on the point
//     alone);
//  2. eval: with a moment table (T) one thread per queued position, its
//     value from the table; else the block's whole waves take the chunks in
//     turn, one pass of b64_multi over the union of a chunk's windows;
//     results to LDS;
//  3. resolve: the queued points decide on their FP64 values.
// Every dependency stays in the block, so one launch serves a level.
template <int PREC, int W, bool T>
__device__ void select_block(const Inst& I, int local, int level, int want_l0, SelItem* sq, double* sres,
                             int* s_cnt) {
  constexpr int G = kWave / W;
  constexpr int NP = kSelWaves * G;  // points per block
  const int wid = threadIdx.x / kWave, g = ((int)threadIdx.x % kWave) / W, lane = (int)threadIdx.x % W;
  const int grp = wid * G + g;
  const int i = local * NP + grp;
  const bool have = i < I.n_x;
  Queued Q;
  Q.todo = 0ull;
  Q.kind = 0;
  Q.c = 0.0;
  double c = 0.0, B32 = INFINITY, B64 = NAN;
  bool in_set = false;
  int n_eval = 0;
  if (have) band_point<PREC, W, T>(I, level, i, lane, want_l0, n_eval, Q, c, B32, B64, in_set);
  const int nq = __popcll(Q.todo);
  if (lane == 0) s_cnt[grp] = pad_chunk(nq);
  __syncthreads();
  int base = 0, total = 0;
  for (int k = 0; k < NP; ++k) {
    const int n = s_cnt[k];
    base += k < grp ? n : 0;
    total += n;
  }
  if (Q.todo) {
    if ((Q.todo >> lane) & 1ull) {
      SelItem it;
      it.i = i;
      it.c = Q.c;
      sq[base + __popcll(Q.todo & ((1ull << lane) - 1ull))] = it;
    }
    if (lane >= nq && lane < pad_chunk(nq)) {
      SelItem it;
      it.i = -1;
      it.c = 0.0;
      sq[base + lane] = it;
    }
  }
  __syncthreads();
  int n_gt = 0;  // values this thread took from the moment table
  if (total) {
    if constexpr (T) {
      // one thread per queued position, its value from the moment table
      for (int e = (int)threadIdx.x; e < total; e += kSelWaves * kWave) {
        const SelItem it = sq[e];
        if (it.i < 0) continue;
        const double z = (I.x_lo + (double)it.i * I.dx) + it.c;
        sres[e] = I.k2 * it.c * it.c + gt_noise_sum(I, z);
        ++n_gt;
      }
    } else {
      const int wl = (int)threadIdx.x % kWave;
      for (int ch = wid; ch * kEvalChunk < total; ch += kSelWaves) {
        SelItem it[kEvalChunk];
#pragma unroll
        for (int q = 0; q < kEvalChunk; ++q) it[q] = sq[ch * kEvalChunk + q];
        int cnt = 0;  // valid entries lead the chunk
#pragma unroll
        for (int q = 0; q < kEvalChunk; ++q) cnt += it[q].i >= 0;
        if (cnt == 0) continue;
        const double x = I.x_lo + (double)it[0].i * I.dx;
        double z[kEvalChunk], v[kEvalChunk];
#pragma unroll
        for (int q = 0; q < kEvalChunk; ++q) z[q] = x + (q < cnt ? it[q].c : it[0].c);  // static indices only
        if (cnt == 1) v[0] = b64_wave(I, z[0], wl);
        else if (cnt == 2) b64_multi<2>(I, z, wl, v);
        else if (cnt == 3) b64_multi<3>(I, z, wl, v);
        else b64_multi<4>(I, z, wl, v);
        if (wl == 0) {
#pragma unroll
          for (int q = 0; q < kEvalChunk; ++q)
            if (q < cnt) sres[ch * kEvalChunk + q] = I.k2 * it[q].c * it[q].c + v[q];
        }
        n_eval += wl == 0 ? cnt : 0;
      }
    }
    __syncthreads();
    if (Q.kind) {
      const double qv = (Q.todo >> lane) & 1ull ? sres[base + __popcll(Q.todo & ((1ull << lane) - 1ull))] : NAN;
      resolve_point<PREC, W, T>(I, level, i, lane, want_l0, n_eval, Q.kind, qv, c, B32, B64, in_set);
    }
  }
  // one count per wave: the group leaders' counts (band and resolve, and
  // the wave's chunk counts, kept by its first lane) and every thread's
  // values from the moment table
  int ne = (lane == 0 ? n_eval : 0) + n_gt;
  for (int o = kWave / 2; o > 0; o >>= 1) ne += __shfl_xor(ne, o);
  if ((int)threadIdx.x % kWave == 0) count_evals(I, ne);
}

// T: the instances of this launch take their FP64 values from the moment
// table (FP32 modes on grids that have one; the window-sum code is then not
// compiled in, which keeps the kernel's registers, and so its occupancy,
// those of the band and resolve phases alone).  The table variant waits on
// memory most of its cycles and runs at 8 waves per SIMD (64 registers, a
// few spilled), where more waves hide more of that latency than the spills
// cost.
template <int PREC, bool T>
__global__ __launch_bounds__(kSelWaves * kWave, T ? 8 : 2) void k_select(Launch L, int level, int want_l0) {
  __shared__ SelItem sq[kSelWaves * 2 * kSelCapMax];
  __shared__ double sres[kSelWaves * 2 * kSelCapMax];
  __shared__ int s_cnt[kSelWaves * 2];
  const int u = blockIdx.x;
  const int b = find_inst(L.pre, L.n_inst, u);
  const Inst& I = L.insts[b];
  const int local = u - L.pre[b];
  if (sel_width(I) == 32) {
    select_block<PREC, 32, T>(I, local, level, want_l0, sq, sres, s_cnt);
  } else {
    // 4 points per block, half of a tile of partial sums.  Workgroups go to
    // the XCDs in turn (workgroup w to XCD w mod 8), so within each 16
    // blocks the two halves of a tile go to blocks 8 apart: one XCD, one L2.
    const int units = L.pre[b + 1] - L.pre[b];
    int lb = local;
    if (local < units / 16 * 16) {
      const int r = local % 16;
      lb = local - r + 2 * (r % 8) + r / 8;
    }
    select_block<PREC, kWave, T>(I, lb, level, want_l0, sq, sres, s_cnt);
  }
}

static hipError_t launch_select_one(const Launch& L, int level, int prec, int want_l0, bool table, hipStream_t st,
                                    hipEvent_t e0, hipEvent_t e1) {
  const dim3 blk(kSelWaves * kWave);
  if (prec == UCP_FP64)
    hipExtLaunchKernelGGL((k_select<UCP_FP64, false>), dim3(L.total), blk, 0, st, e0, e1, 0, L, level, want_l0);
  else if (prec == UCP_FP64_GT)  // decides on FP64 values directly; its table serves any L_0 left open
    hipExtLaunchKernelGGL((k_select<UCP_FP64_GT, true>), dim3(L.total), blk, 0, st, e0, e1, 0, L, level, want_l0);
  else if (prec == UCP_FP32_KAHAN && table)
    hipExtLaunchKernelGGL((k_select<UCP_FP32_KAHAN, true>), dim3(L.total), blk, 0, st, e0, e1, 0, L, level, want_l0);
  else if (prec == UCP_FP32_KAHAN)
    hipExtLaunchKernelGGL((k_select<UCP_FP32_KAHAN, false>), dim3(L.total), blk, 0, st, e0, e1, 0, L, level, want_l0);
  else if (table)
    hipExtLaunchKernelGGL((k_select<UCP_FP32, true>), dim3(L.total), blk, 0, st, e0, e1, 0, L, level, want_l0);
  else
    hipExtLaunchKernelGGL((k_select<UCP_FP32, false>), dim3(L.total), blk, 0, st, e0, e1, 0, L, level, want_l0);
  return hipGetLastError();
}

hipError_t launch_select(const Launch& Lw, const Launch& Lt, int level, int prec, int want_l0, hipStream_t st,
                         hipEvent_t e0, hipEvent_t e1) {
  const bool w = Lw.total > 0, t = Lt.total > 0;
  hipError_t e = hipSuccess;
  if (w) e = launch_select_one(Lw, level, prec, want_l0, false, st, e0, t ? nullptr : e1);
  if (e == hipSuccess && t) e = launch_select_one(Lt, level, prec, want_l0, true, st, w ? nullptr : e0, e1);
  return e;
}

// ------------------------------------------------------------ u1 update
//
// u1_j = y_j - v_j with v_j = sum_i w_ij d_ij / sum_i w_ij, d_ij = y_j - x1_i,
// w_ij = exp(l_ij - M), l_ij = log f_i - d_ij^2 / 2 (the conditional mean
// written around the y nodes so the numerator terms stay small).  Unit =
// (tile of y nodes, slice of x nodes), each lane taking u1_npl consecutive
// nodes of the tile; each slice keeps an online maximum M, and the combine
// kernel merges the slices in a fixed order.  Chunks of x nodes whose
// weights are negligible for the whole tile are skipped.

// y nodes per tile: one block of lanes, u1_npl nodes each
__host__ __device__ inline int u1_tile_nodes(const Inst& I) { return kU1Block * I.u1_npl; }
__host__ __device__ inline int u1_tiles(const Inst& I) { return (I.n_y + u1_tile_nodes(I) - 1) / u1_tile_nodes(I); }
__host__ __device__ inline int u1_slen(const Inst& I) { return (I.n_x + I.u1_slices - 1) / I.u1_slices; }
__host__ __device__ inline int u1_cps(const Inst& I) { return (u1_slen(I) + kU1Chunk - 1) / kU1Chunk; }

int32_t units_u1_partial(const Inst& I) { return u1_tiles(I) * I.u1_slices; }
// The combine gives each y node a group of kU1Grp lanes, lane g taking the
// slices g, g + kU1Grp, ... (at most 32 slices), so a block covers
// kU1Block / kU1Grp nodes.
constexpr int kU1Grp = 8;
int32_t units_u1_combine(const Inst& I) { return (I.n_y + kU1Block / kU1Grp - 1) / (kU1Block / kU1Grp); }

// Block maximum of v (every thread gets it); `sw` holds one value per wave.
__device__ __forceinline__ double block_max_d(double v, double* sw) {
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  if (threadIdx.x % kWave == 0) sw[threadIdx.x / kWave] = v;
  __syncthreads();
  v = sw[0];
  for (int w = 1; w < (int)blockDim.x / kWave; ++w) v = fmax(v, sw[w]);
  return v;
}

// Culling data of the u1 sums, each part depending on one tile or one chunk
// alone (so the partial-sum blocks need not recompute it): per tile the
// lower bound lb of its logit maxima, per chunk of a slice the range of its
// x1 and its largest log f (NaN when the chunk holds a non-finite x1 or
// log f).  Layout: [tiles] bounds, then [slices][chunks per slice][3].
size_t u1stat_doubles(const Inst& I) { return (size_t)u1_tiles(I) + (size_t)I.u1_slices * u1_cps(I) * 3; }

// One unit per tile (its bound) and one per slice (its chunks).
int32_t units_u1_stats(const Inst& I) { return u1_tiles(I) + I.u1_slices; }

__global__ __launch_bounds__(kU1Block) void k_u1_stats(Launch L) {
  constexpr int NW = kU1Block / kWave;
  __shared__ double sb[3][NW];
  const int u = blockIdx.x;
  const int b = find_inst(L.pre, L.n_inst, u);
  const Inst& I = L.insts[b];
  const int local = u - L.pre[b];
  const int ntiles = u1_tiles(I);
  const int tile = local < ntiles ? local : -1;
  const int slice = local < ntiles ? -1 : local - ntiles;
  const int nx = I.n_x;
  const double x_lo = I.x_lo, dx = I.dx;
  const double h2 = 0.5 * I.isw * I.isw;
  const glb_dptr u0g = (glb_dptr)I.u0, lfg = (glb_dptr)I.logf;
  if (tile >= 0) {
    // A lower bound on the logit maximum M_j of every node of the tile: any x
    // node gives one, M_j >= l_ij >= log f_i - max over the tile's y of
    // (y - x1_i)^2 / (2 s^2); every kU1Sample-th node is taken.
    const int j0 = tile * u1_tile_nodes(I), j1 = min(I.n_y, j0 + u1_tile_nodes(I)) - 1;
    const double ya = I.y_lo + (double)j0 * I.dy, yb = I.y_lo + (double)j1 * I.dy;
    double lb = -INFINITY;
    for (int i = (int)threadIdx.x * kU1Sample; i < nx; i += kU1Block * kU1Sample) {
      const double x1 = (x_lo + (double)i * dx) + u0g[i];
      const double da = ya - x1, db = yb - x1;
      lb = fmax(lb, lfg[i] - h2 * fmax(da * da, db * db));  // NaN terms drop out
    }
    lb = block_max_d(lb, sb[0]);
    if (threadIdx.x == 0) I.u1stat[tile] = lb;
  } else {
    const int slen = u1_slen(I);
    const int i0 = slice * slen, i1 = min(nx, i0 + slen);
    double* cs = I.u1stat + u1_tiles(I) + (size_t)slice * u1_cps(I) * 3;
    for (int c0 = i0, k = 0; c0 < i1; c0 += kU1Chunk, ++k) {
      const int cn = min(kU1Chunk, i1 - c0);
      double xmn = INFINITY, xmx = -INFINITY, fmx = -INFINITY;
      bool bad = false;
      for (int t = threadIdx.x; t < cn; t += kU1Block) {
        const int i = c0 + t;
        const double x1 = (x_lo + (double)i * dx) + u0g[i];
        const double lf = lfg[i];
        xmn = fmin(xmn, x1);
        xmx = fmax(xmx, x1);
        fmx = fmax(fmx, lf);
        bad |= !isfinite(x1) || isnan(lf);
      }
      for (int o = kWave / 2; o > 0; o >>= 1) {
        xmn = fmin(xmn, __shfl_xor(xmn, o));
        xmx = fmax(xmx, __shfl_xor(xmx, o));
        fmx = fmax(fmx, __shfl_xor(fmx, o));
      }
      const bool wbad = __ballot(bad) != 0ull;
      if (threadIdx.x % kWave == 0) {
        sb[0][threadIdx.x / kWave] = xmn;
        sb[1][threadIdx.x / kWave] = xmx;
        sb[2][threadIdx.x / kWave] = wbad ? NAN : fmx;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        bool cbad = false;
        for (int w = 0; w < NW; ++w) {
          xmn = fmin(xmn, sb[0][w]);
          xmx = fmax(xmx, sb[1][w]);
          fmx = fmax(fmx, sb[2][w]);
          cbad |= isnan(sb[2][w]);
        }
        cs[k * 3 + 0] = xmn;
        cs[k * 3 + 1] = xmx;
        cs[k * 3 + 2] = cbad ? NAN : fmx;
      }
      __syncthreads();
    }
  }
}

// The sums of one unit, NPL consecutive y nodes per lane.  Around the
// middle node y_c of the tile, y_j - x1_i = eta_j + D_i with eta_j = y_j -
// y_c and D_i = y_c - x1_i, so the log2 weight (s the noise sd)
//   log2(e) (log f_i - (y_j - x1_i)^2 / (2 s^2) - M) = P_i + Q_j + E_j D_i,
// P_i = log2(e) (log f_i - D_i^2 / (2 s^2)) staged per node, Q_j =
// -log2(e) (M + eta_j^2 / (2 s^2)) and E_j = -log2(e) eta_j / s^2 per lane:
// one add and one fma in FP64.  The FP64 numerator sums w D_i (one fma);
// eta_j times the denominator is added once at the end (sum_i w (y_j -
// x1_i) = sum_i w D_i + eta_j sum_i w).  With NPL > 1 the lane's first node
// takes its weight as above and node m + 1 the weight of node m times
// R_i = exp2(-log2(e) dy D_i / s^2), staged per x node (one exponential per
// x node and lane instead of one per term).  That product differs from
// node m + 1's weight by the factor exp(-(eta_{m+1}^2 - eta_m^2) / (2 s^2)),
// which depends on neither i nor the slice: every slice's sums of the node
// carry it, so it cancels in the combine's ratio and is left out.  M is one
// shift for the lane's nodes, taken from its second node's logits: the
// nodes lie within a few dy of each other (dy <= kU1NplMaxStep noise sds),
// so no weight leaves the FP32 range.
template <int PREC, int NPL>
__device__ __forceinline__ void u1_partial_sums(const Inst& I, int tile, int slice, double* sD, double* sP,
                                                float* sDf, float* sPf, double* sR) {
  const int tn = kU1Block * NPL;
  const int jb = tile * tn + (int)threadIdx.x * NPL;  // the lane's first node
  const bool act = jb < I.n_y;
  const double y = I.y_lo + (double)(NPL == 1 && !act ? 0 : jb) * I.dy;
  const int slen = u1_slen(I);
  const int i0 = slice * slen, i1 = min(I.n_x, i0 + slen);
  const double log2e = 1.4426950408889634073599246810019;
  // the noise variance s^2 divides every squared distance: h2 = 1 / (2 s^2)
  const double is2 = I.isw * I.isw, h2 = 0.5 * is2;
  const double c2 = h2 * log2e;
  const int j0 = tile * tn, j1 = min(I.n_y, j0 + tn) - 1;
  const double ya = I.y_lo + (double)j0 * I.dy, yb = I.y_lo + (double)j1 * I.dy;
  // the instance is read through a generic pointer, which the LDS stores
  // below could alias: its fields and arrays are taken into registers and
  // global-space pointers once
  const double x_lo = I.x_lo, dx = I.dx, dy = I.dy;
  const glb_dptr u0g = (glb_dptr)I.u0, lfg = (glb_dptr)I.logf;
  const double lb = I.u1stat[tile];  // lower bound of the tile's logit maxima (k_u1_stats)
  const double* cstat = I.u1stat + u1_tiles(I) + (size_t)slice * u1_cps(I) * 3;
  const double yc = I.y_lo + (double)((j0 + j1) / 2) * I.dy;
  const double eta = y - yc;
  const double E = -log2e * eta * is2;
  const double Es = -log2e * dy * is2;  // log2 of the weight ratio per node and unit D
  // the node whose logits set the shift
  const double etaR = NPL > 1 ? eta + dy : eta;
  const float etaRf = (float)etaR;
  double M = -INFINITY, den[NPL], num[NPL];
#pragma unroll
  for (int m = 0; m < NPL; ++m) den[m] = num[m] = 0.0;
  for (int c0 = i0, k = 0; c0 < i1; c0 += kU1Chunk, ++k) {
    const int cn = min(kU1Chunk, i1 - c0);
    // the chunk's largest possible logit over the tile's nodes:
    // max log f - (distance from [ya, yb] to [min x1, max x1])^2 / (2 s^2);
    // skipped weights are below exp(-kU1Cull) of the largest: none of the
    // sums moves (n_x exp(-kU1Cull) < 2^-60).  A chunk with a non-finite x1
    // or log f (NaN maximum) is never skipped.
    const double xmn = cstat[k * 3 + 0], xmx = cstat[k * 3 + 1], fmx = cstat[k * 3 + 2];
    const double dist = fmax(0.0, fmax(xmn - yb, ya - xmx));
    if (!isnan(fmx) && fmx - h2 * dist * dist < lb - kU1Cull) continue;
    __syncthreads();  // the previous chunk's readers are done
    for (int t = threadIdx.x; t < cn; t += kU1Block) {
      const int i = c0 + t;
      const double x1 = (x_lo + (double)i * dx) + u0g[i];
      const double lf = lfg[i];
      const double D = yc - x1;
      const double Pn = lf - h2 * D * D;
      sD[t] = D;
      sP[t] = Pn * log2e;
      sDf[t] = (float)(D * is2);
      sPf[t] = (float)Pn;
      if (NPL > 1) sR[t] = exp2(Es * D);
    }
    __syncthreads();
    // chunk maximum of the logits, in FP32: only a shift, any value near
    // the maximum works (the sums below use exact FP64 exponents)
    float mcf = -INFINITY;
    for (int t = 0; t < cn; ++t) mcf = fmaxf(mcf, fmaf(-etaRf, sDf[t], sPf[t]));
    const double mc = (double)mcf - h2 * etaR * etaR;
    if (mc > M) {  // rescale what was summed under the old maximum
      const double r = M == -INFINITY ? 0.0 : exp(M - mc);
#pragma unroll
      for (int m = 0; m < NPL; ++m) {
        den[m] *= r;
        num[m] *= r;
      }
      M = mc;
    }
    if (!(M > -INFINITY)) continue;  // every logit is -inf (or NaN): nothing to add
    const double Q = -log2e * M - c2 * eta * eta;
    for (int t = 0; t < cn; ++t) {
      const double D = sD[t];
      const double a = fma(E, D, sP[t] + Q);  // log2 of the shifted weight
      // FP64 weight in FP64 mode, else the FP32 exp2 of the rounded exponent
      double w = PREC == UCP_FP64 ? exp2(a) : (double)__builtin_amdgcn_exp2f((float)a);
      num[0] = fma(w, D, num[0]);
      den[0] += w;
      if (NPL > 1) {
        const double R = sR[t];
#pragma unroll
        for (int m = 1; m < NPL; ++m) {
          w *= R;
          num[m] = fma(w, D, num[m]);
          den[m] += w;
        }
      }
    }
  }
#pragma unroll
  for (int m = 0; m < NPL; ++m) {
    const int j = jb + m;
    if (j >= I.n_y) break;
    const double em = NPL == 1 ? eta : (I.y_lo + (double)j * dy) - yc;
    double* o = I.u1part + ((size_t)slice * I.n_y + j) * 3;
    o[0] = M;
    o[1] = num[m] + em * den[m];
    o[2] = den[m];
  }
}

template <int PREC>
__global__ __launch_bounds__(kU1Block, 5) void k_u1_partial(Launch L) {
  __shared__ double sD[kU1Chunk];    // D_i = y_c - x1_i
  __shared__ double sP[kU1Chunk];    // P_i = log2(e) (log f_i - D_i^2 / (2 s^2)), s the noise sd
  __shared__ float sDf[kU1Chunk];    // D_i / s^2 in FP32 (maximum pass only)
  __shared__ float sPf[kU1Chunk];    // log f_i - D_i^2 / (2 s^2) in FP32 (maximum pass only)
  __shared__ double sR[kU1Chunk];    // R_i = exp2(-log2(e) dy D_i / s^2) (several nodes per lane only)
  const int u = blockIdx.x;
  const int b = find_inst(L.pre, L.n_inst, u);
  const Inst& I = L.insts[b];
  const int local = u - L.pre[b];
  const int slice = local % I.u1_slices;
  const int tile = local / I.u1_slices;
  if (I.u1_npl == kU1Npl)
    u1_partial_sums<PREC, kU1Npl>(I, tile, slice, sD, sP, sDf, sPf, sR);
  else
    u1_partial_sums<PREC, 1>(I, tile, slice, sD, sP, sDf, sPf, sR);
}

__global__ __launch_bounds__(kU1Block) void k_u1_combine(Launch L) {
  const int u = blockIdx.x;
  const int b = find_inst(L.pre, L.n_inst, u);
  const Inst& I = L.insts[b];
  const int g = (int)threadIdx.x % kU1Grp;
  const int j = (u - L.pre[b]) * (kU1Block / kU1Grp) + (int)threadIdx.x / kU1Grp;
  const bool act = j < I.n_y;
  const int jj = act ? j : I.n_y - 1;
  constexpr int kPer = 32 / kU1Grp;  // slices per lane
  double pm[kPer], pn[kPer], pd[kPer];
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const int s = g + t * kU1Grp;
    pm[t] = -INFINITY;
    pn[t] = pd[t] = 0.0;
    if (s < I.u1_slices) {
      const double* p = I.u1part + ((size_t)s * I.n_y + jj) * 3;
      pm[t] = p[0];
      pn[t] = p[1];
      pd[t] = p[2];
    }
  }
  double M = pm[0];
#pragma unroll
  for (int t = 1; t < kPer; ++t) M = fmax(M, pm[t]);
  for (int o = 1; o < kU1Grp; o <<= 1) M = fmax(M, __shfl_xor(M, o));
  double num = 0.0, den = 0.0;
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    if (!(pm[t] > -INFINITY)) continue;
    const double r = exp(pm[t] - M);
    num += pn[t] * r;
    den += pd[t] * r;
  }
  // fixed pairing over the group: the same order for every node and launch
  for (int o = 1; o < kU1Grp; o <<= 1) {
    num += __shfl_xor(num, o);
    den += __shfl_xor(den, o);
  }
  if (!act || g != 0) return;
  const double y = I.y_lo + (double)j * I.dy;
  const double vres = num / den;
  const double u1 = y - vres;
  I.u1[j] = u1;
  // the residual from the stored u1, exactly as k_v_from_u1 forms it, so a
  // u0 update sees the same FP32 residual whether u1 came from here or
  // from the caller
  I.v[j] = (float)(I.alpha * (y - u1));
  if (!isfinite(u1)) atomicOr(I.flags, 1);
}

hipError_t launch_u1_partial(const Launch& Ls, const Launch& L, int prec, hipStream_t st, hipEvent_t e0) {
  if (L.total == 0) return hipSuccess;
  hipExtLaunchKernelGGL(k_u1_stats, dim3(Ls.total), dim3(kU1Block), 0, st, e0, nullptr, 0, Ls);
  if (prec == UCP_FP64 || prec == UCP_FP64_GT)  // the u1 update of UCP_FP64_GT is UCP_FP64's
    hipLaunchKernelGGL(k_u1_partial<UCP_FP64>, dim3(L.total), dim3(kU1Block), 0, st, L);
  else if (prec == UCP_FP32_KAHAN)
    hipLaunchKernelGGL(k_u1_partial<UCP_FP32_KAHAN>, dim3(L.total), dim3(kU1Block), 0, st, L);
  else
    hipLaunchKernelGGL(k_u1_partial<UCP_FP32>, dim3(L.total), dim3(kU1Block), 0, st, L);
  return hipGetLastError();
}

hipError_t launch_u1_combine(const Launch& L, hipStream_t st, hipEvent_t e1) {
  if (L.total == 0) return hipSuccess;
  hipExtLaunchKernelGGL(k_u1_combine, dim3(L.total), dim3(kU1Block), 0, st, nullptr, e1, 0, L);
  return hipGetLastError();
}

// ------------------------------------------------------------- objective

// With a moment table (built from the u1 the objective is taken with) one
// thread per point, else one wave per kJPts points.
int32_t units_j_rows(const Inst& I) {
  return I.gts ? (I.n_x + kJWaves * kWave - 1) / (kJWaves * kWave) : (I.n_x + kJWaves * kJPts - 1) / (kJWaves * kJPts);
}

__global__ __launch_bounds__(kJWaves * kWave) void k_j_rows(Launch L) {
  const int u = blockIdx.x;
  const int b = find_inst(L.pre, L.n_inst, u);
  const Inst& I = L.insts[b];
  if (I.gts) {  // the point's noise sum from the moment table
    const int i = (u - L.pre[b]) * (kJWaves * kWave) + (int)threadIdx.x;
    if (i >= I.n_x) return;
    const double u0 = I.u0[i];
    const double z = (I.x_lo + (double)i * I.dx) + u0;
    I.jrow[i] = I.f[i] * (I.k2 * u0 * u0 + gt_noise_sum(I, z));
    return;
  }
  const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  // kJPts consecutive points per wave: their x1 mostly coincide (the
  // controller is a staircase), so one pass over the union of their windows
  const int i0 = ((u - L.pre[b]) * kJWaves + wid) * kJPts;
  if (i0 >= I.n_x) return;
  const int cnt = min(kJPts, I.n_x - i0);
  double u0[kJPts], z[kJPts], v[kJPts];
#pragma unroll
  for (int p = 0; p < kJPts; ++p) {
    const int i = i0 + min(p, cnt - 1);
    u0[p] = I.u0[i];
    z[p] = (I.x_lo + (double)i * I.dx) + u0[p];
  }
  if (cnt == 1) v[0] = b64_wave(I, z[0], lane);
  else if (cnt == 2) b64_multi<2>(I, z, lane, v);
  else if (cnt == 3) b64_multi<3>(I, z, lane, v);
  else b64_multi<4>(I, z, lane, v);
  if (lane == 0) {
#pragma unroll
    for (int p = 0; p < kJPts; ++p)
      if (p < cnt) I.jrow[i0 + p] = I.f[i0 + p] * (I.k2 * u0[p] * u0[p] + v[p]);
  }
}

// One block per instance: fixed-order sum of the rows (each thread four
// independent strided partial sums, so the loads overlap, then a tree),
// times dx.  `t` selects the J_hist entry.
constexpr int kJRed = 1024;
__global__ __launch_bounds__(kJRed) void k_j_reduce(Launch L, int t) {
  __shared__ double red[kJRed];
  const int b = find_inst(L.pre, L.n_inst, blockIdx.x);
  const Inst& I = L.insts[b];
  const int n = I.n_x;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int i = threadIdx.x;
  for (; i + 3 * kJRed < n; i += 4 * kJRed) {
    s0 += I.jrow[i];
    s1 += I.jrow[i + kJRed];
    s2 += I.jrow[i + 2 * kJRed];
    s3 += I.jrow[i + 3 * kJRed];
  }
  for (; i < n; i += kJRed) s0 += I.jrow[i];
  red[threadIdx.x] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  for (int o = kJRed / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double J = I.dx * red[0];
    I.J_out[t] = J;
    if (!isfinite(J)) atomicOr(I.flags, 1);
  }
}

hipError_t launch_j_rows(const Launch& L, hipStream_t st, hipEvent_t e0) {
  if (L.total == 0) return hipSuccess;
  hipExtLaunchKernelGGL(k_j_rows, dim3(L.total), dim3(kJWaves * kWave), 0, st, e0, nullptr, 0, L);
  return hipGetLastError();
}

hipError_t launch_j_reduce_t(const Launch& L, int t, hipStream_t st, hipEvent_t e1) {
  if (L.total == 0) return hipSuccess;
  hipExtLaunchKernelGGL(k_j_reduce, dim3(L.total), dim3(kJRed), 0, st, nullptr, e1, 0, L, t);
  return hipGetLastError();
}

hipError_t launch_j_reduce(const Launch& L, hipStream_t st) { return launch_j_reduce_t(L, 0, st); }

// ----------------------------------------------------------- u0 advance

__global__ __launch_bounds__(256) void k_copy_u0(Launch L) {
  const int u = blockIdx.x;
  const int b = find_inst(L.pre, L.n_inst, u);
  const Inst& I = L.insts[b];
  const int i = (u - L.pre[b]) * 256 + threadIdx.x;
  if (i < I.n_x) I.u0[i] = I.u0_next[i];
}

hipError_t launch_copy_u0(const Launch& L, hipStream_t st) {
  if (L.total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_u0, dim3(L.total), dim3(256), 0, st, L);
  return hipGetLastError();
}

// Residual v_j = alpha (y_j - u1_j) in FP32 from a given u1 (argmin and
// marginal-cost calls, where u1 is an input).
__global__ __launch_bounds__(256) void k_v_from_u1(Launch L) {
  const int u = blockIdx.x;
  const int b = find_inst(L.pre, L.n_inst, u);
  const Inst& I = L.insts[b];
  const int j = (u - L.pre[b]) * 256 + threadIdx.x;
  if (j >= I.n_y) return;
  const double y = I.y_lo + (double)j * I.dy;
  I.v[j] = (float)(I.alpha * (y - I.u1[j]));
}

hipError_t launch_v_from_u1(const Launch& L, hipStream_t st) {
  if (L.total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_v_from_u1, dim3(L.total), dim3(256), 0, st, L);
  return hipGetLastError();
}

hipError_t launch_finish_free(const Launch& L, double* out, int prec, hipStream_t st) {
  if (L.total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mc_finish, dim3(L.total), dim3(256), 0, st, L, out, prec);
  return hipGetLastError();
}

// ------------------------------------------- generic solver (Algorithm 1)
//
// The paper's own minimiser per controller: local updates (modified Newton
// on the marginal cost) and partial exhaustion over the values a controller
// takes on the neighbouring grid nodes (the domain ball of Eq. (2)).  All in
// FP64; the kernels take the instance record directly (one instance).

namespace {

// B, B' and B'' of one position over a group of W lanes: the window of
// b64_wave (11 noise sds around the nearest node), the same shifted
// Gaussian with its reseeded recurrence, and with T_j = (y_j - z) / s^2,
// e_j = z - u1_j the three sums
//   S0 = sum g e^2,  S1 = sum g (T e^2 + 2 e),
//   S2 = sum g ((T^2 - 1/s^2) e^2 + 4 T e + 2),
// since d phi_s(y - z)/dz = T phi_s.  Returns dy/(s sqrt(2 pi))
// exp(-delta^2/2) times each.
template <int W>
__device__ void b64_derivs(const Inst& I, double z, int lane, double& S0, double& S1, double& S2) {
  const int jr = nearest_node(I, z);
  const double delta = ((I.y_lo + (double)jr * I.dy) - z) * I.isw;  // in noise sds
  const int klo = max(-I.nw64, -jr), khi = min(I.nw64, I.n_y - 1 - jr);
  const int n = khi - klo + 1;
  const double dy = I.dy * I.isw, D = (double)W * dy;
  const double q = exp(-D * D);
  const double is2 = I.isw * I.isw;
  const int rs = I.rs64;
  glb_dptr u1 = (glb_dptr)(I.u1 + jr + klo + lane);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  B64Walk w;
  const int steps = (n + W - 1) / W;
  for (int m = 0; m < steps; ++m) {
    if ((m & (rs - 1)) == 0) b64_reseed<W>(w, klo, lane, m, dy, delta, D);
    if (lane + W * m < n) {
      const double t = (double)(klo + lane + W * m) * dy + delta;  // (y_j - z) / s
      const double T = t * I.isw;
      const double e = z - u1[W * m];
      const double e2 = e * e;
      a0 = fma(w.g, e2, a0);
      a1 = fma(w.g, fma(T, e2, 2.0 * e), a1);
      a2 = fma(w.g, fma(T * T - is2, e2, fma(4.0 * T, e, 2.0)), a2);
    }
    w.g *= w.r;
    w.r *= q;
  }
  const double sc = I.phi_scale * exp(-0.5 * delta * delta);
  S0 = sc * grp_sum_d<W>(a0);
  S1 = sc * grp_sum_d<W>(a1);
  S2 = sc * grp_sum_d<W>(a2);
}

// The selection rule among n values (relative tie band, nearest to the
// incumbent, then the smaller u), serially in one lane.
__device__ int pick_serial(int n, const double* c, const double* B, double inc, double tie) {
  double m = B[0];
  for (int s = 1; s < n; ++s) m = fmin(m, B[s]);
  const double thr = m * (1.0 + tie);
  int best = -1;
  double bd = 0.0;
  for (int s = 0; s < n; ++s) {
    if (!(B[s] <= thr)) continue;
    const double d = fabs(c[s] - inc);
    if (best < 0 || d < bd || (d == bd && c[s] < c[best])) {
      best = s;
      bd = d;
    }
  }
  return best < 0 ? 0 : best;
}

}  // namespace

// Local update of u0: one wave per point.
__global__ __launch_bounds__(256) void k_a1_local_u0(const Inst* __restrict__ Ip, double tau,
                                                     const double* __restrict__ u0_in, double* __restrict__ u0_out) {
  const Inst& I = *Ip;
  const int lane = (int)threadIdx.x % kWave;
  const int i = blockIdx.x * (256 / kWave) + (int)threadIdx.x / kWave;
  if (i >= I.n_x) return;  // whole waves
  const double u = u0_in[i];
  const double x = I.x_lo + (double)i * I.dx;
  double S0, S1, S2;
  b64_derivs<kWave>(I, x + u, lane, S0, S1, S2);
  if (lane == 0) {
    const double B1 = 2.0 * I.k2 * u + S1, B2 = 2.0 * I.k2 + S2;
    const double v = B2 > 0.0 ? u - B1 / B2 : u - tau * B1;
    u0_out[i] = v;
    if (!isfinite(v)) atomicOr(I.flags, 1);
  }
}

// Partial exhaustion of u0: one wave per point; the R = 2r + 1 values of
// u0_in at the nodes within r (an out-of-grid neighbour stands in as the
// point's own value, which the set holds anyway) share one FP64 pass over
// the union of their windows.
template <int R>
__global__ __launch_bounds__(256) void k_a1_pe_u0(const Inst* __restrict__ Ip, double tie,
                                                  const double* __restrict__ u0_in, double* __restrict__ u0_out) {
  const Inst& I = *Ip;
  const int lane = (int)threadIdx.x % kWave;
  const int i = blockIdx.x * (256 / kWave) + (int)threadIdx.x / kWave;
  if (i >= I.n_x) return;
  constexpr int r = R / 2;
  const double x = I.x_lo + (double)i * I.dx;
  const double inc = u0_in[i];
  double c[R], z[R], v[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const int k = i - r + m;
    c[m] = (k >= 0 && k < I.n_x) ? u0_in[k] : inc;
    z[m] = x + c[m];
  }
  b64_multi<R>(I, z, lane, v);
  if (lane == 0) {
    double B[R];
#pragma unroll
    for (int m = 0; m < R; ++m) B[m] = I.k2 * c[m] * c[m] + v[m];
    const double res = c[pick_serial(R, c, B, inc, tie)];
    u0_out[i] = res;
    if (!isfinite(res)) atomicOr(I.flags, 1);
  }
}

// Partial exhaustion of u1, first pass: as k_u1_partial<UCP_FP64> (x nodes
// of one slice staged in LDS, FP64 weights max-shifted, negligible chunks
// skipped, one or u1_npl consecutive y nodes per lane, the weights of a
// lane's later nodes by the staged ratio R_i), accumulating for each node j
// the weighted moments T_a = sum_i w (x1_i - u1_in[j])^a, a = 0, 1, 2.  The
// candidates' sums follow from them: for c_m = u1_in[j] + delta_m,
// sum_i w (x1_i - c_m)^2 = T_2 - 2 delta_m T_1 + delta_m^2 T_0.  The ratio
// leaves out a factor common to the node's slices and candidates, which
// the selection rule (relative to the minimum) does not see.  Writes
// [slice][n_y][2 r + 2]: the slice's maximum and T_0, T_1, T_2.
template <int NPL>
__device__ __forceinline__ void a1_u1_moments(const Inst& I, int tile, int slice, const double* __restrict__ u1_in,
                                              double* __restrict__ part, int stride, double* sD, double* sP,
                                              double* sR, double* sb) {
  constexpr int NW = kU1Block / kWave;
  const int tn = kU1Block * NPL;
  const int jb = tile * tn + (int)threadIdx.x * NPL;  // the lane's first node
  const int slen = (I.n_x + I.u1_slices - 1) / I.u1_slices;
  const int i0 = slice * slen, i1 = min(I.n_x, i0 + slen);
  const double log2e = 1.4426950408889634073599246810019;
  const double is2 = I.isw * I.isw, h2 = 0.5 * is2, c2 = h2 * log2e;
  const int nx = I.n_x;
  const double x_lo = I.x_lo, dx = I.dx, dy = I.dy;
  const glb_dptr u0g = (glb_dptr)I.u0, lfg = (glb_dptr)I.logf;
  double cref[NPL];  // each node's own u1 value, the moments' origin
#pragma unroll
  for (int m = 0; m < NPL; ++m) cref[m] = u1_in[min(jb + m, I.n_y - 1)];
  // a lower bound on the logit maximum of every node of the tile (as in
  // k_u1_stats): chunks whose logits all lie kU1Cull below it are skipped
  const int j0 = tile * tn, j1 = min(I.n_y, j0 + tn) - 1;
  const double ya = I.y_lo + (double)j0 * dy, yb = I.y_lo + (double)j1 * dy;
  double lb = -INFINITY;
  for (int i = (int)threadIdx.x * kU1Sample; i < nx; i += kU1Block * kU1Sample) {
    const double x1 = (x_lo + (double)i * dx) + u0g[i];
    const double da = ya - x1, db = yb - x1;
    lb = fmax(lb, lfg[i] - h2 * fmax(da * da, db * db));
  }
  lb = block_max_d(lb, sb);
  // logits around the tile's middle node y_c as in k_u1_partial
  const double yc = I.y_lo + (double)((j0 + j1) / 2) * dy;
  const double eta = (I.y_lo + (double)(NPL == 1 ? min(jb, I.n_y - 1) : jb) * dy) - yc;
  const double E = -log2e * eta * is2;
  const double Es = -log2e * dy * is2;
  const double etaR = NPL > 1 ? eta + dy : eta;  // the node whose logits set the shift
  double M = -INFINITY, T0[NPL], T1[NPL], T2[NPL];
#pragma unroll
  for (int m = 0; m < NPL; ++m) T0[m] = T1[m] = T2[m] = 0.0;
  for (int c0 = i0; c0 < i1; c0 += kU1Chunk) {
    const int cn = min(kU1Chunk, i1 - c0);
    __syncthreads();  // the previous chunk's readers are done
    double xmn = INFINITY, xmx = -INFINITY, fmx = -INFINITY;
    bool bad = false;
    for (int t = threadIdx.x; t < cn; t += kU1Block) {
      const int i = c0 + t;
      const double x1 = (x_lo + (double)i * dx) + u0g[i];
      const double lf = lfg[i];
      const double D = yc - x1;
      sD[t] = D;
      sP[t] = (lf - h2 * D * D) * log2e;
      if (NPL > 1) sR[t] = exp2(Es * D);
      xmn = fmin(xmn, x1);
      xmx = fmax(xmx, x1);
      fmx = fmax(fmx, lf);
      bad |= !isfinite(x1) || isnan(lf);
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
      xmn = fmin(xmn, __shfl_xor(xmn, o));
      xmx = fmax(xmx, __shfl_xor(xmx, o));
      fmx = fmax(fmx, __shfl_xor(fmx, o));
    }
    const bool wbad = __ballot(bad) != 0ull;
    if (threadIdx.x % kWave == 0) {
      sb[NW + threadIdx.x / kWave] = xmn;
      sb[2 * NW + threadIdx.x / kWave] = xmx;
      sb[3 * NW + threadIdx.x / kWave] = wbad ? NAN : fmx;
    }
    __syncthreads();
    for (int w = 0; w < NW; ++w) {
      xmn = fmin(xmn, sb[NW + w]);
      xmx = fmax(xmx, sb[2 * NW + w]);
      fmx = fmax(fmx, sb[3 * NW + w]);
      bad |= isnan(sb[3 * NW + w]);
    }
    const double dist = fmax(0.0, fmax(xmn - yb, ya - xmx));
    if (!bad && fmx - h2 * dist * dist < lb - kU1Cull) continue;
    // the chunk's largest logit of the shift node (in log2 units)
    const double ER = -log2e * etaR * is2;
    double mc = -INFINITY;
    for (int t = 0; t < cn; ++t) mc = fmax(mc, fma(ER, sD[t], sP[t]));
    mc = mc / log2e - h2 * etaR * etaR;
    if (mc > M) {
      const double sc = M == -INFINITY ? 0.0 : exp(M - mc);
#pragma unroll
      for (int m = 0; m < NPL; ++m) {
        T0[m] *= sc;
        T1[m] *= sc;
        T2[m] *= sc;
      }
      M = mc;
    }
    if (!(M > -INFINITY)) continue;
    const double Q = -log2e * M - c2 * eta * eta;
    for (int t = 0; t < cn; ++t) {
      const double D = sD[t];
      double w = exp2(fma(E, D, sP[t] + Q));
      const double x1 = yc - D;
#pragma unroll
      for (int m = 0; m < NPL; ++m) {
        if (m) w *= sR[t];
        const double e = x1 - cref[m];
        const double we = w * e;
        T0[m] += w;
        T1[m] += we;
        T2[m] = fma(we, e, T2[m]);
      }
    }
  }
#pragma unroll
  for (int m = 0; m < NPL; ++m) {
    const int j = jb + m;
    if (j >= I.n_y) break;
    double* o = part + ((size_t)slice * I.n_y + j) * stride;
    o[0] = M;
    o[1] = T0[m];
    o[2] = T1[m];
    o[3] = T2[m];
  }
}

template <int R>
__global__ __launch_bounds__(kU1Block, 4) void k_a1_pe_u1_partial(const Inst* __restrict__ Ip,
                                                                  const double* __restrict__ u1_in,
                                                                  double* __restrict__ part) {
  __shared__ double sD[kU1Chunk];  // D_i = y_c - x1_i
  __shared__ double sP[kU1Chunk];  // log2(e) (log f_i - D_i^2 / (2 s^2))
  __shared__ double sR[kU1Chunk];  // exp2(-log2(e) dy D_i / s^2) (several nodes per lane only)
  __shared__ double sb[4 * (kU1Block / kWave)];
  const Inst& I = *Ip;
  const int u = blockIdx.x;
  const int slice = u % I.u1_slices;
  const int tile = u / I.u1_slices;
  if (I.u1_npl == kU1Npl)
    a1_u1_moments<kU1Npl>(I, tile, slice, u1_in, part, R + 1, sD, sP, sR, sb);
  else
    a1_u1_moments<1>(I, tile, slice, u1_in, part, R + 1, sD, sP, sR, sb);
}

// Second pass: merge the slices' moments at the common maximum (in slice
// order), form each candidate's sum from them and apply the selection rule
// among the R candidates, the node's own value the incumbent.
template <int R>
__global__ __launch_bounds__(256) void k_a1_pe_u1_select(const Inst* __restrict__ Ip, double tie,
                                                         const double* __restrict__ u1_in,
                                                         const double* __restrict__ part, double* __restrict__ u1_out) {
  const Inst& I = *Ip;
  constexpr int r = R / 2;
  const int j = blockIdx.x * 256 + (int)threadIdx.x;
  if (j >= I.n_y) return;
  double M = -INFINITY;
  for (int s = 0; s < I.u1_slices; ++s) M = fmax(M, part[((size_t)s * I.n_y + j) * (R + 1)]);
  double T0 = 0.0, T1 = 0.0, T2 = 0.0;
  for (int s = 0; s < I.u1_slices; ++s) {
    const double* p = part + ((size_t)s * I.n_y + j) * (R + 1);
    if (!(p[0] > -INFINITY)) continue;
    const double sc = exp(p[0] - M);
    T0 += p[1] * sc;
    T1 += p[2] * sc;
    T2 += p[3] * sc;
  }
  const double inc = u1_in[j];
  double C[R], c[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const int k = j - r + m;
    c[m] = (k >= 0 && k < I.n_y) ? u1_in[k] : inc;
    const double d = c[m] - inc;
    C[m] = fma(d, fma(d, T0, -2.0 * T1), T2);
  }
  const double res = c[pick_serial(R, c, C, inc, tie)];
  u1_out[j] = res;
  if (!isfinite(res)) atomicOr(I.flags, 1);
}

hipError_t launch_a1_local_u0(const Inst* dI, int n_x, double tau, const double* u0_in, double* u0_out,
                              hipStream_t st) {
  const int blocks = (n_x + 3) / 4;
  hipLaunchKernelGGL(k_a1_local_u0, dim3(blocks), dim3(256), 0, st, dI, tau, u0_in, u0_out);
  return hipGetLastError();
}

hipError_t launch_a1_pe_u0(const Inst* dI, int n_x, int r, double tie, const double* u0_in, double* u0_out,
                           hipStream_t st) {
  const int blocks = (n_x + 3) / 4;
  if (r == 1)
    hipLaunchKernelGGL(k_a1_pe_u0<3>, dim3(blocks), dim3(256), 0, st, dI, tie, u0_in, u0_out);
  else
    hipLaunchKernelGGL(k_a1_pe_u0<5>, dim3(blocks), dim3(256), 0, st, dI, tie, u0_in, u0_out);
  return hipGetLastError();
}

hipError_t launch_a1_pe_u1(const Inst& I, const Inst* dI, int r, double tie, const double* u1_in, double* part,
                           double* u1_out, hipStream_t st) {
  const int units = u1_tiles(I) * I.u1_slices;
  const int blocks = (I.n_y + 255) / 256;
  if (r == 1) {
    hipLaunchKernelGGL(k_a1_pe_u1_partial<3>, dim3(units), dim3(kU1Block), 0, st, dI, u1_in, part);
    hipLaunchKernelGGL(k_a1_pe_u1_select<3>, dim3(blocks), dim3(256), 0, st, dI, tie, u1_in, part, u1_out);
  } else {
    hipLaunchKernelGGL(k_a1_pe_u1_partial<5>, dim3(units), dim3(kU1Block), 0, st, dI, u1_in, part);
    hipLaunchKernelGGL(k_a1_pe_u1_select<5>, dim3(blocks), dim3(256), 0, st, dI, tie, u1_in, part, u1_out);
  }
  return hipGetLastError();
}

}  // namespace ucp
