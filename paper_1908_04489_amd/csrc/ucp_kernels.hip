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
//   k_select<P>    per point: level minimum, FP32 tie band, FP64
//                  re-evaluation of the band, selection rule, next bracket,
//                  and after the last level the comparison with the
//                  incumbent
//   k_u1_partial<P>/k_u1_combine   closed-form second controller
//   k_j_rows/k_j_reduce            objective in FP64, fixed-order reduction
#include <hip/hip_runtime.h>

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
// Butterfly sum: every lane ends with the same bits (each step adds the same
// two values, and IEEE addition is commutative).
__device__ __forceinline__ double wave_sum_d(double v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
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

// FP64 window sum for one position z, spread over the 64 lanes of a wave:
// returns dy/sqrt(2 pi) * sum_j phi(y_j - z) (z - u1_j)^2 over the nodes
// within kWin64 of the node nearest z.  The Gaussian is max-shifted to that
// node, g_k = exp(-(t_k^2 - delta^2)/2) = exp(-d (d + 2 delta)/2) with
// d = k dy, and the shift exp(-delta^2/2) is applied once at the end.
// Lane l takes k = klo + l + 64 m; along m the Gaussian obeys the exact
// recurrence g_{k+64} = g_k r_k, r_{k+64} = r_k q with
// r_k = exp(-64 dy t_k - (64 dy)^2 / 2) and q = exp(-(64 dy)^2), so two
// multiplies replace an exp; both are recomputed by exp every kReseed steps,
// which bounds the relative error of any weight by ~kReseed^2/2 ulp
// (5.7e-14).  Loads are issued kPrefetch at a time; two accumulators split
// the dependency chain of the sum.
constexpr int kReseed = 32;
constexpr int kPrefetch = 16;

__device__ double b64_wave(const Inst& I, double z, int lane) {
  const int jr = nearest_node(I, z);
  const double delta = (I.y_lo + (double)jr * I.dy) - z;
  const int klo = max(-I.nw64, -jr), khi = min(I.nw64, I.n_y - 1 - jr);
  const double dy = I.dy, D = (double)kWave * dy;
  const double q = exp(-D * D);
  const double* __restrict__ u1 = I.u1 + jr;
  double s0 = 0.0, s1 = 0.0;
  // this lane's nodes: k = klo + lane + 64 m for m = 0 .. steps - 1
  const int steps = (khi - klo + kWave) / kWave;
  for (int m0 = 0; m0 < steps; m0 += kReseed) {
    const int kb = klo + lane + kWave * m0;
    const double d = (double)kb * dy;
    double g = exp(-0.5 * d * (d + 2.0 * delta));
    double r = exp(-D * (d + delta) - 0.5 * D * D);
    for (int p0 = 0; p0 < kReseed && m0 + p0 < steps; p0 += kPrefetch) {
      double uv[kPrefetch];
#pragma unroll
      for (int mm = 0; mm < kPrefetch; ++mm) {  // loads first, so they overlap
        const int k = kb + kWave * (p0 + mm);
        uv[mm] = k <= khi ? u1[k] : z;  // past the window: e = 0, no term
      }
#pragma unroll
      for (int mm = 0; mm < kPrefetch; mm += 2) {
        const double e0 = z - uv[mm];
        s0 = fma(g * e0, e0, s0);
        g *= r;
        r *= q;
        const double e1 = z - uv[mm + 1];
        s1 = fma(g * e1, e1, s1);
        g *= r;
        r *= q;
      }
    }
  }
  const double s = wave_sum_d(s0 + s1);
  return I.phi_scale * exp(-0.5 * delta * delta) * s;
}

// Algorithmic terms of one (point, candidate): the y nodes within kWin32
// noise sds of z (the work the method needs for FP64-level accuracy; the
// kernels may evaluate a few more).  Summed per wave, one atomic per wave.
__device__ __forceinline__ void count_terms(const Inst& I, double z, bool act, int lane) {
  long long n = 0;
  if (act && I.terms) {
    double lo = ceil((z - kWin32 - I.y_lo) * I.inv_dy);
    double hi = floor((z + kWin32 - I.y_lo) * I.inv_dy);
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

// Offset table of the marginal-cost kernel: G_k = exp(-(k dy)^2 / 2) =
// exp2(-(k alpha dy)^2) for |k| <= nw32, rounded once from FP64.
__global__ __launch_bounds__(256) void k_gtab(Launch L) {
  const int u = blockIdx.x;
  const int b = find_inst(L.pre, L.n_inst, u);
  const Inst& I = L.insts[b];
  const int k = (u - L.pre[b]) * 256 + (int)threadIdx.x - I.nw32;
  if (k > I.nw32) return;
  const double d = (double)k * I.dy;
  I.gtab[k + I.nw32] = (float)exp(-0.5 * d * d);
}

int32_t units_gtab(const Inst& I) { return (2 * I.nw32 + 1 + 255) / 256; }

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
// Every lane of a wave is at the same window offset k, so G_k is one LDS
// broadcast; E_k costs one v_exp_f32 per block of 8 offsets times the
// per-lane constants exp2(beta m), m < 8.  The residual z - u1 = v - T with
// T = alpha t (v = alpha (y - u1), formed in FP64 by the u1 kernel).  After
// the shift every weight is <= 1, so FP32 neither overflows nor underflows
// where terms matter.  The block stages the residual nodes it touches and
// the G values of its offsets in LDS (falls back to global loads for the
// residual when its node range exceeds kMcLds, e.g. across a jump of the
// controller).

int32_t units_mc(const Inst& I, int level) {
  if (level >= 0 && level >= I.levels) return 0;
  const int tiles = (I.n_x + kMcBlock - 1) / kMcBlock;
  const int kq = level == 0 ? I.cands + 1 : I.cands;  // level < 0: explicit candidates
  return tiles * kq * I.segs;
}

typedef const __attribute__((address_space(3))) float* lds_cptr;
typedef const __attribute__((address_space(1))) float* glb_cptr;

__device__ __forceinline__ void kahan_add(float x, float& acc, float& comp) {
  const float y = x - comp;
  const float t = acc + y;
  comp = (t - acc) - y;
  acc = t;
}

constexpr int kMcUnroll = 8;

// Per-lane constants of one unit.
struct McLane {
  float aDy;             // alpha dy
  float Dl;              // alpha delta
  float beta;            // -2 alpha^2 dy delta
  float R[kMcUnroll];    // exp2(beta m)
  float Dm[kMcUnroll];   // Dl + m alpha dy
};

// Offsets k in [k0, k1] (wave-uniform bounds, every lane in range): blocks of
// 8 terms summed plainly in two chains, each block sum added with
// compensation (KAHAN) or plainly.
template <bool KAHAN, typename P>
__device__ __forceinline__ void mc_bulk(P v, lds_cptr G, int k0, int k1, const McLane& c, float& acc,
                                        float& comp) {
  int k = k0;
  for (; k + kMcUnroll - 1 <= k1; k += kMcUnroll) {
    const float kf = (float)k;
    // E_{k+m} = E_k R_m: the common factor E_k multiplies the block sum
    const float E0 = __builtin_amdgcn_exp2f(c.beta * kf);
    float b0 = 0.0f, b1 = 0.0f;
#pragma unroll
    for (int m = 0; m < kMcUnroll; m += 2) {
      const float T0 = fmaf(kf, c.aDy, c.Dm[m]);
      const float g0 = G[k + m] * c.R[m];
      const float e0 = v[k + m] - T0;
      const float T1 = fmaf(kf, c.aDy, c.Dm[m + 1]);
      const float g1 = G[k + m + 1] * c.R[m + 1];
      const float e1 = v[k + m + 1] - T1;
      b0 = fmaf(g0 * e0, e0, b0);
      b1 = fmaf(g1 * e1, e1, b1);
    }
    if (KAHAN) kahan_add(E0 * (b0 + b1), acc, comp);
    else acc = fmaf(E0, b0 + b1, acc);
  }
  for (; k <= k1; ++k) {
    const float kf = (float)k;
    const float g = G[k] * __builtin_amdgcn_exp2f(c.beta * kf);
    const float e = v[k] - fmaf(kf, c.aDy, c.Dl);
    if (KAHAN) kahan_add((g * e) * e, acc, comp);
    else acc = fmaf(g * e, e, acc);
  }
}

// Offsets k in [k0, k1] restricted to the lane's own range [klo, khi].
template <bool KAHAN, typename P>
__device__ __forceinline__ void mc_masked(P v, lds_cptr G, int k0, int k1, int klo, int khi, const McLane& c,
                                          float& acc, float& comp) {
  for (int k = k0; k <= k1; ++k) {
    if (k >= klo && k <= khi) {
      const float kf = (float)k;
      const float g = G[k] * __builtin_amdgcn_exp2f(c.beta * kf);
      const float e = v[k] - fmaf(kf, c.aDy, c.Dl);
      if (KAHAN) kahan_add((g * e) * e, acc, comp);
      else acc = fmaf(g * e, e, acc);
    }
  }
}

// The lane's window [klo, khi] (empty when klo > khi): the range common to
// every non-empty lane of the wave runs unmasked, the ragged ends masked.
template <bool KAHAN, typename P>
__device__ __forceinline__ void mc_lane(P v, lds_cptr G, int klo, int khi, const McLane& c, float& acc,
                                        float& comp) {
  const bool empty = klo > khi;
  const int kc_lo = __builtin_amdgcn_readfirstlane(wave_max_i(empty ? INT_MIN : klo));
  const int kc_hi = __builtin_amdgcn_readfirstlane(wave_min_i(empty ? INT_MAX : khi));
  const int ku_lo = __builtin_amdgcn_readfirstlane(wave_min_i(empty ? INT_MAX : klo));
  const int ku_hi = __builtin_amdgcn_readfirstlane(wave_max_i(empty ? INT_MIN : khi));
  if (ku_lo > ku_hi || empty) return;
  if (kc_lo > kc_hi) {
    mc_masked<KAHAN>(v, G, ku_lo, ku_hi, klo, khi, c, acc, comp);
    return;
  }
  mc_masked<KAHAN>(v, G, ku_lo, kc_lo - 1, klo, khi, c, acc, comp);
  mc_bulk<KAHAN>(v, G, kc_lo, kc_hi, c, acc, comp);
  mc_masked<KAHAN>(v, G, kc_hi + 1, ku_hi, klo, khi, c, acc, comp);
}

template <int PREC>
__global__ __launch_bounds__(kMcBlock) void k_mc32(Launch L, int level) {
  constexpr bool KAHAN = PREC == UCP_FP32_KAHAN;
  __shared__ float sv[kMcLds];
  __shared__ float sg[kMcSegMax];
  __shared__ int sred[4][kMcBlock / kWave];
  const int u = blockIdx.x;
  const int b = find_inst(L.pre, L.n_inst, u);
  const Inst& I = L.insts[b];
  int local = u - L.pre[b];
  const int S = I.segs;
  const int kq = level < 0 ? I.cands : (level == 0 ? I.cands + 1 : I.cands);
  const int pstride = level < 0 ? I.cands : I.cands + 1;
  const int seg = local % S;
  local /= S;
  const int q = local % kq;
  const int tile = local / kq;
  const int i = tile * kMcBlock + (int)threadIdx.x;
  const bool act = i < I.n_x;
  const int ii = act ? i : I.n_x - 1;

  const double c = cand_pos(I, level, q, ii);
  const double x = I.x_lo + (double)ii * I.dx;
  const double z = x + c;
  const int jr = nearest_node(I, z);
  const double delta = (I.y_lo + (double)jr * I.dy) - z;
  const int nw = I.nw32;
  const int seglen = (2 * nw + 1 + S - 1) / S;
  const int s_lo = -nw + seg * seglen;
  const int s_hi = min(nw, s_lo + seglen - 1);
  int klo = max(s_lo, -jr), khi = min(s_hi, I.n_y - 1 - jr);
  if (!act) { klo = 1; khi = 0; }

  // node range and offset range of the block, for LDS staging
  const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const bool ne = klo <= khi;
  const int jlo = wave_min_i(ne ? jr + klo : INT_MAX);
  const int jhi = wave_max_i(ne ? jr + khi : INT_MIN);
  const int klw = wave_min_i(ne ? klo : INT_MAX);
  const int khw = wave_max_i(ne ? khi : INT_MIN);
  if (lane == 0) {
    sred[0][wid] = jlo;
    sred[1][wid] = jhi;
    sred[2][wid] = klw;
    sred[3][wid] = khw;
  }
  __syncthreads();
  int blo = INT_MAX, bhi = INT_MIN, bklo = INT_MAX, bkhi = INT_MIN;
  for (int w = 0; w < kMcBlock / kWave; ++w) {
    blo = min(blo, sred[0][w]);
    bhi = max(bhi, sred[1][w]);
    bklo = min(bklo, sred[2][w]);
    bkhi = max(bkhi, sred[3][w]);
  }
  if (seg == 0) {
    count_terms(I, z, act, lane);
    // terms this unit's (point, candidate) evaluates over all its segments
    long long ev = act ? (long long)(min(nw, I.n_y - 1 - jr) - max(-nw, -jr) + 1) : 0;
    for (int o = kWave / 2; o > 0; o >>= 1) ev += __shfl_xor(ev, o);
    if (lane == 0 && ev > 0 && I.terms)
      atomicAdd(I.terms + kCountEvalTerms + (blockIdx.x & (kCountSlots - 1)) * kCountStride, (unsigned long long)ev);
  }
  const bool staged = bhi >= blo && bhi - blo + 1 <= kMcLds;
  if (staged)
    for (int j = blo + (int)threadIdx.x; j <= bhi; j += kMcBlock) sv[j - blo] = I.v[j];
  // offsets lie inside the segment, so at most kMcSegMax of them
  if (bkhi >= bklo)
    for (int k = bklo + (int)threadIdx.x; k <= bkhi; k += kMcBlock) sg[k - bklo] = I.gtab[k + nw];
  __syncthreads();

  McLane cl;
  const double alpha = sqrt(kAlpha2);
  cl.aDy = (float)(alpha * I.dy);
  cl.Dl = (float)(alpha * delta);
  const double beta = -2.0 * kAlpha2 * I.dy * delta;
  cl.beta = (float)beta;
#pragma unroll
  for (int m = 0; m < kMcUnroll; ++m) {
    cl.R[m] = __builtin_amdgcn_exp2f((float)(beta * m));
    cl.Dm[m] = (float)(alpha * (delta + m * I.dy));
  }

  float acc = 0.0f, comp = 0.0f;
  lds_cptr G = (lds_cptr)(sg - (bkhi >= bklo ? bklo : 0));
  if (staged) {
    lds_cptr v = (lds_cptr)(sv + (jr - blo));
    mc_lane<KAHAN>(v, G, klo, khi, cl, acc, comp);
  } else {
    glb_cptr v = (glb_cptr)(I.v + jr);
    mc_lane<KAHAN>(v, G, klo, khi, cl, acc, comp);
  }
  if (act) I.part[((size_t)i * pstride + q) * S + seg] = KAHAN ? (double)acc - (double)comp : (double)acc;
}

// FP64 marginal cost (precision-study mode): lane = point, window kWin64,
// the same shifted Gaussian as b64_wave, walked node by node with the exact
// recurrence g_{k+1} = g_k r_k, r_{k+1} = r_k exp(-dy^2),
// r_k = exp(-dy t_k - dy^2/2), reseeded by exp every kReseed nodes.
__global__ __launch_bounds__(kMcBlock) void k_mc64(Launch L, int level) {
  const int u = blockIdx.x;
  const int b = find_inst(L.pre, L.n_inst, u);
  const Inst& I = L.insts[b];
  int local = u - L.pre[b];
  const int kq = level < 0 ? I.cands : (level == 0 ? I.cands + 1 : I.cands);
  const int pstride = level < 0 ? I.cands : I.cands + 1;
  const int q = local % kq;
  const int tile = local / kq;
  const int i = tile * kMcBlock + (int)threadIdx.x;
  const bool act = i < I.n_x;
  const double c = cand_pos(I, level, q, act ? i : I.n_x - 1);
  const double z = (I.x_lo + (double)(act ? i : I.n_x - 1) * I.dx) + c;
  count_terms(I, z, act, (int)threadIdx.x % kWave);
  if (!act) return;
  const int jr = nearest_node(I, z);
  const double delta = (I.y_lo + (double)jr * I.dy) - z;
  const int klo = max(-I.nw64, -jr), khi = min(I.nw64, I.n_y - 1 - jr);
  const double dy = I.dy, qd = exp(-dy * dy);
  const double* __restrict__ u1 = I.u1 + jr;
  double s0 = 0.0, s1 = 0.0;
  for (int k0 = klo; k0 <= khi; k0 += kReseed) {
    const double d = (double)k0 * dy;
    double g = exp(-0.5 * d * (d + 2.0 * delta));
    double r = exp(-dy * (d + delta) - 0.5 * dy * dy);
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
  I.part[(size_t)i * pstride + q] = s0 + s1;
}

hipError_t launch_mc(const Launch& L, int level, int prec, hipStream_t st) {
  if (L.total == 0) return hipSuccess;
  if (prec == UCP_FP64)
    hipLaunchKernelGGL(k_mc64, dim3(L.total), dim3(kMcBlock), 0, st, L, level);
  else if (prec == UCP_FP32_KAHAN)
    hipLaunchKernelGGL(k_mc32<UCP_FP32_KAHAN>, dim3(L.total), dim3(kMcBlock), 0, st, L, level);
  else
    hipLaunchKernelGGL(k_mc32<UCP_FP32>, dim3(L.total), dim3(kMcBlock), 0, st, L, level);
  return hipGetLastError();
}

// B from the partial sums of candidate lane q: k^2 c^2 + dy/sqrt(2 pi)
// exp(-delta^2/2) * sum (the FP32 sums carry the factor alpha^2).
__device__ __forceinline__ double b_from_parts(const Inst& I, int i, int q, int pstride, int S,
                                               double c, int prec) {
  const double z = (I.x_lo + (double)i * I.dx) + c;
  const int jr = nearest_node(I, z);
  const double delta = (I.y_lo + (double)jr * I.dy) - z;
  const double* p = I.part + ((size_t)i * pstride + q) * S;
  double s = 0.0;
  for (int g = 0; g < S; ++g) s += p[g];
  if (prec != UCP_FP64) s = s / kAlpha2;
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
  out[idx] = I.f[i] * b_from_parts(I, i, q, I.cands, S, c, prec);
}

// ------------------------------------------------------------- selection
//
// One wave per point.  Lane q holds candidate q of the level (lane `cands`
// holds the best so far from the previous level, or at level 0 the
// incumbent, whose FP32-path B is kept for the final comparison).

int32_t units_select(const Inst& I) { return (I.n_x + kSelWaves - 1) / kSelWaves; }

struct Pick {
  int lane;
  double B64;  // FP64 B of the pick (NaN if not evaluated)
};

// Selection rule over the lanes with in_set: in FP64 modes the band is
// B <= m (1 + tau64); in FP32 modes a band B32 <= m32 (1 + tau32) is formed
// first and its members are re-evaluated in FP64.  Among the FP64 band the
// member nearest the incumbent wins, then the smaller u, then the lower lane.
__device__ Pick select_rule(const Inst& I, bool in_set, double c, double B32, double B64, double x,
                            double uinc, int lane, int prec, int32_t* bad, int& n_eval) {
  const double big = INFINITY;
  const bool fin = in_set && isfinite(B32);
  const double m32 = wave_min_d(fin ? B32 : big);
  Pick r{0, NAN};
  if (!(m32 < big)) {  // no finite candidate: flag and keep lane 0
    if (lane == 0) atomicOr(bad, 1);
    r.lane = 0;
    r.B64 = __shfl(B64, 0);
    return r;
  }
  double Bf;  // FP64 value used by the rule
  bool band;
  if (prec == UCP_FP64) {
    Bf = B32;
    band = fin && B32 <= m32 * (1.0 + kTau64);
  } else {
    // FP32 band: relative part for the weights and the sum, absolute part
    // kKappa32 sqrt(m) for the rounding of z - u1 (|dB| grows like sqrt(B))
    const double tau = prec == UCP_FP32_KAHAN ? kTau32Kahan : kTau32Plain;
    const bool b32 = fin && B32 <= m32 * (1.0 + tau) + kKappa32 * sqrt(m32);
    const unsigned long long mask = __ballot(b32);
    if (__popcll(mask) == 1) {
      r.lane = __ffsll((long long)mask) - 1;
      r.B64 = __shfl(B64, r.lane);
      return r;
    }
    unsigned long long todo = __ballot(b32 && isnan(B64));
    while (todo) {
      const int L = __ffsll((long long)todo) - 1;
      todo &= todo - 1;
      const double cl = __shfl(c, L);
      const double v = I.k2 * cl * cl + b64_wave(I, x + cl, lane);
      if (lane == L) B64 = v;
      ++n_eval;
    }
    Bf = B64;
    const double m64 = wave_min_d(b32 ? B64 : big);
    band = b32 && B64 <= m64 * (1.0 + kTau64);
  }
  // lexicographic (|c - uinc|, c, lane) minimum over the band
  double k1 = band ? fabs(c - uinc) : big;
  double k2 = band ? c : big;
  int k3 = band ? lane : INT_MAX;
  for (int o = kWave / 2; o > 0; o >>= 1) {
    double o1 = __shfl_xor(k1, o), o2 = __shfl_xor(k2, o);
    int o3 = __shfl_xor(k3, o);
    bool take = (o1 < k1) || (o1 == k1 && (o2 < k2 || (o2 == k2 && o3 < k3)));
    if (take) { k1 = o1; k2 = o2; k3 = o3; }
  }
  r.lane = k3 == INT_MAX ? 0 : k3;
  r.B64 = __shfl(prec == UCP_FP64 ? Bf : B64, r.lane);
  return r;
}

template <int PREC>
__global__ __launch_bounds__(kSelWaves * kWave) void k_select(Launch L, int level, int want_l0) {
  const int u = blockIdx.x;
  const int b = find_inst(L.pre, L.n_inst, u);
  const Inst& I = L.insts[b];
  const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int i = (u - L.pre[b]) * kSelWaves + wid;
  if (i >= I.n_x) return;  // whole wave leaves; no block barrier below
  const int K = I.cands;
  const int S = I.segs;
  const double uinc = I.u0[i];
  const double x = I.x_lo + (double)i * I.dx;
  const int kq = level == 0 ? K + 1 : K;

  double c = 0.0, B32 = INFINITY, B64 = NAN;
  if (lane < kq) {
    c = cand_pos(I, level, lane, i);
    B32 = b_from_parts(I, i, lane, K + 1, S, c, PREC);
    if (PREC == UCP_FP64) B64 = B32;
  }
  if (level == 0 && lane == K) I.b32inc[i] = B32;
  if (level > 0 && lane == K) {
    c = I.cbest[i];
    B32 = I.b32best[i];
    B64 = I.b64best[i];
  }
  const bool in_set = level == 0 ? lane < K : lane <= K;
  int n_eval = 0;
  Pick p = select_rule(I, in_set, c, B32, B64, x, uinc, lane, PREC, I.flags, n_eval);
  const double cw = __shfl(c, p.lane);
  const double B32w = __shfl(B32, p.lane);
  double B64w = p.B64;
  if (lane == 0) {
    I.cbest[i] = cw;
    I.b32best[i] = B32w;
    I.b64best[i] = B64w;
  }
  if (level != I.levels - 1) {
    if (lane == 0 && n_eval && I.terms) atomicAdd(I.terms + kCountEvals + (blockIdx.x & (kCountSlots - 1)) * kCountStride, (unsigned long long)n_eval);
    return;
  }

  // acceptance against the incumbent
  double res = cw, Bres = B64w;
  if (!(cw == uinc)) {
    const double B32i = I.b32inc[i];
    const bool in2 = lane < 2;
    const double c2 = lane == 0 ? cw : uinc;
    const double b32_2 = lane == 0 ? B32w : B32i;
    const double b64_2 = lane == 0 ? B64w : (PREC == UCP_FP64 ? B32i : NAN);
    Pick q = select_rule(I, in2, c2, b32_2, b64_2, x, uinc, lane, PREC, I.flags, n_eval);
    res = __shfl(c2, q.lane);
    Bres = q.B64;
  }
  if (want_l0 && isnan(Bres)) Bres = I.k2 * res * res + b64_wave(I, x + res, lane);
  if (lane == 0 && n_eval && I.terms) atomicAdd(I.terms + kCountEvals + (blockIdx.x & (kCountSlots - 1)) * kCountStride, (unsigned long long)n_eval);
  if (lane == 0) {
    I.u0_next[i] = res;
    if (!isfinite(res)) atomicOr(I.flags, 1);
    if (want_l0) I.L0_out[i] = I.f[i] * Bres;
  }
}

hipError_t launch_select(const Launch& L, int level, int prec, int want_l0, hipStream_t st) {
  if (L.total == 0) return hipSuccess;
  dim3 blk(kSelWaves * kWave);
  if (prec == UCP_FP64)
    hipLaunchKernelGGL(k_select<UCP_FP64>, dim3(L.total), blk, 0, st, L, level, want_l0);
  else if (prec == UCP_FP32_KAHAN)
    hipLaunchKernelGGL(k_select<UCP_FP32_KAHAN>, dim3(L.total), blk, 0, st, L, level, want_l0);
  else
    hipLaunchKernelGGL(k_select<UCP_FP32>, dim3(L.total), blk, 0, st, L, level, want_l0);
  return hipGetLastError();
}

// ------------------------------------------------------------ u1 update
//
// u1_j = y_j - v_j with v_j = sum_i w_ij d_ij / sum_i w_ij, d_ij = y_j - x1_i,
// w_ij = exp(l_ij - M), l_ij = log f_i - d_ij^2 / 2 (the conditional mean
// written around y_j so the numerator terms stay small).  Unit = (tile of
// 256 y nodes, slice of x nodes); each slice keeps an online maximum M, and
// the combine kernel merges the slices in a fixed order.

int32_t units_u1_partial(const Inst& I) { return ((I.n_y + kU1Block - 1) / kU1Block) * I.u1_slices; }
int32_t units_u1_combine(const Inst& I) { return (I.n_y + kU1Block - 1) / kU1Block; }

template <int PREC>
__global__ __launch_bounds__(kU1Block) void k_u1_partial(Launch L) {
  __shared__ double sx1[kU1Chunk];   // x1_i
  __shared__ double sL[kU1Chunk];    // log2(e) log f_i
  __shared__ float sx1f[kU1Chunk];   // x1_i in FP32 (maximum pass only)
  __shared__ float slff[kU1Chunk];   // log f_i in FP32 (maximum pass only)
  const int u = blockIdx.x;
  const int b = find_inst(L.pre, L.n_inst, u);
  const Inst& I = L.insts[b];
  const int local = u - L.pre[b];
  const int slice = local % I.u1_slices;
  const int tile = local / I.u1_slices;
  const int j = tile * kU1Block + (int)threadIdx.x;
  const bool act = j < I.n_y;
  const double y = I.y_lo + (double)(act ? j : 0) * I.dy;
  const float yf = (float)y;
  const int slen = (I.n_x + I.u1_slices - 1) / I.u1_slices;
  const int i0 = slice * slen, i1 = min(I.n_x, i0 + slen);
  const double log2e = 1.4426950408889634073599246810019;
  const double c2 = 0.5 * log2e;
  double M = -INFINITY, den = 0.0, num64 = 0.0;
  float num = 0.0f, comp = 0.0f;
  for (int c0 = i0; c0 < i1; c0 += kU1Chunk) {
    const int cn = min(kU1Chunk, i1 - c0);
    __syncthreads();
    for (int t = threadIdx.x; t < cn; t += kU1Block) {
      const int i = c0 + t;
      const double x1 = (I.x_lo + (double)i * I.dx) + I.u0[i];
      const double lf = I.logf[i];
      sx1[t] = x1;
      sL[t] = lf * log2e;
      sx1f[t] = (float)x1;
      slff[t] = (float)lf;
    }
    __syncthreads();
    // chunk maximum of the logits, in FP32: only a shift, any value near
    // the maximum works (the sums below use exact FP64 exponents)
    float mcf = -INFINITY;
    for (int t = 0; t < cn; ++t) {
      const float d = yf - sx1f[t];
      mcf = fmaxf(mcf, fmaf(-0.5f * d, d, slff[t]));
    }
    const double mc = (double)mcf;
    if (mc > M) {  // rescale what was summed under the old maximum
      const double r = M == -INFINITY ? 0.0 : exp(M - mc);
      den *= r;
      if (PREC == UCP_FP64) num64 *= r;
      else { num = (float)((double)num * r); comp = (float)((double)comp * r); }
      M = mc;
    }
    if (!(M > -INFINITY)) continue;  // every logit is -inf (or NaN): nothing to add
    const double Ml = M * log2e;
    for (int t = 0; t < cn; ++t) {
      const double d = y - sx1[t];
      const double a = fma(d, -c2 * d, sL[t] - Ml);  // log2 of the shifted weight
      if (PREC == UCP_FP64) {
        const double w = exp2(a);
        num64 = fma(w, d, num64);
        den += w;
      } else {
        const float w = __builtin_amdgcn_exp2f((float)a);
        const float term = w * (float)d;
        if (PREC == UCP_FP32_KAHAN) {
          const float yy = term - comp;
          const float tt = num + yy;
          comp = (tt - num) - yy;
          num = tt;
        } else {
          num += term;
        }
        den += (double)w;
      }
    }
  }
  if (!act) return;
  double* o = I.u1part + ((size_t)slice * I.n_y + j) * 3;
  o[0] = M;
  o[1] = PREC == UCP_FP64 ? num64 : (double)num - (double)comp;
  o[2] = den;
}

__global__ __launch_bounds__(kU1Block) void k_u1_combine(Launch L) {
  const int u = blockIdx.x;
  const int b = find_inst(L.pre, L.n_inst, u);
  const Inst& I = L.insts[b];
  const int j = (u - L.pre[b]) * kU1Block + (int)threadIdx.x;
  if (j >= I.n_y) return;
  double M = -INFINITY;
  for (int s = 0; s < I.u1_slices; ++s) M = fmax(M, I.u1part[((size_t)s * I.n_y + j) * 3]);
  double num = 0.0, den = 0.0;
  for (int s = 0; s < I.u1_slices; ++s) {
    const double* p = I.u1part + ((size_t)s * I.n_y + j) * 3;
    if (!(p[0] > -INFINITY)) continue;
    const double r = exp(p[0] - M);
    num += p[1] * r;
    den += p[2] * r;
  }
  const double y = I.y_lo + (double)j * I.dy;
  const double vres = num / den;
  const double u1 = y - vres;
  I.u1[j] = u1;
  // the residual from the stored u1, exactly as k_v_from_u1 forms it, so a
  // u0 update sees the same FP32 residual whether u1 came from here or
  // from the caller
  I.v[j] = (float)(sqrt(kAlpha2) * (y - u1));
  if (!isfinite(u1)) atomicOr(I.flags, 1);
}

hipError_t launch_u1_partial(const Launch& L, int prec, hipStream_t st) {
  if (L.total == 0) return hipSuccess;
  if (prec == UCP_FP64)
    hipLaunchKernelGGL(k_u1_partial<UCP_FP64>, dim3(L.total), dim3(kU1Block), 0, st, L);
  else if (prec == UCP_FP32_KAHAN)
    hipLaunchKernelGGL(k_u1_partial<UCP_FP32_KAHAN>, dim3(L.total), dim3(kU1Block), 0, st, L);
  else
    hipLaunchKernelGGL(k_u1_partial<UCP_FP32>, dim3(L.total), dim3(kU1Block), 0, st, L);
  return hipGetLastError();
}

hipError_t launch_u1_combine(const Launch& L, hipStream_t st) {
  if (L.total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_u1_combine, dim3(L.total), dim3(kU1Block), 0, st, L);
  return hipGetLastError();
}

// ------------------------------------------------------------- objective

int32_t units_j_rows(const Inst& I) { return (I.n_x + kJWaves - 1) / kJWaves; }

__global__ __launch_bounds__(kJWaves * kWave) void k_j_rows(Launch L) {
  const int u = blockIdx.x;
  const int b = find_inst(L.pre, L.n_inst, u);
  const Inst& I = L.insts[b];
  const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int i = (u - L.pre[b]) * kJWaves + wid;
  if (i >= I.n_x) return;
  const double u0 = I.u0[i];
  const double x1 = (I.x_lo + (double)i * I.dx) + u0;
  const double inner = b64_wave(I, x1, lane);
  if (lane == 0) I.jrow[i] = I.f[i] * (I.k2 * u0 * u0 + inner);
}

// One block per instance: fixed-order sum of the rows (strided per thread,
// then a tree), times dx.  `t` selects the J_hist entry.
__global__ __launch_bounds__(256) void k_j_reduce(Launch L, int t) {
  __shared__ double red[256];
  const int b = find_inst(L.pre, L.n_inst, blockIdx.x);
  const Inst& I = L.insts[b];
  double s = 0.0;
  for (int i = threadIdx.x; i < I.n_x; i += 256) s += I.jrow[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double J = I.dx * red[0];
    I.J_out[t] = J;
    if (!isfinite(J)) atomicOr(I.flags, 1);
  }
}

hipError_t launch_j_rows(const Launch& L, hipStream_t st) {
  if (L.total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_j_rows, dim3(L.total), dim3(kJWaves * kWave), 0, st, L);
  return hipGetLastError();
}

hipError_t launch_j_reduce_t(const Launch& L, int t, hipStream_t st) {
  if (L.total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_j_reduce, dim3(L.total), dim3(256), 0, st, L, t);
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
  I.v[j] = (float)(sqrt(kAlpha2) * (y - I.u1[j]));
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

}  // namespace ucp
