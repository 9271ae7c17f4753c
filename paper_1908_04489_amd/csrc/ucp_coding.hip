// Zero-delay source-channel coding (Section V-B) on the device, all FP64:
// x0 ~ prior f, x1 = u0(x0) + w with w ~ U(-1, 1), y1 = x1,
// J = E[lam u0(x0)^2 + (u1(y1) - x0)^2].
//
// The uniform noise turns every window sum into a box: the marginal cost of
// a candidate u needs the sums of u1 and u1^2 over the y nodes within 1 of
// u, which double-double prefix sums give in O(1).  So the encoder search
// takes one lane per candidate and one lane group per point, the objective
// one lane per point, and the decoder's closed form (a box-filtered
// conditional mean over the x nodes) is the only quadratic-cost step; its
// tiles of x nodes that lie wholly inside or outside a wave's windows cost
// O(1) each.
//
//   k_cd_prior      f and f x at the x nodes
//   k_cd_extent     per tile of x nodes: min and max of u0, sums of f and f x
//   k_cd_u1_part    decoder sums for 64 y nodes over one segment (tile) of x nodes
//   k_cd_fin_scan   decoder ratio (segment partials added in order) and the
//                   block-local double-double prefix sums of u1 and u1^2
//   k_cd_scan_top   exclusive prefix of the block totals (one block)
//   k_cd_search<G>  per point, G lanes: the coarse-to-fine search of B(u; x_i)
//   k_cd_mc         L_0 = f B for explicit candidates
//   k_cd_jrows / k_cd_jsum   objective rows f_i B(u0_i; x_i), block sums, total
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cmath>
#include <cstring>

#include "ucp.h"
#include "ucp_runtime.h"

namespace ucp {
namespace {

constexpr int kCdTile = 256;    // x nodes per extent tile and per LDS stage
constexpr int kCdSegMax = 128;  // decoder segments (at most; one tile each where possible)
constexpr size_t kCdPartBytes = size_t(1) << 28;  // bound of the decoder's partial sums
constexpr int kCdYGrp = 64;     // y nodes per decoder wave
constexpr int kCdBlk = 64;      // y nodes per block (one wave) of the local prefix sums
constexpr int kCdScan = 1024;   // threads of the top-level prefix block
// A tile whose u0 range lies within these distances of a wave's y range is
// wholly outside (skipped) or wholly inside (its sums added) every window of
// the wave; the margins exceed any rounding of y - u0 for |y|, |u0| <= 1e6,
// and the exact test decides every other tile node by node.
constexpr double kCdOut = 1.0 + 1e-6;
constexpr double kCdIn = 1.0 - 1e-6;

struct CdParams {
  double lam;
  int n_comp;
  int n_x, n_y;
  double w[UCP_MAX_COMP], mu[UCP_MAX_COMP], sd[UCP_MAX_COMP];
  double x_lo, dx;  // x node i = x_lo + i * dx
  double y_lo, dy;  // y node j = y_lo + j * dy
  double inv_dy;
  double u_lo, u_hi;
  int levels, cands;
  double h[UCP_MAX_LEVELS];  // candidate spacing per level
  double tau;                // relative tie band of the selection rule
  int seg_tiles;             // decoder segment length in tiles
  int n_seg;                 // decoder segments
  int n_blk;                 // blocks of the local prefix sums
};

// Prefix sums of u1 and u1^2 in double-double, in two levels: L holds the
// inclusive sums within each block of kCdBlk nodes (four arrays of n_y:
// S1 high, S1 low, S2 high, S2 low), off the exclusive sums of the block
// totals (four arrays of n_blk).
struct Pre {
  const double* L;
  const double* off;
};

// ------------------------------------------------------------ arithmetic

struct dd {
  double h, l;
};
__device__ __forceinline__ dd two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ dd fast_two_sum(double a, double b) {
  const double s = a + b;
  return {s, b - (s - a)};
}
__device__ __forceinline__ dd two_prod(double a, double b) {
  const double p = a * b;
  return {p, fma(a, b, -p)};
}
__device__ __forceinline__ dd dd_add(dd a, dd b) {
  dd s = two_sum(a.h, b.h);
  return fast_two_sum(s.h, s.l + (a.l + b.l));
}
__device__ __forceinline__ dd dd_neg(dd a) { return {-a.h, -a.l}; }
__device__ __forceinline__ dd dd_mul_d(dd a, double d) {
  dd p = two_prod(a.h, d);
  return fast_two_sum(p.h, p.l + a.l * d);
}

__device__ __forceinline__ double xnode(const CdParams& P, int i) { return P.x_lo + (double)i * P.dx; }
__device__ __forceinline__ double ynode(const CdParams& P, int j) { return P.y_lo + (double)j * P.dy; }

// Noise support test of the density p_w(y_j - v): |y_j - v| <= 1.
__device__ __forceinline__ bool in_box(const CdParams& P, int j, double v) {
  return fabs(ynode(P, j) - v) <= 1.0;
}

// The y nodes with |y_j - v| <= 1 form one index interval [a, b] (b < a
// when empty): the rounded difference is monotone in j.  The estimate from
// the grid spacing is corrected by walking with the exact test; the walks
// move monotonically within [-1, n_y], so they end.
__device__ void box_window(const CdParams& P, double v, int& a, int& b) {
  const int n = P.n_y;
  double ta = (v - 1.0 - P.y_lo) * P.inv_dy;
  double tb = (v + 1.0 - P.y_lo) * P.inv_dy;
  ta = fmin(fmax(ta, 0.0), (double)(n - 1));
  tb = fmin(fmax(tb, 0.0), (double)(n - 1));
  int ja = (int)ceil(ta), jb = (int)floor(tb);
  // lower end: step down over window nodes and nodes above v, then up over
  // nodes below the window
  while (ja > 0 && (in_box(P, ja - 1, v) || ynode(P, ja - 1) > v)) --ja;
  while (ja < n && !in_box(P, ja, v) && ynode(P, ja) < v) ++ja;
  // upper end: the mirror image
  while (jb < n - 1 && (in_box(P, jb + 1, v) || ynode(P, jb + 1) < v)) ++jb;
  while (jb >= 0 && !in_box(P, jb, v) && ynode(P, jb) > v) --jb;
  a = ja;
  b = jb;
}

// Sums of u1 and u1^2 over the nodes below j (0 <= j <= n_y).
__device__ __forceinline__ void pre_at(const CdParams& P, const Pre& S, int j, dd& s1, dd& s2) {
  if (j == 0) {
    s1 = s2 = {0.0, 0.0};
    return;
  }
  const int n = P.n_y, nb = P.n_blk, k = j - 1, b = k / kCdBlk;
  s1 = dd_add({S.L[k], S.L[n + k]}, {S.off[b], S.off[nb + b]});
  s2 = dd_add({S.L[2 * n + k], S.L[3 * n + k]}, {S.off[2 * nb + b], S.off[3 * nb + b]});
}

// B(u; x) = lam u^2 + dy * 1/2 * sum over the box window of (u1_j - x)^2,
// the window sum expanded as S2 - 2 x S1 + n x^2 in double-double.
__device__ double cd_B(const CdParams& P, const Pre& S, double x, double u) {
  int a, b;
  box_window(P, u, a, b);
  double s = 0.0;
  if (b >= a) {
    dd hi1, hi2, lo1, lo2;
    pre_at(P, S, b + 1, hi1, hi2);
    pre_at(P, S, a, lo1, lo2);
    const dd s1 = dd_add(hi1, dd_neg(lo1));
    const dd s2 = dd_add(hi2, dd_neg(lo2));
    dd t = dd_add(s2, dd_mul_d(s1, -2.0 * x));
    t = dd_add(t, dd_mul_d(two_prod(x, x), (double)(b - a + 1)));
    s = 0.5 * (t.h + t.l);
  }
  return P.lam * u * u + P.dy * s;
}

// ---------------------------------------------------------------- kernels

__global__ __launch_bounds__(256) void k_cd_prior(CdParams P, double* __restrict__ f, double* __restrict__ fx) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= P.n_x) return;
  const double x = xnode(P, i);
  const double r2pi = sqrt(2.0 * 3.14159265358979323846);
  double sum = 0.0;
  for (int c = 0; c < P.n_comp; ++c) {
    const double d = (x - P.mu[c]) / P.sd[c];
    sum += P.w[c] * exp(-0.5 * d * d) / (P.sd[c] * r2pi);
  }
  f[i] = sum;
  fx[i] = sum * x;
}

__device__ __forceinline__ double wave_sum_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// ext[4 t .. 4 t + 3] = min and max of u0 over tile t (NaN makes the range
// infinite, so the tile goes through the exact test), sum of f, sum of f x
// (fixed order: wave trees, then the waves in order).
__global__ __launch_bounds__(kCdTile) void k_cd_extent(int n_x, const double* __restrict__ u0,
                                                       const double* __restrict__ f,
                                                       const double* __restrict__ fx,
                                                       double* __restrict__ ext) {
  __shared__ double sh[4][kCdTile / 64];
  const int i = blockIdx.x * kCdTile + threadIdx.x;
  double lo = INFINITY, hi = -INFINITY, sf = 0.0, sfx = 0.0;
  if (i < n_x) {
    const double v = u0[i];
    lo = hi = v;
    if (v != v) {
      lo = -INFINITY;
      hi = INFINITY;
    }
    sf = f[i];
    sfx = fx[i];
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o));
    hi = fmax(hi, __shfl_xor(hi, o));
  }
  sf = wave_sum_d(sf);
  sfx = wave_sum_d(sfx);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][wv] = lo;
    sh[1][wv] = hi;
    sh[2][wv] = sf;
    sh[3][wv] = sfx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kCdTile / 64; ++k) {
      lo = fmin(lo, sh[0][k]);
      hi = fmax(hi, sh[1][k]);
      sf += sh[2][k];
      sfx += sh[3][k];
    }
    ext[4 * blockIdx.x] = lo;
    ext[4 * blockIdx.x + 1] = hi;
    ext[4 * blockIdx.x + 2] = sf;
    ext[4 * blockIdx.x + 3] = sfx;
  }
}

// One wave: 64 consecutive y nodes (lane = node) against the x nodes of
// segment blockIdx.y, tile by tile in ascending order.  A tile wholly
// outside every window of the wave is skipped, one wholly inside adds its
// sums, any other is staged in LDS and tested node by node.
// part[(seg * n_y + j) * 2 + {0, 1}] = (sum f x, sum f) over the nodes with
// |y_j - u0_i| <= 1.
__global__ __launch_bounds__(kCdYGrp) void k_cd_u1_part(CdParams P, const double* __restrict__ u0,
                                                        const double* __restrict__ f,
                                                        const double* __restrict__ fx,
                                                        const double* __restrict__ ext,
                                                        double* __restrict__ part) {
  __shared__ double su[kCdTile], sf[kCdTile], sfx[kCdTile];
  const int j0 = blockIdx.x * kCdYGrp;
  const int j = j0 + threadIdx.x;
  const bool live = j < P.n_y;
  const double y = ynode(P, live ? j : P.n_y - 1);
  const double ya = ynode(P, j0), yb = ynode(P, min(P.n_y - 1, j0 + kCdYGrp - 1));
  const int n_tiles = (P.n_x + kCdTile - 1) / kCdTile;
  const int t0 = blockIdx.y * P.seg_tiles, t1 = min(n_tiles, t0 + P.seg_tiles);
  double num = 0.0, den = 0.0;
  for (int t = t0; t < t1; ++t) {
    const double tmin = ext[4 * t], tmax = ext[4 * t + 1];
    if (!(tmin - yb <= kCdOut) || !(ya - tmax <= kCdOut)) continue;  // also skips an empty range
    if (tmax - ya <= kCdIn && yb - tmin <= kCdIn) {
      num += ext[4 * t + 3];
      den += ext[4 * t + 2];
      continue;
    }
    const int i0 = t * kCdTile;
    const int cnt = min(kCdTile, P.n_x - i0);
    for (int k = threadIdx.x; k < cnt; k += kCdYGrp) {
      su[k] = u0[i0 + k];
      sf[k] = f[i0 + k];
      sfx[k] = fx[i0 + k];
    }
    __syncthreads();
    // branch-free: a node outside the window adds an exact zero
#pragma unroll 8
    for (int k = 0; k < cnt; ++k) {
      const bool in = fabs(y - su[k]) <= 1.0;
      num += in ? sfx[k] : 0.0;
      den += in ? sf[k] : 0.0;
    }
    __syncthreads();
  }
  if (live) {
    const long o = ((long)blockIdx.y * P.n_y + j) * 2;
    part[o] = num;
    part[o + 1] = den;
  }
}

// One wave per kCdBlk y nodes.  FROM_PARTS: u1_j = (sum of the segment
// partials of f x) / (sum of those of f), 0 where nothing reaches y_j, and
// u1 is written; otherwise u1 is read.  Then the wave's inclusive
// double-double prefix sums of u1 and u1^2 (Hillis-Steele over lane
// shuffles) go to L and the wave totals to tot (four arrays of n_blk).
template <bool FROM_PARTS>
__global__ __launch_bounds__(kCdBlk) void k_cd_fin_scan(CdParams P, const double* __restrict__ part, double* u1,
                                                        double* __restrict__ L, double* __restrict__ tot) {
  const int t = threadIdx.x;
  const int j = blockIdx.x * kCdBlk + t;
  const int n = P.n_y;
  double v = 0.0;
  if (j < n) {
    if (FROM_PARTS) {
      double num = 0.0, den = 0.0;
      for (int s = 0; s < P.n_seg; ++s) {
        const long o = ((long)s * n + j) * 2;
        num += part[o];
        den += part[o + 1];
      }
      v = den > 0.0 ? num / den : 0.0;
      u1[j] = v;
    } else {
      v = u1[j];
    }
  }
  dd a1 = {v, 0.0}, a2 = two_prod(v, v);
  for (int o = 1; o < kCdBlk; o <<= 1) {
    const dd b1 = {__shfl_up(a1.h, o), __shfl_up(a1.l, o)};
    const dd b2 = {__shfl_up(a2.h, o), __shfl_up(a2.l, o)};
    if (t >= o) {
      a1 = dd_add(b1, a1);
      a2 = dd_add(b2, a2);
    }
  }
  if (j < n) {
    L[j] = a1.h;
    L[n + j] = a1.l;
    L[2 * n + j] = a2.h;
    L[3 * n + j] = a2.l;
  }
  if (t == kCdBlk - 1) {
    const int nb = P.n_blk, b = blockIdx.x;
    tot[b] = a1.h;
    tot[nb + b] = a1.l;
    tot[2 * nb + b] = a2.h;
    tot[3 * nb + b] = a2.l;
  }
}

// One block: exclusive prefix of the n_blk block totals.  Thread t adds a
// contiguous chunk, the chunk sums are scanned in LDS, then each thread
// writes its chunk's running sums.
__global__ __launch_bounds__(kCdScan) void k_cd_scan_top(int nb, const double* __restrict__ tot,
                                                         double* __restrict__ off) {
  __shared__ double sh[4][kCdScan];
  const int t = threadIdx.x;
  const int chunk = (nb + kCdScan - 1) / kCdScan;
  const int lo = min(nb, t * chunk), hi = min(nb, lo + chunk);
  dd a1 = {0.0, 0.0}, a2 = {0.0, 0.0};
  for (int b = lo; b < hi; ++b) {
    a1 = dd_add(a1, {tot[b], tot[nb + b]});
    a2 = dd_add(a2, {tot[2 * nb + b], tot[3 * nb + b]});
  }
  sh[0][t] = a1.h;
  sh[1][t] = a1.l;
  sh[2][t] = a2.h;
  sh[3][t] = a2.l;
  __syncthreads();
  for (int o = 1; o < kCdScan; o <<= 1) {
    const bool take = t >= o;
    dd b1 = {0.0, 0.0}, b2 = {0.0, 0.0};
    if (take) {
      b1 = {sh[0][t - o], sh[1][t - o]};
      b2 = {sh[2][t - o], sh[3][t - o]};
    }
    __syncthreads();
    if (take) {
      a1 = dd_add(b1, a1);
      a2 = dd_add(b2, a2);
      sh[0][t] = a1.h;
      sh[1][t] = a1.l;
      sh[2][t] = a2.h;
      sh[3][t] = a2.l;
    }
    __syncthreads();
  }
  dd r1 = {0.0, 0.0}, r2 = {0.0, 0.0};
  if (t > 0) {
    r1 = {sh[0][t - 1], sh[1][t - 1]};
    r2 = {sh[2][t - 1], sh[3][t - 1]};
  }
  for (int b = lo; b < hi; ++b) {
    off[b] = r1.h;
    off[nb + b] = r1.l;
    off[2 * nb + b] = r2.h;
    off[3 * nb + b] = r2.l;
    r1 = dd_add(r1, {tot[b], tot[nb + b]});
    r2 = dd_add(r2, {tot[2 * nb + b], tot[3 * nb + b]});
  }
}

__device__ __forceinline__ double level_cand(const CdParams& P, int l, int q, double cs) {
  if (l == 0) return P.u_lo + (double)q * P.h[0];
  double v = cs - P.h[l - 1] + (double)q * P.h[l];
  if (v < P.u_lo) v = P.u_lo;
  if (v > P.u_hi) v = P.u_hi;
  return v;
}

// The selection rule as a reduction over a group of G lanes: among the
// candidates with B within the relative band tau of the minimum, the
// smallest (distance to the incumbent, u, index) wins - the nearest, then
// the smaller u, then the earlier candidate.  Lanes out of the band carry
// infinite keys.  Every lane of the group ends with the winner.
template <int G>
__device__ __forceinline__ void group_pick(double& d, double& c, int& q, double& B) {
  for (int o = G / 2; o > 0; o >>= 1) {
    const double od = __shfl_xor(d, o, G), oc = __shfl_xor(c, o, G), oB = __shfl_xor(B, o, G);
    const int oq = __shfl_xor(q, o, G);
    if (od < d || (od == d && (oc < c || (oc == c && oq < q)))) {
      d = od;
      c = oc;
      q = oq;
      B = oB;
    }
  }
}
template <int G>
__device__ __forceinline__ double group_min(double v) {
  for (int o = G / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, G));
  return v;
}

// G lanes per point, lane q = candidate q of the level; the best so far
// (index K) and the incumbent's final comparison are handled by every lane
// alike.  u0_in and u0_out may alias: a group reads its entry before lane 0
// writes it.
template <int G>
__global__ __launch_bounds__(256) void k_cd_search(CdParams P, Pre S, const double* __restrict__ f,
                                                   const double* u0_in, double* u0_out, double* L0_out) {
  const int i = (blockIdx.x * 256 + threadIdx.x) / G;
  const int q = threadIdx.x % G;
  if (i >= P.n_x) return;  // whole groups
  const double x = xnode(P, i);
  const double uinc = u0_in[i];
  const int K = P.cands;
  double cs = 0.0, Bs = 0.0;
  for (int l = 0; l < P.levels; ++l) {
    const bool live = q < K;
    const double c = live ? level_cand(P, l, q, cs) : 0.0;
    const double B = live ? cd_B(P, S, x, c) : INFINITY;
    double m = group_min<G>(B);
    if (l > 0 && Bs < m) m = Bs;
    const double thr = m * (1.0 + P.tau);
    double kd = INFINITY, kc = INFINITY, kB = B;
    int kq = 1 << 30;
    if (live && B <= thr) {
      kd = fabs(c - uinc);
      kc = c;
      kq = q;
    }
    group_pick<G>(kd, kc, kq, kB);
    if (l > 0 && Bs <= thr) {  // the best so far, index K, after every lane
      const double ds = fabs(cs - uinc);
      if (kq == (1 << 30) || ds < kd || (ds == kd && cs < kc)) {
        kc = cs;
        kB = Bs;
      }
    }
    cs = kc;
    Bs = kB;
  }
  // acceptance against the incumbent (index 1, after the search's winner)
  const double Binc = cd_B(P, S, x, uinc);
  double m = Bs;
  if (Binc < m) m = Binc;
  const double thr = m * (1.0 + P.tau);
  double rc = cs, rB = Bs;
  const bool win_in = Bs <= thr;
  if (Binc <= thr) {
    const double ds = fabs(cs - uinc), di = fabs(uinc - uinc);
    if (!win_in || di < ds || (di == ds && uinc < cs)) {
      rc = uinc;
      rB = Binc;
    }
  }
  if (q == 0) {
    u0_out[i] = rc;
    if (L0_out) L0_out[i] = f[i] * rB;
  }
}

__global__ __launch_bounds__(256) void k_cd_mc(CdParams P, Pre S, const double* __restrict__ f,
                                               const double* __restrict__ u, int n_cand, double* __restrict__ out) {
  const long g = (long)blockIdx.x * 256 + threadIdx.x;
  if (g >= (long)P.n_x * n_cand) return;
  const int i = (int)(g / n_cand);
  out[g] = f[i] * cd_B(P, S, xnode(P, i), u[g]);
}

// Objective rows f_i B(u0_i; x_i), one lane per x node, summed per block in a
// fixed tree into jpart[block].
__global__ __launch_bounds__(256) void k_cd_jrows(CdParams P, Pre S, const double* __restrict__ u0,
                                                  const double* __restrict__ f, double* __restrict__ jpart) {
  __shared__ double sh[256];
  const int i = blockIdx.x * 256 + threadIdx.x;
  double r = 0.0;
  if (i < P.n_x) r = f[i] * cd_B(P, S, xnode(P, i), u0[i]);
  sh[threadIdx.x] = r;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) jpart[blockIdx.x] = sh[0];
}

// J = dx * sum of the block sums, in a fixed order (strided partials, then a tree).
__global__ __launch_bounds__(256) void k_cd_jsum(int n, double dx, const double* __restrict__ jpart,
                                                 double* __restrict__ J) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += jpart[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *J = dx * sh[0];
}

// ------------------------------------------------------------------- host

inline size_t al(size_t v) { return (v + 255) & ~(size_t)255; }

struct CdWork {
  double *f, *fx, *L, *tot, *off, *ext, *part, *jpart;
  Pre pre() const { return {L, off}; }
};

int cd_params(const ucp_coding_problem* p, const ucp_search* s, CdParams& P) {
  if (!p) return fail(UCP_EINVAL, "problem is NULL");
  if (!(p->lam >= 0.0) || !std::isfinite(p->lam)) return fail(UCP_EINVAL, "lam must be finite and >= 0");
  ucp_problem q;
  std::memset(&q, 0, sizeof q);
  q.k = 0.0;
  q.n_comp = p->n_comp;
  std::memcpy(q.w, p->w, sizeof q.w);
  std::memcpy(q.mu, p->mu, sizeof q.mu);
  std::memcpy(q.sd, p->sd, sizeof q.sd);
  q.x_lo = p->x_lo;
  q.x_hi = p->x_hi;
  q.n_x = p->n_x;
  q.y_lo = p->y_lo;
  q.y_hi = p->y_hi;
  q.n_y = p->n_y;
  int rc = check_problem(&q);
  if (rc) return rc;
  if (s && (rc = check_search(s))) return rc;
  std::memset(&P, 0, sizeof P);
  P.lam = p->lam;
  P.n_comp = p->n_comp;
  P.n_x = (int)p->n_x;
  P.n_y = (int)p->n_y;
  for (int c = 0; c < p->n_comp; ++c) {
    P.w[c] = p->w[c];
    P.mu[c] = p->mu[c];
    P.sd[c] = p->sd[c];
  }
  P.x_lo = p->x_lo;
  P.dx = (p->x_hi - p->x_lo) / (double)(p->n_x - 1);
  P.y_lo = p->y_lo;
  P.dy = (p->y_hi - p->y_lo) / (double)(p->n_y - 1);
  P.inv_dy = 1.0 / P.dy;
  P.tau = tie_band(s);
  if (s) {
    P.u_lo = s->u_lo;
    P.u_hi = s->u_hi;
    P.levels = s->levels;
    P.cands = s->cands;
    P.h[0] = (s->u_hi - s->u_lo) / (double)(s->cands - 1);
    for (int l = 1; l < s->levels; ++l) P.h[l] = 2.0 * P.h[l - 1] / (double)(s->cands - 1);
  }
  // decoder segments: as many as tiles (a wave's run of exact tests is then
  // one tile long), at most kCdSegMax and within kCdPartBytes of partials
  const int n_tiles = (P.n_x + kCdTile - 1) / kCdTile;
  size_t cap = kCdPartBytes / (16 * (size_t)P.n_y);
  if (cap < 1) cap = 1;
  int n_seg = n_tiles;
  if (n_seg > kCdSegMax) n_seg = kCdSegMax;
  if ((size_t)n_seg > cap) n_seg = (int)cap;
  P.seg_tiles = (n_tiles + n_seg - 1) / n_seg;
  P.n_seg = (n_tiles + P.seg_tiles - 1) / P.seg_tiles;
  P.n_blk = (P.n_y + kCdBlk - 1) / kCdBlk;
  return UCP_OK;
}

int cd_work(ucp_handle* h, const CdParams& P, CdWork& W) {
  const size_t nx = (size_t)P.n_x, ny = (size_t)P.n_y, nb = (size_t)P.n_blk;
  const size_t n_tiles = (nx + kCdTile - 1) / kCdTile;
  const size_t sz[8] = {al(8 * nx), al(8 * nx), al(8 * 4 * ny), al(8 * 4 * nb), al(8 * 4 * nb),
                        al(8 * 4 * n_tiles), al(8 * 2 * (size_t)P.n_seg * ny), al(8 * ((nx + 255) / 256))};
  size_t total = 0;
  for (size_t v : sz) total += v;
  void* base = nullptr;
  int rc = handle_workspace(h, total, &base);
  if (rc) return rc;
  char* p = (char*)base;
  double** slot[8] = {&W.f, &W.fx, &W.L, &W.tot, &W.off, &W.ext, &W.part, &W.jpart};
  for (int k = 0; k < 8; ++k) {
    *slot[k] = (double*)p;
    p += sz[k];
  }
  return UCP_OK;
}

#define CD_TRY(expr, what)                           \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

inline unsigned blocks(long n, int per) { return (unsigned)((n + per - 1) / per); }

hipError_t cd_prior(const CdParams& P, const CdWork& W, hipStream_t st) {
  hipLaunchKernelGGL(k_cd_prior, dim3(blocks(P.n_x, 256)), dim3(256), 0, st, P, W.f, W.fx);
  return hipGetLastError();
}

// Prefix sums of a given u1 (an input array).
hipError_t cd_scan_input(ucp_handle* h, const CdParams& P, const CdWork& W, const double* u1, hipStream_t st) {
  hipEvent_t a, b;
  hipError_t e = handle_events(h, UCP_PROF_SELECT, &a, &b);
  if (e != hipSuccess) return e;
  hipExtLaunchKernelGGL(k_cd_fin_scan<false>, dim3(P.n_blk), dim3(kCdBlk), 0, st, a, nullptr, 0, P,
                        (const double*)nullptr, const_cast<double*>(u1), W.L, W.tot);
  hipExtLaunchKernelGGL(k_cd_scan_top, dim3(1), dim3(kCdScan), 0, st, nullptr, b, 0, P.n_blk,
                        (const double*)W.tot, W.off);
  return hipGetLastError();
}

// Decoder of u0 into u1, and the prefix sums of the new u1.
hipError_t cd_u1(ucp_handle* h, const CdParams& P, const CdWork& W, const double* u0, double* u1,
                 hipStream_t st) {
  hipEvent_t a, b;
  hipError_t e = handle_events(h, UCP_PROF_U1, &a, &b);
  if (e != hipSuccess) return e;
  const unsigned n_tiles = blocks(P.n_x, kCdTile);
  hipExtLaunchKernelGGL(k_cd_extent, dim3(n_tiles), dim3(kCdTile), 0, st, a, nullptr, 0, P.n_x, u0,
                        (const double*)W.f, (const double*)W.fx, W.ext);
  hipLaunchKernelGGL(k_cd_u1_part, dim3(blocks(P.n_y, kCdYGrp), P.n_seg), dim3(kCdYGrp), 0, st, P, u0,
                     (const double*)W.f, (const double*)W.fx, (const double*)W.ext, W.part);
  hipExtLaunchKernelGGL(k_cd_fin_scan<true>, dim3(P.n_blk), dim3(kCdBlk), 0, st, nullptr, b, 0, P,
                        (const double*)W.part, u1, W.L, W.tot);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipEvent_t a2, b2;
  e = handle_events(h, UCP_PROF_SELECT, &a2, &b2);
  if (e != hipSuccess) return e;
  hipExtLaunchKernelGGL(k_cd_scan_top, dim3(1), dim3(kCdScan), 0, st, a2, b2, 0, P.n_blk, (const double*)W.tot,
                        W.off);
  return hipGetLastError();
}

template <int G>
void launch_search(const CdParams& P, const CdWork& W, const double* u0_in, double* u0_out, double* L0_out,
                   hipEvent_t a, hipEvent_t b, hipStream_t st) {
  hipExtLaunchKernelGGL(k_cd_search<G>, dim3(blocks((long)P.n_x * G, 256)), dim3(256), 0, st, a, b, 0, P,
                        W.pre(), (const double*)W.f, u0_in, u0_out, L0_out);
}

hipError_t cd_search(ucp_handle* h, const CdParams& P, const CdWork& W, const double* u0_in, double* u0_out,
                     double* L0_out, hipStream_t st) {
  hipEvent_t a, b;
  hipError_t e = handle_events(h, UCP_PROF_MC, &a, &b);
  if (e != hipSuccess) return e;
  if (P.cands <= 2) launch_search<2>(P, W, u0_in, u0_out, L0_out, a, b, st);
  else if (P.cands <= 4) launch_search<4>(P, W, u0_in, u0_out, L0_out, a, b, st);
  else if (P.cands <= 8) launch_search<8>(P, W, u0_in, u0_out, L0_out, a, b, st);
  else if (P.cands <= 16) launch_search<16>(P, W, u0_in, u0_out, L0_out, a, b, st);
  else if (P.cands <= 32) launch_search<32>(P, W, u0_in, u0_out, L0_out, a, b, st);
  else launch_search<64>(P, W, u0_in, u0_out, L0_out, a, b, st);
  return hipGetLastError();
}

hipError_t cd_objective(ucp_handle* h, const CdParams& P, const CdWork& W, const double* u0, double* J,
                        hipStream_t st) {
  hipEvent_t a, b;
  hipError_t e = handle_events(h, UCP_PROF_J, &a, &b);
  if (e != hipSuccess) return e;
  const unsigned nb = blocks(P.n_x, 256);
  hipExtLaunchKernelGGL(k_cd_jrows, dim3(nb), dim3(256), 0, st, a, nullptr, 0, P, W.pre(), u0, (const double*)W.f,
                        W.jpart);
  hipExtLaunchKernelGGL(k_cd_jsum, dim3(1), dim3(256), 0, st, nullptr, b, 0, (int)nb, P.dx,
                        (const double*)W.jpart, J);
  return hipGetLastError();
}

// After the argument checks: the handle's device made current.
int cd_begin(ucp_handle* h) {
  hipError_t e = hipSetDevice(handle_device(h));
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  return UCP_OK;
}

}  // namespace
}  // namespace ucp

using namespace ucp;

extern "C" {

int ucp_coding_marginal_cost(ucp_handle* h, const ucp_coding_problem* prob, const double* u1, const double* u,
                             int64_t n_cand, double* L0_out, void* stream) {
  int rc;
  CdParams P;
  if (!h) return fail(UCP_EINVAL, "handle is NULL");
  if ((rc = cd_params(prob, nullptr, P))) return rc;
  if (!u1 || !u || !L0_out) return fail(UCP_EINVAL, "NULL array argument");
  if (n_cand < 1 || n_cand > 4096) return fail(UCP_EINVAL, "n_cand must be 1..4096");
  if ((int64_t)P.n_x * n_cand > ((int64_t)1 << 30)) return fail(UCP_EINVAL, "n_x * n_cand too large");
  if ((rc = cd_begin(h))) return rc;
  CdWork W;
  if ((rc = cd_work(h, P, W))) return rc;
  hipStream_t st = (hipStream_t)stream;
  CD_TRY(cd_prior(P, W, st), "prior kernel");
  CD_TRY(cd_scan_input(nullptr, P, W, u1, st), "prefix-sum kernels");
  hipLaunchKernelGGL(k_cd_mc, dim3(blocks((long)P.n_x * n_cand, 256)), dim3(256), 0, st, P, W.pre(),
                     (const double*)W.f, u, (int)n_cand, L0_out);
  CD_TRY(hipGetLastError(), "marginal-cost kernel");
  return UCP_OK;
}

int ucp_coding_argmin(ucp_handle* h, const ucp_coding_problem* prob, const ucp_search* search, const double* u1,
                      const double* u0_in, double* u0_out, double* L0_out, void* stream) {
  int rc;
  CdParams P;
  if (!h) return fail(UCP_EINVAL, "handle is NULL");
  if (!search) return fail(UCP_EINVAL, "search is NULL");
  if ((rc = cd_params(prob, search, P))) return rc;
  if (!u1 || !u0_in || !u0_out) return fail(UCP_EINVAL, "NULL array argument");
  if ((rc = cd_begin(h))) return rc;
  CdWork W;
  if ((rc = cd_work(h, P, W))) return rc;
  hipStream_t st = (hipStream_t)stream;
  CD_TRY(cd_prior(P, W, st), "prior kernel");
  CD_TRY(cd_scan_input(nullptr, P, W, u1, st), "prefix-sum kernels");
  CD_TRY(cd_search(nullptr, P, W, u0_in, u0_out, L0_out, st), "search kernel");
  return UCP_OK;
}

int ucp_coding_update_u1(ucp_handle* h, const ucp_coding_problem* prob, const double* u0, double* u1_out,
                         void* stream) {
  int rc;
  CdParams P;
  if (!h) return fail(UCP_EINVAL, "handle is NULL");
  if ((rc = cd_params(prob, nullptr, P))) return rc;
  if (!u0 || !u1_out) return fail(UCP_EINVAL, "NULL array argument");
  if ((rc = cd_begin(h))) return rc;
  CdWork W;
  if ((rc = cd_work(h, P, W))) return rc;
  hipStream_t st = (hipStream_t)stream;
  CD_TRY(cd_prior(P, W, st), "prior kernel");
  CD_TRY(cd_u1(nullptr, P, W, u0, u1_out, st), "decoder kernels");
  return UCP_OK;
}

int ucp_coding_objective(ucp_handle* h, const ucp_coding_problem* prob, const double* u0, const double* u1,
                         double* J_out, void* stream) {
  int rc;
  CdParams P;
  if (!h) return fail(UCP_EINVAL, "handle is NULL");
  if ((rc = cd_params(prob, nullptr, P))) return rc;
  if (!u0 || !u1 || !J_out) return fail(UCP_EINVAL, "NULL array argument");
  if ((rc = cd_begin(h))) return rc;
  CdWork W;
  if ((rc = cd_work(h, P, W))) return rc;
  hipStream_t st = (hipStream_t)stream;
  CD_TRY(cd_prior(P, W, st), "prior kernel");
  CD_TRY(cd_scan_input(nullptr, P, W, u1, st), "prefix-sum kernels");
  CD_TRY(cd_objective(nullptr, P, W, u0, J_out, st), "objective kernels");
  return UCP_OK;
}

int ucp_coding_solve(ucp_handle* h, const ucp_coding_problem* prob, const ucp_search* search, int32_t iters,
                     const double* u0_init, double* u0_out, double* u1_out, double* J_hist, void* stream) {
  int rc;
  CdParams P;
  if (!h) return fail(UCP_EINVAL, "handle is NULL");
  if (!search) return fail(UCP_EINVAL, "search is NULL");
  if ((rc = cd_params(prob, search, P))) return rc;
  if (!u0_init || !u0_out || !u1_out || !J_hist) return fail(UCP_EINVAL, "NULL array argument");
  if (iters < 0) return fail(UCP_EINVAL, "iters must be >= 0");
  if ((rc = cd_begin(h))) return rc;
  CdWork W;
  if ((rc = cd_work(h, P, W))) return rc;
  hipStream_t st = (hipStream_t)stream;
  CD_TRY(cd_prior(P, W, st), "prior kernel");
  if (u0_out != u0_init)
    CD_TRY(hipMemcpyAsync(u0_out, u0_init, sizeof(double) * P.n_x, hipMemcpyDeviceToDevice, st), "copy u0");
  // every round ends with the prefix sums of its u1, which the objective
  // and the next round's search read
  CD_TRY(cd_u1(h, P, W, u0_out, u1_out, st), "decoder kernels");
  CD_TRY(cd_objective(h, P, W, u0_out, J_hist, st), "objective kernels");
  for (int t = 1; t <= iters; ++t) {
    CD_TRY(cd_search(h, P, W, u0_out, u0_out, nullptr, st), "search kernel");
    CD_TRY(cd_u1(h, P, W, u0_out, u1_out, st), "decoder kernels");
    CD_TRY(cd_objective(h, P, W, u0_out, J_hist + t, st), "objective kernels");
  }
  if (handle_profiling(h)) {
    CD_TRY(hipStreamSynchronize(st), "synchronise");
    handle_harvest(h);
  }
  return UCP_OK;
}

}  // extern "C"
