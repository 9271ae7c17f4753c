// Two-dimensional Witsenhausen counterexample (Section V-D) on the device,
// FP64: x0 in R^2 with independent coordinates from the prior, x1 = x0 + u0,
// y1 = x1 + w with w ~ N(0, I_2), x2 = x1 - u1(y1),
// J = 1/2 E[k^2 |u0|^2 + |x2|^2], on tensor-product grids (node (i1, i2) at
// i1 * n + i2; vector fields as two planes).
//
//   k_w2_prior    1-D prior f at the x nodes (the 2-D prior is f(x1) f(x2))
//   k_w2_search   one wave per point: every level of the coarse-to-fine
//                 search (the wave sums the candidates of one grid column
//                 kW2Grp at a time over their shared column window, lanes
//                 along the columns; lane q keeps candidate q) and the
//                 incumbent comparison, the selection rule as a wave
//                 reduction
//   k_w2_mc       L_0 = f B for explicit candidates, one lane each
//   k_w2_u1_part  u1 sums for 64 y nodes over one segment of x nodes,
//                 max-shifted within the segment
//   k_w2_u1_fin   segments merged (shift to the common maximum), the ratio
//   k_w2_jrows / k_w2_jsum   objective rows f B(u0), block sums, total
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cmath>
#include <cstring>

#include "ucp.h"
#include "ucp_runtime.h"

namespace ucp {
namespace {

constexpr double kW2Win = 10.0;  // noise sds (window half-width floor(kW2Win / dy) nodes)
constexpr int kW2Seg = 16;       // x segments of the u1 sums (at most)
constexpr int kW2Tile = 256;     // x nodes staged in LDS per step of the u1 sums
constexpr int kW2Grp = 4;        // candidates of a grid column summed together by the search

struct W2Params {
  double k;
  int n_comp;
  int n, ny;  // nodes per coordinate of the x and y grids
  double w[UCP_MAX_COMP], mu[UCP_MAX_COMP], sd[UCP_MAX_COMP];
  double x_lo, dx, y_lo, dy, inv_dy;
  double Q;  // exp(-dy^2): step of the Gaussian recurrence along a row
  int wn;    // window half-width in y nodes
  double u_lo, u_hi;
  int levels, cands;
  double h[UCP_MAX_LEVELS];
  double tau;          // relative tie band of the selection rule
  int seg_len, n_seg;  // u1 sums: x nodes per segment, segments
};

__device__ __forceinline__ double xnode(const W2Params& P, int i) { return P.x_lo + (double)i * P.dx; }
__device__ __forceinline__ double ynode(const W2Params& P, int j) { return P.y_lo + (double)j * P.dy; }

__device__ __forceinline__ double phi(double t) {
  return exp(-0.5 * t * t) / sqrt(2.0 * 3.14159265358979323846);
}

// Nodes within wn of the node nearest z (clamped to the grid).
__device__ __forceinline__ void w2_window(const W2Params& P, double z, int& a, int& b) {
  double c = rint((z - P.y_lo) * P.inv_dy);
  c = fmin(fmax(c, 0.0), (double)(P.ny - 1));
  const int ci = (int)c;
  a = max(0, ci - P.wn);
  b = min(P.ny - 1, ci + P.wn);
}

// B(u; x) = 1/2 [k^2 |u|^2 + dy^2 sum phi(y1 - z1) phi(y2 - z2) |z - u1(y)|^2]
// over the window; along a row the second factor follows the exact
// recurrence phi(t + dy) = phi(t) exp(-t dy - dy^2 / 2), restarted per row.
__device__ double w2_B(const W2Params& P, const double* __restrict__ u1a, const double* __restrict__ u1b,
                       double x1, double x2, double ua, double ub) {
  const double z1 = x1 + ua, z2 = x2 + ub;
  int a1, b1, a2, b2;
  w2_window(P, z1, a1, b1);
  w2_window(P, z2, a2, b2);
  const double t0 = ynode(P, a2) - z2;
  const double r0 = phi(t0);
  const double q0 = exp(-t0 * P.dy - 0.5 * P.dy * P.dy);
  double s = 0.0;
  for (int j1 = a1; j1 <= b1; ++j1) {
    const double g1 = phi(ynode(P, j1) - z1);
    const double* ra = u1a + (long)j1 * P.ny;
    const double* rb = u1b + (long)j1 * P.ny;
    double r = r0, q = q0, row = 0.0;
    for (int j2 = a2; j2 <= b2; ++j2) {
      const double e1 = z1 - ra[j2];
      const double e2 = z2 - rb[j2];
      row = fma(r, e1 * e1 + e2 * e2, row);
      r *= q;
      q *= P.Q;
    }
    s = fma(g1, row, s);
  }
  return 0.5 * (P.k * P.k * (ua * ua + ub * ub) + P.dy * P.dy * s);
}

__global__ __launch_bounds__(256) void k_w2_prior(W2Params P, double* __restrict__ f) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= P.n) return;
  const double x = xnode(P, i);
  const double r2pi = sqrt(2.0 * 3.14159265358979323846);
  double sum = 0.0;
  for (int c = 0; c < P.n_comp; ++c) {
    const double d = (x - P.mu[c]) / P.sd[c];
    sum += P.w[c] * exp(-0.5 * d * d) / (P.sd[c] * r2pi);
  }
  f[i] = sum;
}

__device__ __forceinline__ double cand(const W2Params& P, int l, int qi, double s) {
  if (l == 0) return P.u_lo + (double)qi * P.h[0];
  double v = s - P.h[l - 1] + (double)qi * P.h[l];
  if (v < P.u_lo) v = P.u_lo;
  if (v > P.u_hi) v = P.u_hi;
  return v;
}

// Wave-wide selection key: smallest (squared distance to the incumbent,
// first coordinate, second coordinate, index); lanes out of the band carry
// infinite keys.  Every lane ends with the winner.
__device__ __forceinline__ void wave_pick(double& d, double& ca, double& cb, int& q, double& B) {
  for (int o = 32; o > 0; o >>= 1) {
    const double od = __shfl_xor(d, o), oa = __shfl_xor(ca, o), ob = __shfl_xor(cb, o), oB = __shfl_xor(B, o);
    const int oq = __shfl_xor(q, o);
    if (od < d || (od == d && (oa < ca || (oa == ca && (ob < cb || (ob == cb && oq < q)))))) {
      d = od;
      ca = oa;
      cb = ob;
      q = oq;
      B = oB;
    }
  }
}

// The rule's comparison of a later candidate (s) against the current winner
// (w): the later one wins on a smaller key only.
__device__ __forceinline__ bool later_wins(double ds, double sa, double sb, double dw, double wa, double wb) {
  return ds < dw || (ds == dw && (sa < wa || (sa == wa && sb < wb)));
}

// B of the nc <= NC candidates (x1 + c1[q], x2 + c2) that share their
// second coordinate, summed together by a whole wave: they share the
// column window and its factors phi(y_c - z2), so each row segment of u1
// is loaded once for all of them.  Lane t takes columns chunk + t; the rows
// run over the union of the candidates' row windows, a row outside a
// candidate's window weighing zero for it; the row factors of a chunk of
// 64 rows sit in LDS (tab, NC x 64).  Every lane returns the nc values in Bq.
template <int NC>
__device__ void w2_B_column(const W2Params& P, const double* __restrict__ u1a, const double* __restrict__ u1b,
                            double x1, double x2, const double* c1, double c2, int nc, double* Bq,
                            double* tab) {
  const int t = threadIdx.x & 63;
  double z1[NC];
  int ra[NC], rb[NC];
  int ua = P.ny, ub = -1;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    z1[q] = x1 + c1[q];
    ra[q] = 1;
    rb[q] = 0;
    if (q < nc) {
      w2_window(P, z1[q], ra[q], rb[q]);
      ua = min(ua, ra[q]);
      ub = max(ub, rb[q]);
    }
  }
  const double z2 = x2 + c2;
  int a2, b2;
  w2_window(P, z2, a2, b2);
  double acc[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) acc[q] = 0.0;
  for (int cc = a2; cc <= b2; cc += 64) {
    const int c = cc + t;
    const bool have = c <= b2;
    const double g2 = have ? phi(ynode(P, c) - z2) : 0.0;
    const int cl = have ? c : a2;
    for (int r0 = ua; r0 <= ub; r0 += 64) {
      const int nr = min(64, ub - r0 + 1);
      const int row = r0 + t;
#pragma unroll
      for (int q = 0; q < NC; ++q)
        tab[q * 64 + t] = (t < nr && row >= ra[q] && row <= rb[q]) ? phi(ynode(P, row) - z1[q]) : 0.0;
      __syncthreads();
      for (int k = 0; k < nr; ++k) {
        const long o = (long)(r0 + k) * P.ny + cl;
        const double a = u1a[o];
        const double e2 = z2 - u1b[o];
        const double e22 = e2 * e2;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
          if (q < nc) {
            const double e1 = z1[q] - a;
            acc[q] = fma(tab[q * 64 + k] * g2, fma(e1, e1, e22), acc[q]);
          }
        }
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    double v = acc[q];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    Bq[q] = 0.5 * (P.k * P.k * (c1[q] * c1[q] + c2 * c2) + P.dy * P.dy * v);
  }
}

// One wave per point.  u0_in and u0_out (two planes each) may alias: the
// wave reads its point before lane 0 writes it.  The wave sums the
// candidates column by column of the K x K grid, kW2Grp at a time
// (w2_B_column: fewer at once keeps the registers at three waves per SIMD),
// and lane q keeps candidate q's B.
__global__ __launch_bounds__(64) void k_w2_search(W2Params P, const double* __restrict__ f,
                                                  const double* __restrict__ u1, const double* u0_in,
                                                  double* u0_out, double* L0_out) {
  const int i = blockIdx.x;
  const int q = threadIdx.x;
  const int nn = P.n * P.n, K = P.cands, KK = K * K;
  const double x1 = xnode(P, i / P.n), x2 = xnode(P, i % P.n);
  const double ia = u0_in[i], ib = u0_in[nn + i];
  const double* u1a = u1;
  const double* u1b = u1 + (long)P.ny * P.ny;
  __shared__ double tab[kW2Grp * 64];
  double sa = 0.0, sb = 0.0, sB = 0.0;
  for (int l = 0; l < P.levels; ++l) {
    const bool live = q < KK;
    const double ca = live ? cand(P, l, q / K, sa) : 0.0;
    const double cb = live ? cand(P, l, q % K, sb) : 0.0;
    double c1[8], Bq[kW2Grp];
#pragma unroll
    for (int r = 0; r < 8; ++r) c1[r] = r < K ? cand(P, l, r, sa) : 0.0;
    double B = INFINITY;
    for (int q2 = 0; q2 < K; ++q2) {
      const double c2 = cand(P, l, q2, sb);
      for (int h = 0; h < K; h += kW2Grp) {  // the column's candidates kW2Grp at a time
        w2_B_column<kW2Grp>(P, u1a, u1b, x1, x2, c1 + h, c2, min(kW2Grp, K - h), Bq, tab);
#pragma unroll
        for (int r = 0; r < kW2Grp; ++r)
          if (h + r < K && q == (h + r) * K + q2) B = Bq[r];
      }
    }
    double m = B;
    for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o));
    if (l > 0 && sB < m) m = sB;
    const double thr = m * (1.0 + P.tau);
    double kd = INFINITY, ka = INFINITY, kb = INFINITY, kB = B;
    int kq = 1 << 30;
    if (live && B <= thr) {
      const double da = ca - ia, db = cb - ib;
      kd = da * da + db * db;
      ka = ca;
      kb = cb;
      kq = q;
    }
    wave_pick(kd, ka, kb, kq, kB);
    if (l > 0 && sB <= thr) {  // the best so far, index K^2, after every lane
      const double da = sa - ia, db = sb - ib;
      const double ds = da * da + db * db;
      if (kq == (1 << 30) || later_wins(ds, sa, sb, kd, ka, kb)) {
        ka = sa;
        kb = sb;
        kB = sB;
      }
    }
    sa = ka;
    sb = kb;
    sB = kB;
  }
  // acceptance against the incumbent (index 1, after the search's winner)
  double ci[kW2Grp] = {ia}, Bi8[kW2Grp];
  w2_B_column<kW2Grp>(P, u1a, u1b, x1, x2, ci, ib, 1, Bi8, tab);
  const double Bi = Bi8[0];
  double m = sB;
  if (Bi < m) m = Bi;
  const double thr = m * (1.0 + P.tau);
  double ra = sa, rb = sb, rB = sB;
  if (Bi <= thr) {
    const double da = sa - ia, db = sb - ib;
    const double ds = da * da + db * db;
    const double ea = ia - ia, eb = ib - ib;
    const double di = ea * ea + eb * eb;
    if (!(sB <= thr) || later_wins(di, ia, ib, ds, sa, sb)) {
      ra = ia;
      rb = ib;
      rB = Bi;
    }
  }
  if (q == 0) {
    u0_out[i] = ra;
    u0_out[nn + i] = rb;
    if (L0_out) L0_out[i] = f[i / P.n] * f[i % P.n] * rB;
  }
}

// u: [2][n^2][n_cand]; out: [n^2][n_cand].
__global__ __launch_bounds__(256) void k_w2_mc(W2Params P, const double* __restrict__ f,
                                               const double* __restrict__ u1, const double* __restrict__ u,
                                               int n_cand, double* __restrict__ out) {
  const long nn = (long)P.n * P.n;
  const long g = (long)blockIdx.x * 256 + threadIdx.x;
  if (g >= nn * n_cand) return;
  const int i = (int)(g / n_cand);
  const double* u1b = u1 + (long)P.ny * P.ny;
  out[g] = f[i / P.n] * f[i % P.n] *
           w2_B(P, u1, u1b, xnode(P, i / P.n), xnode(P, i % P.n), u[g], u[nn * n_cand + g]);
}

// One wave: 64 consecutive y nodes (lane = node) against segment blockIdx.y
// of the x nodes: pass 1 finds the segment's maximum of
// l = log f(x_i) - |y - x1_i|^2 / 2, pass 2 sums x1_i e^(l - M) and e^(l - M).
// part[((seg * ny^2 + j) * 4 + {0..3}] = (M, sum x1a e, sum x1b e, sum e).
__global__ __launch_bounds__(64) void k_w2_u1_part(W2Params P, const double* __restrict__ f,
                                                   const double* __restrict__ u0, double* __restrict__ part) {
  __shared__ double sa[kW2Tile], sb[kW2Tile], sl[kW2Tile];
  const int nn = P.n * P.n, m = P.ny * P.ny;
  const int j = blockIdx.x * 64 + threadIdx.x;
  const bool live = j < m;
  const int jj = live ? j : m - 1;
  const double ya = ynode(P, jj / P.ny), yb = ynode(P, jj % P.ny);
  const int i0 = blockIdx.y * P.seg_len, i1 = min(nn, i0 + P.seg_len);
  double M = -INFINITY, na = 0.0, nb = 0.0, den = 0.0;
  for (int pass = 0; pass < 2; ++pass) {
    for (int t0 = i0; t0 < i1; t0 += kW2Tile) {
      const int cnt = min(kW2Tile, i1 - t0);
      for (int k = threadIdx.x; k < cnt; k += 64) {
        const int i = t0 + k;
        sa[k] = xnode(P, i / P.n) + u0[i];
        sb[k] = xnode(P, i % P.n) + u0[nn + i];
        sl[k] = log(f[i / P.n]) + log(f[i % P.n]);
      }
      __syncthreads();
      for (int k = 0; k < cnt; ++k) {
        const double da = ya - sa[k], db = yb - sb[k];
        const double l = sl[k] - 0.5 * (da * da + db * db);
        if (pass == 0) {
          M = fmax(M, l);
        } else {
          const double e = M == -INFINITY ? 0.0 : exp(l - M);  // a segment whose prior underflows
          na = fma(sa[k], e, na);
          nb = fma(sb[k], e, nb);
          den += e;
        }
      }
      __syncthreads();
    }
  }
  if (live) {
    const long o = ((long)blockIdx.y * m + j) * 4;
    part[o] = M;
    part[o + 1] = na;
    part[o + 2] = nb;
    part[o + 3] = den;
  }
}

__global__ __launch_bounds__(256) void k_w2_u1_fin(W2Params P, const double* __restrict__ part,
                                                   double* __restrict__ u1) {
  const int m = P.ny * P.ny;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= m) return;
  double M = -INFINITY;
  for (int s = 0; s < P.n_seg; ++s) M = fmax(M, part[((long)s * m + j) * 4]);
  double na = 0.0, nb = 0.0, den = 0.0;
  for (int s = 0; s < P.n_seg; ++s) {
    const long o = ((long)s * m + j) * 4;
    const double c = part[o] == -INFINITY ? 0.0 : exp(part[o] - M);
    na = fma(part[o + 1], c, na);
    nb = fma(part[o + 2], c, nb);
    den = fma(part[o + 3], c, den);
  }
  u1[j] = den > 0.0 ? na / den : 0.0;
  u1[m + j] = den > 0.0 ? nb / den : 0.0;
}

// Objective rows f_i B(u0_i; x_i), one lane per point, block sums in a
// fixed tree.
__global__ __launch_bounds__(256) void k_w2_jrows(W2Params P, const double* __restrict__ f,
                                                  const double* __restrict__ u0, const double* __restrict__ u1,
                                                  double* __restrict__ jpart) {
  __shared__ double sh[256];
  const int nn = P.n * P.n;
  const int i = blockIdx.x * 256 + threadIdx.x;
  double r = 0.0;
  if (i < nn)
    r = f[i / P.n] * f[i % P.n] *
        w2_B(P, u1, u1 + (long)P.ny * P.ny, xnode(P, i / P.n), xnode(P, i % P.n), u0[i], u0[nn + i]);
  sh[threadIdx.x] = r;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) jpart[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_w2_jsum(int n, double w, const double* __restrict__ jpart,
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
  if (threadIdx.x == 0) *J = w * sh[0];
}

// ------------------------------------------------------------------- host

inline size_t al(size_t v) { return (v + 255) & ~(size_t)255; }
inline unsigned blocks(long n, int per) { return (unsigned)((n + per - 1) / per); }

struct W2Work {
  double *f, *part, *jpart;
};

int w2_params(const ucp_problem* p, const ucp_search* s, W2Params& P) {
  int rc = check_problem(p);
  if (rc) return rc;
  if (p->noise_sd != 0.0 && p->noise_sd != 1.0)
    return fail(UCP_EINVAL, "the 2-D problem has unit noise N(0, I_2): noise_sd must be 0 or 1");
  if (p->n_x > 4096 || p->n_y > 4096) return fail(UCP_EINVAL, "2-D grids take at most 4096 nodes per coordinate");
  if (s) {
    if ((rc = check_search(s))) return rc;
    if (s->cands > 8) return fail(UCP_EINVAL, "2-D search takes at most 8 x 8 candidates per level");
  }
  std::memset(&P, 0, sizeof P);
  P.tau = tie_band(s);
  P.k = p->k;
  P.n_comp = p->n_comp;
  P.n = (int)p->n_x;
  P.ny = (int)p->n_y;
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
  P.Q = std::exp(-P.dy * P.dy);
  // the window runs wn = floor(kW2Win / dy) nodes either side of z's
  // nearest node, so every node it drops lies at least (wn + 1/2) dy >=
  // kW2Win - dy / 2 from z; on the paper's grid (dy = 50/159) that is 31
  // nodes each side, 63 columns, one chunk of a wave's lanes
  const double wn = std::floor(kW2Win * P.inv_dy);
  P.wn = (int)std::fmax(1.0, std::fmin(wn, (double)P.ny));
  if (s) {
    P.u_lo = s->u_lo;
    P.u_hi = s->u_hi;
    P.levels = s->levels;
    P.cands = s->cands;
    P.h[0] = (s->u_hi - s->u_lo) / (double)(s->cands - 1);
    for (int l = 1; l < s->levels; ++l) P.h[l] = 2.0 * P.h[l - 1] / (double)(s->cands - 1);
  }
  const int nn = P.n * P.n;
  P.n_seg = std::min(kW2Seg, (nn + kW2Tile - 1) / kW2Tile);
  P.seg_len = (nn + P.n_seg - 1) / P.n_seg;
  P.n_seg = (nn + P.seg_len - 1) / P.seg_len;
  return UCP_OK;
}

int w2_work(ucp_handle* h, const W2Params& P, W2Work& W) {
  const size_t nn = (size_t)P.n * P.n, m = (size_t)P.ny * P.ny;
  const size_t sz[3] = {al(8 * (size_t)P.n), al(8 * 4 * (size_t)P.n_seg * m), al(8 * ((nn + 255) / 256))};
  void* base = nullptr;
  int rc = handle_workspace(h, sz[0] + sz[1] + sz[2], &base);
  if (rc) return rc;
  char* p = (char*)base;
  W.f = (double*)p;
  W.part = (double*)(p + sz[0]);
  W.jpart = (double*)(p + sz[0] + sz[1]);
  return UCP_OK;
}

#define W2_TRY(expr, what)                           \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

hipError_t w2_prior(const W2Params& P, const W2Work& W, hipStream_t st) {
  hipLaunchKernelGGL(k_w2_prior, dim3(blocks(P.n, 256)), dim3(256), 0, st, P, W.f);
  return hipGetLastError();
}

hipError_t w2_search(ucp_handle* h, const W2Params& P, const W2Work& W, const double* u1, const double* u0_in,
                     double* u0_out, double* L0_out, hipStream_t st) {
  hipEvent_t a, b;
  hipError_t e = handle_events(h, UCP_PROF_MC, &a, &b);
  if (e != hipSuccess) return e;
  hipExtLaunchKernelGGL(k_w2_search, dim3(P.n * P.n), dim3(64), 0, st, a, b, 0, P, (const double*)W.f, u1, u0_in,
                        u0_out, L0_out);
  return hipGetLastError();
}

hipError_t w2_u1(ucp_handle* h, const W2Params& P, const W2Work& W, const double* u0, double* u1, hipStream_t st) {
  hipEvent_t a, b;
  hipError_t e = handle_events(h, UCP_PROF_U1, &a, &b);
  if (e != hipSuccess) return e;
  const long m = (long)P.ny * P.ny;
  hipExtLaunchKernelGGL(k_w2_u1_part, dim3(blocks(m, 64), P.n_seg), dim3(64), 0, st, a, nullptr, 0, P,
                        (const double*)W.f, u0, W.part);
  hipExtLaunchKernelGGL(k_w2_u1_fin, dim3(blocks(m, 256)), dim3(256), 0, st, nullptr, b, 0, P,
                        (const double*)W.part, u1);
  return hipGetLastError();
}

hipError_t w2_objective(ucp_handle* h, const W2Params& P, const W2Work& W, const double* u0, const double* u1,
                        double* J, hipStream_t st) {
  hipEvent_t a, b;
  hipError_t e = handle_events(h, UCP_PROF_J, &a, &b);
  if (e != hipSuccess) return e;
  const unsigned nb = blocks((long)P.n * P.n, 256);
  hipExtLaunchKernelGGL(k_w2_jrows, dim3(nb), dim3(256), 0, st, a, nullptr, 0, P, (const double*)W.f, u0, u1,
                        W.jpart);
  hipExtLaunchKernelGGL(k_w2_jsum, dim3(1), dim3(256), 0, st, nullptr, b, 0, (int)nb, P.dx * P.dx,
                        (const double*)W.jpart, J);
  return hipGetLastError();
}

int w2_begin(ucp_handle* h) {
  hipError_t e = hipSetDevice(handle_device(h));
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  return UCP_OK;
}

}  // namespace
}  // namespace ucp

using namespace ucp;

extern "C" {

int ucp_w2_marginal_cost(ucp_handle* h, const ucp_problem* prob, const double* u1, const double* u, int64_t n_cand,
                         double* L0_out, void* stream) {
  int rc;
  W2Params P;
  if (!h) return fail(UCP_EINVAL, "handle is NULL");
  if ((rc = w2_params(prob, nullptr, P))) return rc;
  if (!u1 || !u || !L0_out) return fail(UCP_EINVAL, "NULL array argument");
  if (n_cand < 1 || n_cand > 4096) return fail(UCP_EINVAL, "n_cand must be 1..4096");
  if ((int64_t)P.n * P.n * n_cand > ((int64_t)1 << 30)) return fail(UCP_EINVAL, "n_x^2 * n_cand too large");
  if ((rc = w2_begin(h))) return rc;
  W2Work W;
  if ((rc = w2_work(h, P, W))) return rc;
  hipStream_t st = (hipStream_t)stream;
  W2_TRY(w2_prior(P, W, st), "prior kernel");
  hipLaunchKernelGGL(k_w2_mc, dim3(blocks((long)P.n * P.n * n_cand, 256)), dim3(256), 0, st, P, (const double*)W.f,
                     u1, u, (int)n_cand, L0_out);
  W2_TRY(hipGetLastError(), "marginal-cost kernel");
  return UCP_OK;
}

int ucp_w2_argmin(ucp_handle* h, const ucp_problem* prob, const ucp_search* search, const double* u1,
                  const double* u0_in, double* u0_out, double* L0_out, void* stream) {
  int rc;
  W2Params P;
  if (!h) return fail(UCP_EINVAL, "handle is NULL");
  if (!search) return fail(UCP_EINVAL, "search is NULL");
  if ((rc = w2_params(prob, search, P))) return rc;
  if (!u1 || !u0_in || !u0_out) return fail(UCP_EINVAL, "NULL array argument");
  if ((rc = w2_begin(h))) return rc;
  W2Work W;
  if ((rc = w2_work(h, P, W))) return rc;
  hipStream_t st = (hipStream_t)stream;
  W2_TRY(w2_prior(P, W, st), "prior kernel");
  W2_TRY(w2_search(nullptr, P, W, u1, u0_in, u0_out, L0_out, st), "search kernel");
  return UCP_OK;
}

int ucp_w2_update_u1(ucp_handle* h, const ucp_problem* prob, const double* u0, double* u1_out, void* stream) {
  int rc;
  W2Params P;
  if (!h) return fail(UCP_EINVAL, "handle is NULL");
  if ((rc = w2_params(prob, nullptr, P))) return rc;
  if (!u0 || !u1_out) return fail(UCP_EINVAL, "NULL array argument");
  if ((rc = w2_begin(h))) return rc;
  W2Work W;
  if ((rc = w2_work(h, P, W))) return rc;
  hipStream_t st = (hipStream_t)stream;
  W2_TRY(w2_prior(P, W, st), "prior kernel");
  W2_TRY(w2_u1(nullptr, P, W, u0, u1_out, st), "u1 kernels");
  return UCP_OK;
}

int ucp_w2_objective(ucp_handle* h, const ucp_problem* prob, const double* u0, const double* u1, double* J_out,
                     void* stream) {
  int rc;
  W2Params P;
  if (!h) return fail(UCP_EINVAL, "handle is NULL");
  if ((rc = w2_params(prob, nullptr, P))) return rc;
  if (!u0 || !u1 || !J_out) return fail(UCP_EINVAL, "NULL array argument");
  if ((rc = w2_begin(h))) return rc;
  W2Work W;
  if ((rc = w2_work(h, P, W))) return rc;
  hipStream_t st = (hipStream_t)stream;
  W2_TRY(w2_prior(P, W, st), "prior kernel");
  W2_TRY(w2_objective(nullptr, P, W, u0, u1, J_out, st), "objective kernels");
  return UCP_OK;
}

int ucp_w2_solve(ucp_handle* h, const ucp_problem* prob, const ucp_search* search, int32_t iters,
                 const double* u0_init, double* u0_out, double* u1_out, double* J_hist, void* stream) {
  int rc;
  W2Params P;
  if (!h) return fail(UCP_EINVAL, "handle is NULL");
  if (!search) return fail(UCP_EINVAL, "search is NULL");
  if ((rc = w2_params(prob, search, P))) return rc;
  if (!u0_init || !u0_out || !u1_out || !J_hist) return fail(UCP_EINVAL, "NULL array argument");
  if (iters < 0) return fail(UCP_EINVAL, "iters must be >= 0");
  if ((rc = w2_begin(h))) return rc;
  W2Work W;
  if ((rc = w2_work(h, P, W))) return rc;
  hipStream_t st = (hipStream_t)stream;
  W2_TRY(w2_prior(P, W, st), "prior kernel");
  if (u0_out != u0_init)
    W2_TRY(hipMemcpyAsync(u0_out, u0_init, sizeof(double) * 2 * P.n * P.n, hipMemcpyDeviceToDevice, st),
           "copy u0");
  W2_TRY(w2_u1(h, P, W, u0_out, u1_out, st), "u1 kernels");
  W2_TRY(w2_objective(h, P, W, u0_out, u1_out, J_hist, st), "objective kernels");
  for (int t = 1; t <= iters; ++t) {
    W2_TRY(w2_search(h, P, W, u1_out, u0_out, u0_out, nullptr, st), "search kernel");
    W2_TRY(w2_u1(h, P, W, u0_out, u1_out, st), "u1 kernels");
    W2_TRY(w2_objective(h, P, W, u0_out, u1_out, J_hist + t, st), "objective kernels");
  }
  if (handle_profiling(h)) {
    W2_TRY(hipStreamSynchronize(st), "synchronise");
    handle_harvest(h);
  }
  return UCP_OK;
}

}  // extern "C"
