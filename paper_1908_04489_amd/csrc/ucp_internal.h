// Internal definitions shared by the HIP kernels and the host runtime of the
// marginal-cost solver.  Not part of the public ABI (include/ucp.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "ucp.h"

namespace ucp {

constexpr int kMaxLevels = UCP_MAX_LEVELS;
constexpr int kMaxComp = UCP_MAX_COMP;
constexpr int kWave = 64;
constexpr int kMcBlock = 256;   // marginal-cost kernel: one lane per point, 4 waves
// FP32 nodes staged in LDS per block (40 KiB: with the block's other LDS,
// four blocks fill a CU's 160 KiB, the occupancy the registers allow anyway)
constexpr int kMcLds = 10208;
// longest window segment of one marginal-cost work unit (a block's stage,
// 256 points plus a segment, still fits the LDS stage)
constexpr int kMcSegMax = 8192;
constexpr int kGtabPad = 16;    // offset-table entries past the window (>= the marginal-cost unroll)
// reference form when every z of a block lies within this of the block's
// centre: wide enough for the jumps of a point's best candidate on the
// coarse level-0 grid within a block, narrow enough that the staged
// differences round no worse than the residual form's
constexpr double kMcRefHalf = 2.5;
constexpr double kMcBetaMax = 4.0; // blocked sums only where weights change by <= 2^4 per node
constexpr int kSelWaves = 4;    // selection kernel: waves per block
constexpr int kU1Block = 256;   // u1 kernels: lanes per block (one or kU1Npl y nodes each)
constexpr int kU1Chunk = 512;   // x nodes staged in LDS per step of the u1 sums
constexpr int kU1Sample = 32;   // x-node stride of the sample bounding a tile's logit maximum
constexpr double kU1Cull = 64.0; // chunks whose logits all lie this far below that bound are skipped
// y nodes per lane of the u1 sums on large, fine grids (one exponential
// per x node and lane, the other nodes' weights by a staged ratio)
constexpr int kU1Npl = 4;
constexpr int kU1NplMinNodes = 16384;  // grids of at least this many y nodes
constexpr double kU1NplMaxStep = 0.05; // and a spacing of at most this many noise sds
constexpr int kJWaves = 4;      // objective: one wave ...
constexpr int kJPts = 4;        // ... per kJPts consecutive x nodes
// FP32 tie band B32 <= m (1 + tau) + kappa sqrt(m): tau covers the relative
// error of the Gaussian weights and of the sums, kappa sqrt(m) the rounding
// of z - u1 in FP32, which dominates where the cost is small.  The band keeps
// the FP64 minimum (to first order) while every candidate's error stays
// below half of tau B + kappa sqrt(B); measured on solver states of five
// workloads at every level, the worst is 0.28 of it with compensated sums
// and 0.20 with plain sums.
constexpr double kTau32Kahan = 5e-7;
constexpr double kTau32Plain = 5e-6;
constexpr double kKappa32 = 6e-7;
constexpr double kTau64 = 1e-12;// FP64 tie band (relative)
constexpr int kGtN = 12;        // expansion order of the Gauss-transform moment table
constexpr double kGtStep = 0.05; // its rows lie at most this many noise sds apart
constexpr double kWin32 = 9.0;  // window half-width, noise sds (FP32 terms)
// FP64 window half-width, noise sds.  B has no useful lower bound (a point
// whose x0 + u lands on a flat step of u1 has B far below the noise
// variance), so the width is set by the dropped tail against B itself: the
// tail is at most 2 phi(11)/11 max(z - u1)^2 = 3.9e-28 max(z - u1)^2, below
// 1e-16 of B wherever B >= 4e-12 max(z - u1)^2; on solver states of the
// sigma = 10 sign controller (B down to 2e-6) it is 6e-21 of B, where 9
// sds left 3.5e-12.
constexpr double kWin64 = 11.0;
// Device counters (spread over slots on separate cache lines): algorithmic
// marginal-cost terms and FP64 tie re-evaluations.
constexpr int kCountSlots = 32, kCountStride = 16, kCountTerms = 0, kCountEvalTerms = 4, kCountEvals = 8;
constexpr size_t kCountBytes = (size_t)kCountSlots * kCountStride * 8;

// A point's queued FP64 sums take a whole number of chunks of kEvalChunk
// entries (padding entries have i = -1), so the chunks, and the positions
// that share one pass over their windows, depend on the point alone.
constexpr int kEvalChunk = 4;

// One solve instance as the kernels see it: constants of the problem and the
// search, launch geometry, and device pointers to its state.
struct Inst {
  // problem
  double k2;                 // k^2
  double x_lo, dx;           // x node i = x_lo + i * dx
  double y_lo, dy, inv_dy;   // y node j = y_lo + j * dy
  double phi_scale;          // dy / (s sqrt(2 pi)), s the noise sd
  double sw, isw;            // noise sd s and 1 / s
  double alpha, a2;          // sqrt(log2(e) / 2) / s and its square: exp(-t^2 / (2 s^2)) = exp2(-(alpha t)^2)
  double win32;              // FP32 window half-width in y units, kWin32 s
  double w[kMaxComp], mu[kMaxComp], sd[kMaxComp];
  int32_t n_comp;
  int32_t n_x, n_y;
  // search
  int32_t levels, cands;
  double u_lo, u_hi;
  double h[kMaxLevels];      // candidate spacing per level
  double tau64;              // relative FP64 tie band of the selection rule
  double tau32;              // relative part of the FP32 pre-selection band (holds tau64)
  // geometry
  int32_t nw32, nw64;        // window half-widths in y nodes
  int32_t rs64;              // FP64 walks: steps of a wave between reseeds (a power of two, <= 32)
  int32_t gts;               // moment table: rows every gts-th y node (0: no table)
  int32_t gtr;               // its rows, centred on nodes r gts - gto (r < gtr), from at
  int32_t gto;               // least nw64 before the grid to nw64 past it (gto a multiple of gts)
  int32_t segs;              // marginal-cost units (partial sums) per (tile, candidate)
  int32_t wsegs;             // equal window segments (the last one dispatched split in two when segs > wsegs)
  int32_t u1_slices;         // x slices of the u1 sums
  int32_t u1_npl;            // consecutive y nodes per lane of the u1 sums (1 or kU1Npl)
  int32_t prec;              // ucp_prec
  int32_t free_cands;        // 1: explicit candidates (u0 holds [n_x][cands]), no search
  // state
  double* u0;                // current first controller [n_x] (explicit candidates for ucp_marginal_cost)
  double* u0_next;           // updated first controller [n_x]
  double* u1;                // second controller [n_y]
  float* v;                  // alpha * (y_j - u1_j), FP32 [n_y]
  float* gtab;               // exp(-(k dy)^2 / 2) for -nw32 <= k <= nw32 + kGtabPad, FP32
  double* f;                 // prior density at x nodes [n_x]
  double* logf;              // its logarithm [n_x]
  double* cbest;             // best candidate so far [n_x]
  double* b32best;           // its FP32-path cost B [n_x]
  double* b64best;           // its FP64 cost B, NaN when not evaluated [n_x]
  double* b32inc;            // FP32-path cost B of the incumbent [n_x]
  double* part;              // marginal-cost partial sums, part_idx(point, slot, segment)
  double* u1part;            // u1 partial sums [u1_slices][n_y][3]
  double* u1stat;            // u1 culling data: per-tile logit bounds, then per-chunk x1 range and max log f
  double* jrow;              // per-point objective terms [n_x]
  double* gt;                // moment table [gtr][3][kGtN + 1] (A0, A1, A2 by order), or NULL
  double* J_out;             // objective output (one double)
  double* L0_out;            // optional FP64 L_0 of the accepted u0 [n_x] (argmin call only)
  int32_t* flags;            // bit 0: non-finite value met
  unsigned long long* terms; // counters [kCountSlots][kCountStride] (NULL: not counted)
};

// Marginal-cost partial sums: tiles of kPartTile consecutive points, each
// tile laid out [slot][segment][point], so a wave of the marginal-cost
// kernels (64 consecutive points, one slot and segment) writes whole 64-byte
// lines and a selection block (8 consecutive points) reads one contiguous
// span.  n_x is padded to whole tiles.
constexpr int kPartTile = 8;
__host__ __device__ inline size_t part_idx(const Inst& I, int i, int q, int g) {
  return (((size_t)(i / kPartTile) * (size_t)(I.cands + 1) + (size_t)q) * (size_t)I.segs + (size_t)g) * kPartTile +
         (size_t)(i % kPartTile);
}
__host__ __device__ inline size_t part_doubles(const Inst& I) {
  return (size_t)((I.n_x + kPartTile - 1) / kPartTile) * kPartTile * (size_t)(I.cands + 1) * (size_t)I.segs;
}

// Whether the instance's selection takes its FP64 values from the moment
// table (the FP32 modes on grids that have one).
__host__ __device__ inline bool table_select(const Inst& I) {
  return I.gts > 0 && (I.prec == UCP_FP32 || I.prec == UCP_FP32_KAHAN);
}

// Lanes per point in the selection kernels: two points per wave when the
// level's set and the incumbent (cands + 2 lanes) fit in half a wave.
__host__ __device__ inline int sel_width(const Inst& I) { return I.cands + 2 <= 32 ? 32 : 64; }

// alpha^2 = log2(e) / 2, so exp(-t^2 / 2) = exp2(-(alpha t)^2).
constexpr double kAlpha2 = 0.72134752044448170367996234050095;  // log2(e)/2
constexpr double kInvSqrt2Pi = 0.39894228040143267793994605993438;

// Launch tables: prefix sums of work units per instance for each kernel.
struct Launch {
  const Inst* insts;   // device array [n_inst]
  const int32_t* pre;  // device prefix array [n_inst + 1]
  int32_t n_inst;
  int32_t total;       // pre[n_inst]
};

// Kernel launchers (ucp_kernels.hip).  All enqueue on `st`.
hipError_t launch_prior(const Launch& L, hipStream_t st);
hipError_t launch_gtab(const Launch& L, hipStream_t st);
// The moment table of every instance that keeps one (from its current u1)
hipError_t launch_gt_table(const Launch& L, hipStream_t st);
// Launchers that take (e0, e1) record e0 when the first kernel starts and e1
// when the last one ends (hipExtLaunchKernel: no extra packets in the stream).
hipError_t launch_mc(const Launch& L, int level, int prec, hipStream_t st, hipEvent_t e0 = nullptr,
                     hipEvent_t e1 = nullptr);
// The selection of one level: Lw over the instances that settle their FP32
// ties by FP64 window sums, Lt over those that take them from the moment
// table (table_select).
hipError_t launch_select(const Launch& Lw, const Launch& Lt, int level, int prec, int final_l0, hipStream_t st,
                         hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_finish_free(const Launch& L, double* out, int prec, hipStream_t st);
hipError_t launch_j_reduce_t(const Launch& L, int t, hipStream_t st, hipEvent_t e1 = nullptr);
// the u1 partial sums: Ls the culling-data units (kKindU1s), L the
// partial-sum units (kKindU1p) of the same instances
hipError_t launch_u1_partial(const Launch& Ls, const Launch& L, int prec, hipStream_t st, hipEvent_t e0 = nullptr);
hipError_t launch_u1_combine(const Launch& L, hipStream_t st, hipEvent_t e1 = nullptr);
hipError_t launch_j_rows(const Launch& L, hipStream_t st, hipEvent_t e0 = nullptr);
hipError_t launch_j_reduce(const Launch& L, hipStream_t st);
hipError_t launch_copy_u0(const Launch& L, hipStream_t st);

// Generic solver (Algorithm 1) on one instance; dI is the device copy of the
// instance record.  r is the partial-exhaustion radius (1 or 2).
hipError_t launch_a1_local_u0(const Inst* dI, int n_x, double tau, const double* u0_in, double* u0_out,
                              hipStream_t st);
hipError_t launch_a1_pe_u0(const Inst* dI, int n_x, int r, double tie, const double* u0_in, double* u0_out,
                           hipStream_t st);
// part: [u1_slices][n_y][2 r + 2] FP64
hipError_t launch_a1_pe_u1(const Inst& I, const Inst* dI, int r, double tie, const double* u1_in, double* part,
                           double* u1_out, hipStream_t st);

// Units per instance of each kernel (host helpers, ucp_kernels.hip).
int32_t units_mc(const Inst& I, int level);
int32_t units_select(const Inst& I);
int32_t units_u1_partial(const Inst& I);
int32_t units_u1_stats(const Inst& I);
// doubles of the u1 culling data
size_t u1stat_doubles(const Inst& I);
int32_t units_u1_combine(const Inst& I);
int32_t units_j_rows(const Inst& I);
int32_t units_prior(const Inst& I);
int32_t units_gtab(const Inst& I);
int32_t units_gt(const Inst& I);

}  // namespace ucp
