// Host runtime of the marginal-cost solver: argument checks, the handle and
// its device workspace, launch tables over batches of instances, and the
// solve loop.  Everything numerical runs in the HIP kernels
// (ucp_kernels.hip); this file only validates, lays out memory and enqueues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ucp_internal.h"
#include "ucp_runtime.h"

namespace ucp {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(UCP_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int check_problem(const ucp_problem* p) {
  if (!p) return fail(UCP_EINVAL, "problem is NULL");
  if (!(p->k >= 0.0) || !std::isfinite(p->k)) return fail(UCP_EINVAL, "k must be finite and >= 0");
  if (p->n_comp < 1 || p->n_comp > UCP_MAX_COMP) return fail(UCP_EINVAL, "n_comp must be 1..%d", UCP_MAX_COMP);
  double ws = 0.0;
  for (int c = 0; c < p->n_comp; ++c) {
    if (!(p->w[c] > 0.0) || !std::isfinite(p->w[c])) return fail(UCP_EINVAL, "prior weight %d must be > 0", c);
    if (!(p->sd[c] > 0.0) || !std::isfinite(p->sd[c])) return fail(UCP_EINVAL, "prior sd %d must be > 0", c);
    if (!std::isfinite(p->mu[c])) return fail(UCP_EINVAL, "prior mean %d must be finite", c);
    ws += p->w[c];
  }
  if (std::fabs(ws - 1.0) > 1e-9) return fail(UCP_EINVAL, "prior weights must sum to 1 (got %.17g)", ws);
  if (p->n_x < 2 || p->n_y < 2) return fail(UCP_EINVAL, "grids need at least 2 nodes");
  // per-wave work counters are 32-bit sums of up to 64 windows of at most n_y nodes
  if (p->n_x > (int64_t)1 << 24 || p->n_y > (int64_t)1 << 24) return fail(UCP_EINVAL, "grid too large (more than 2^24 nodes)");
  if (!(p->x_lo < p->x_hi) || !std::isfinite(p->x_lo) || !std::isfinite(p->x_hi))
    return fail(UCP_EINVAL, "x grid needs finite x_lo < x_hi");
  if (!(p->y_lo < p->y_hi) || !std::isfinite(p->y_lo) || !std::isfinite(p->y_hi))
    return fail(UCP_EINVAL, "y grid needs finite y_lo < y_hi");
  if (std::fabs(p->x_lo) > 1e6 || std::fabs(p->x_hi) > 1e6 || std::fabs(p->y_lo) > 1e6 || std::fabs(p->y_hi) > 1e6)
    return fail(UCP_EINVAL, "grid bounds beyond 1e6");
  if (!(p->noise_sd >= 0.0) || !(p->noise_sd <= 1e6)) return fail(UCP_EINVAL, "noise_sd must be in [0, 1e6] (0: 1)");
  if (p->noise_sd > 0.0 && p->noise_sd < 1e-6) return fail(UCP_EINVAL, "noise_sd below 1e-6");
  return UCP_OK;
}

int check_search(const ucp_search* s) {
  if (!s) return fail(UCP_EINVAL, "search is NULL");
  if (s->levels < 1 || s->levels > UCP_MAX_LEVELS) return fail(UCP_EINVAL, "levels must be 1..%d", UCP_MAX_LEVELS);
  if (s->cands < 2 || s->cands > UCP_MAX_CANDS) return fail(UCP_EINVAL, "cands must be 2..%d", UCP_MAX_CANDS);
  if (!(s->u_lo < s->u_hi) || !std::isfinite(s->u_lo) || !std::isfinite(s->u_hi))
    return fail(UCP_EINVAL, "search needs finite u_lo < u_hi");
  if (std::fabs(s->u_lo) > 1e6 || std::fabs(s->u_hi) > 1e6) return fail(UCP_EINVAL, "search bounds beyond 1e6");
  if (!(s->tie_rel64 >= 0.0 && s->tie_rel64 <= 1e-3)) return fail(UCP_EINVAL, "tie_rel64 must be in [0, 1e-3]");
  if (!(s->band_rel32 >= 0.0 && s->band_rel32 <= 1e-2)) return fail(UCP_EINVAL, "band_rel32 must be in [0, 1e-2]");
  return UCP_OK;
}

double tie_band(const ucp_search* s) { return s && s->tie_rel64 > 0.0 ? s->tie_rel64 : kTau64; }

int check_prec(int prec) {
  if (prec != UCP_FP32 && prec != UCP_FP32_KAHAN && prec != UCP_FP64 && prec != UCP_FP64_GT)
    return fail(UCP_EINVAL, "unknown precision %d", prec);
  return UCP_OK;
}

int check_gt(const Inst& I) {
  if (I.prec == UCP_FP64_GT && I.gts == 0)
    return fail(UCP_EINVAL, "UCP_FP64_GT needs dy / noise_sd <= %g (the moment table's order is %d); got %g",
                kGtStep, kGtN, I.dy * I.isw);
  return UCP_OK;
}

// Stride of the moment table's rows, in y nodes: the largest m with
// m dy / s <= kGtStep for which order kGtN meets the truncation bound
//   x^{N+1} / (N+1)! / (1 - x / (N+2)) <= 1e-17,  x = h T,
// h = m dy / (2 s) the largest |z - y_k| / s of a position from its row's
// node and T = nw64 dy / s the window's reach (the remainder of the series
// of exp(t d), |t| <= T, |d| <= h).  0 when even m = 1 is too coarse.
static int32_t gt_stride(const Inst& I) {
  const double r = I.dy * I.isw;
  if (r > kGtStep * (1.0 + 1e-12)) return 0;
  const double T = (double)I.nw64 * r;
  int32_t m = std::max(1, (int32_t)std::floor(kGtStep / r * (1.0 + 1e-12)));
  m = std::min(m, std::max(1, I.nw64));
  for (; m >= 1; --m) {
    const double x = 0.5 * (double)m * r * T;
    double b = 1.0;
    for (int n = 1; n <= kGtN + 1; ++n) b *= x / (double)n;
    if (b / (1.0 - x / (double)(kGtN + 2)) <= 1e-17) return m;
  }
  return 0;
}

// Constants and launch geometry of one instance.  Everything here depends on
// the instance alone, never on the batch it runs in.
Inst make_inst(const ucp_problem& p, const ucp_search* s, int prec, int cands_override) {
  Inst I;
  std::memset(&I, 0, sizeof I);
  I.k2 = p.k * p.k;
  I.x_lo = p.x_lo;
  I.dx = (p.x_hi - p.x_lo) / (double)(p.n_x - 1);
  I.y_lo = p.y_lo;
  I.dy = (p.y_hi - p.y_lo) / (double)(p.n_y - 1);
  I.inv_dy = 1.0 / I.dy;
  // noise w ~ N(0, s^2): every Gaussian argument is taken in noise sds
  I.sw = p.noise_sd > 0.0 ? p.noise_sd : 1.0;
  I.isw = 1.0 / I.sw;
  I.alpha = std::sqrt(kAlpha2) * I.isw;
  I.a2 = kAlpha2 * I.isw * I.isw;
  I.win32 = kWin32 * I.sw;
  I.phi_scale = I.dy * kInvSqrt2Pi * I.isw;
  I.n_comp = p.n_comp;
  for (int c = 0; c < p.n_comp; ++c) {
    I.w[c] = p.w[c];
    I.mu[c] = p.mu[c];
    I.sd[c] = p.sd[c];
  }
  I.n_x = (int32_t)p.n_x;
  I.n_y = (int32_t)p.n_y;
  if (s) {
    I.levels = s->levels;
    I.cands = s->cands;
    I.u_lo = s->u_lo;
    I.u_hi = s->u_hi;
    // spacings: h0 spans the range with `cands` nodes, each later level spans
    // twice the previous spacing with `cands` nodes
    I.h[0] = (s->u_hi - s->u_lo) / (double)(s->cands - 1);
    for (int l = 1; l < s->levels; ++l) I.h[l] = 2.0 * I.h[l - 1] / (double)(s->cands - 1);
  } else {
    I.levels = 1;
    I.cands = cands_override;
  }
  if (cands_override > 0) I.cands = cands_override;
  I.tau64 = tie_band(s);
  // the FP32 band holds every candidate the FP64 band could hold
  I.tau32 = (s && s->band_rel32 > 0.0 ? s->band_rel32 : prec == UCP_FP32_KAHAN ? kTau32Kahan : kTau32Plain) + I.tau64;
  I.nw32 = (int32_t)std::min<double>(std::ceil(kWin32 * I.sw / I.dy), (double)I.n_y);
  I.nw64 = (int32_t)std::min<double>(std::ceil(kWin64 * I.sw / I.dy), (double)I.n_y);
  // a wave's FP64 walk steps 64 nodes at a time: reseed at least every 24
  // noise sds, so a weight that underflowed far from its position is
  // recomputed before its peak
  I.rs64 = 32;
  while (I.rs64 > 1 && I.rs64 * 64.0 * I.dy * I.isw > 24.0) I.rs64 /= 2;
  I.prec = prec;
  // the moment table: UCP_FP64_GT takes every cost from it; a search in the
  // FP32 modes takes its FP64 values (tie-breaks, L_0) from it where the
  // grid allows, and from window sums elsewhere.  UCP_FP64 keeps none.
  if (prec == UCP_FP64_GT || (s && prec != UCP_FP64)) {
    I.gts = gt_stride(I);
    if (I.gts) {
      // centres from nw64 nodes before the grid to nw64 past it: every
      // position with a grid node in its window is within half a stride of
      // one
      I.gto = (I.nw64 + I.gts - 1) / I.gts * I.gts;
      I.gtr = (I.n_y - 1 + 2 * I.gto + I.gts - 1) / I.gts + 1;
    }
  }
  // window segments: enough work units to fill the GPU when the instance is
  // small, segments of at least 256 nodes
  if (prec == UCP_FP64 || prec == UCP_FP64_GT) {
    I.segs = 1;
    I.wsegs = 1;
  } else {
    const int tiles = (I.n_x + kMcBlock - 1) / kMcBlock;
    const int kq = I.cands + 1;
    const int wlen = 2 * I.nw32 + 1;
    const int wpb = kMcBlock / 64;  // waves per work unit
    int want = (16384 + tiles * kq * wpb - 1) / (tiles * kq * wpb);  // about 16384 waves per launch
    int cap = std::max(1, wlen / 256);
    int sg = 1;
    while (sg < want && sg < 16) sg <<= 1;
    sg = std::max(1, std::min(sg, cap));
    I.wsegs = std::max(sg, (wlen + kMcSegMax - 1) / kMcSegMax);
    // an instance that needs four or more segments to fill the chip is small
    // enough for the end of each launch to matter: the last segment it
    // dispatches is split in two, so the launch ends on half-length units
    I.segs = I.wsegs >= 4 ? I.wsegs + 1 : I.wsegs;
  }
  // at most 32 slices (the combine kernel's lane groups take 32)
  const int slen = std::max(512, (I.n_x + 31) / 32);
  I.u1_slices = (I.n_x + slen - 1) / slen;
  // several y nodes per lane where the grid is large enough to fill the
  // chip with a quarter of the lanes and fine enough that the weight ratio
  // between neighbouring nodes stays moderate
  I.u1_npl = I.n_y >= kU1NplMinNodes && I.dy <= kU1NplMaxStep * I.sw ? kU1Npl : 1;
  return I;
}

static size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

size_t state_bytes(const Inst& I) {
  size_t nx = (size_t)I.n_x, ny = (size_t)I.n_y;
  size_t b = 0;
  b += 9 * align_up(nx * 8);                                      // u0 u0_next f logf cbest b32best b64best b32inc jrow
  b += align_up(ny * 8) + align_up(ny * 4);                       // u1 v
  b += align_up((size_t)(2 * I.nw32 + 1 + kGtabPad) * 4);          // gtab (padded past the window)
  b += align_up(part_doubles(I) * 8);                             // part
  b += align_up((size_t)I.u1_slices * ny * 3 * 8);                // u1part
  b += align_up(u1stat_doubles(I) * 8);                           // u1stat
  if (I.gts) b += align_up((size_t)I.gtr * 3 * (kGtN + 1) * 8);   // gt
  b += 256 + kCountBytes;                                         // flags, counters
  return b;
}

void carve_state(Inst& I, char*& base) {
  size_t nx = (size_t)I.n_x, ny = (size_t)I.n_y;
  auto take = [&](size_t bytes) {
    char* p = base;
    base += align_up(bytes);
    return p;
  };
  I.u0 = (double*)take(nx * 8);
  I.u0_next = (double*)take(nx * 8);
  I.f = (double*)take(nx * 8);
  I.logf = (double*)take(nx * 8);
  I.cbest = (double*)take(nx * 8);
  I.b32best = (double*)take(nx * 8);
  I.b64best = (double*)take(nx * 8);
  I.b32inc = (double*)take(nx * 8);
  I.jrow = (double*)take(nx * 8);
  I.u1 = (double*)take(ny * 8);
  I.v = (float*)take(ny * 4);
  I.gtab = (float*)take((size_t)(2 * I.nw32 + 1 + kGtabPad) * 4);
  I.part = (double*)take(part_doubles(I) * 8);
  I.u1part = (double*)take((size_t)I.u1_slices * ny * 3 * 8);
  I.u1stat = (double*)take(u1stat_doubles(I) * 8);
  I.gt = I.gts ? (double*)take((size_t)I.gtr * 3 * (kGtN + 1) * 8) : nullptr;
  I.flags = (int32_t*)take(256);
  I.terms = (unsigned long long*)take(kCountBytes);
}

// Zero what a solve expects zero: flags and work counters.
hipError_t clear_state(const Inst& I, hipStream_t st) {
  hipError_t e = hipMemsetAsync(I.flags, 0, 256, st);
  if (e == hipSuccess && I.terms) e = hipMemsetAsync(I.terms, 0, kCountBytes, st);
  return e;
}

// Prefix sums of units for each kernel over a batch, for one set of running
// instances.  Layout: kinds x (n + 1).
std::vector<int32_t> build_tables(const std::vector<Inst>& insts, const std::vector<char>& running) {
  const int n = (int)insts.size();
  std::vector<int32_t> t((size_t)kKinds * (n + 1), 0);
  for (int k = 0; k < kKinds; ++k) {
    int32_t* pre = &t[(size_t)k * (n + 1)];
    pre[0] = 0;
    for (int b = 0; b < n; ++b) {
      const Inst& I = insts[b];
      int32_t u = 0;
      if (running[b]) {
        if (k < kKindSel0) u = I.free_cands ? 0 : units_mc(I, k - kKindMc0);
        else if (k < kKindU1p) u = (k - kKindSel0) < I.levels && !table_select(I) ? units_select(I) : 0;
        else if (k == kKindU1p) u = units_u1_partial(I);
        else if (k == kKindU1c) u = units_u1_combine(I);
        else if (k == kKindJRows) u = units_j_rows(I);
        else if (k == kKindJRed) u = 1;
        else if (k == kKindPrior) u = units_prior(I);
        else if (k == kKindCopy) u = units_prior(I);
        else if (k == kKindFree) u = I.free_cands ? units_mc(I, -1) : 0;
        else if (k == kKindFin) u = I.free_cands ? (int32_t)(((int64_t)I.n_x * I.cands + 255) / 256) : 0;
        else if (k == kKindGtab) u = units_gtab(I);
        else if (k == kKindGt) u = units_gt(I);
        else if (k == kKindU1s) u = units_u1_stats(I);
        else if (k >= kKindSelT0) u = (k - kKindSelT0) < I.levels && table_select(I) ? units_select(I) : 0;
      }
      pre[b + 1] = pre[b] + u;
    }
  }
  return t;
}

}  // namespace ucp

using namespace ucp;

struct ucp_handle {
  int device = 0;
  size_t budget = 0;  // workspace limit in bytes (0: none)
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // kernel timing with HIP events on the caller's stream (ucp_profile)
  int prof = 0;                 // bit k: time launches of kind k
  std::vector<hipEvent_t> ev;   // pool of event pairs
  std::vector<int> ev_kind;     // kind of each recorded pair
  size_t ev_used = 0;           // pairs recorded since the last harvest
  double prof_ms[UCP_PROF_KINDS] = {0};
  int64_t prof_n[UCP_PROF_KINDS] = {0};
  unsigned long long last_terms = 0;  // algorithmic terms of the last solve
  unsigned long long last_evals = 0;  // FP64 tie re-evaluations of the last solve
  unsigned long long last_evaluated = 0;  // marginal-cost terms the kernels evaluated
  // Pinned host staging of the instance and launch tables, a ring of
  // kStageSlots regions: a call writes its tables into the next region and
  // records an event after the copies, which the call that reuses the region
  // waits for.  The caller's host memory is never a copy source.
  static constexpr int kStageSlots = 4;
  char* stage[kStageSlots] = {nullptr};
  size_t stage_cap[kStageSlots] = {0};
  hipEvent_t stage_ev[kStageSlots] = {nullptr};
  int stage_next = 0;
};

// Copy host parts to the device through the handle's next staging region,
// asynchronously on `st`.
struct HostPart {
  void* dst;
  const void* src;
  size_t bytes;
};
static int stage_upload(ucp_handle* h, const std::vector<HostPart>& parts, hipStream_t st) {
  const int k = h->stage_next;
  h->stage_next = (k + 1) % ucp_handle::kStageSlots;
  size_t total = 0;
  for (const HostPart& p : parts) total += align_up(p.bytes);
  hipError_t e;
  if (h->stage_ev[k]) {
    e = hipEventSynchronize(h->stage_ev[k]);  // the region's previous copies have been read
    if (e != hipSuccess) return hip_fail(e, "wait for the staging region");
  } else {
    e = hipEventCreateWithFlags(&h->stage_ev[k], hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "create staging event");
  }
  if (total > h->stage_cap[k]) {
    if (h->stage[k]) (void)hipHostFree(h->stage[k]);
    h->stage[k] = nullptr;
    h->stage_cap[k] = 0;
    e = hipHostMalloc((void**)&h->stage[k], 2 * total, hipHostMallocDefault);
    if (e != hipSuccess) return fail(UCP_ENOMEM, "pinned staging of %zu bytes: %s", 2 * total, hipGetErrorString(e));
    h->stage_cap[k] = 2 * total;
  }
  char* at = h->stage[k];
  for (const HostPart& p : parts) {
    std::memcpy(at, p.src, p.bytes);
    e = hipMemcpyAsync(p.dst, at, p.bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "upload tables");
    at += align_up(p.bytes);
  }
  e = hipEventRecord(h->stage_ev[k], st);
  if (e != hipSuccess) return hip_fail(e, "record staging event");
  return UCP_OK;
}

static int ensure_ws(ucp_handle* h, size_t bytes) {
  if (bytes <= h->ws_bytes) return UCP_OK;
  if (h->budget && bytes > h->budget)
    return fail(UCP_ENOMEM, "workspace of %zu bytes exceeds the handle's budget of %zu", bytes, h->budget);
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  if (h->ws) {
    (void)hipDeviceSynchronize();
    (void)hipFree(h->ws);
    h->ws = nullptr;
    h->ws_bytes = 0;
  }
  size_t want = align_up(bytes + bytes / 8);
  if (h->budget) want = std::max(bytes, std::min(want, h->budget));
  e = hipMalloc(&h->ws, want);
  if (e != hipSuccess) {
    h->ws = nullptr;
    return fail(UCP_ENOMEM, "workspace of %zu bytes: %s", want, hipGetErrorString(e));
  }
  h->ws_bytes = want;
  return UCP_OK;
}

// Event pair for one timed launch (range) of `kind`: both null unless that
// kind is being timed and the launch will run.  The launchers hand the
// events to hipExtLaunchKernel, which records them at the start of the first
// and the end of the last kernel without extra packets in the stream.
struct EvPair {
  hipEvent_t a = nullptr, b = nullptr;
};
static hipError_t prof_pair(ucp_handle* h, int kind, bool runs, EvPair& p) {
  p = EvPair();
  if (!h || !runs || !((h->prof >> kind) & 1)) return hipSuccess;
  if (h->ev_used * 2 + 2 > h->ev.size()) {
    for (int k = 0; k < 64; ++k) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      h->ev.push_back(e);
    }
  }
  if (h->ev_kind.size() <= h->ev_used) h->ev_kind.resize(h->ev_used + 1);
  h->ev_kind[h->ev_used] = kind;
  p.a = h->ev[h->ev_used * 2];
  p.b = h->ev[h->ev_used * 2 + 1];
  h->ev_used++;
  return hipSuccess;
}
// Accumulate the recorded pairs (the stream has been synchronised).
static void prof_harvest(ucp_handle* h) {
  if (!h || !h->prof) return;
  for (size_t p = 0; p < h->ev_used; ++p) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, h->ev[2 * p], h->ev[2 * p + 1]) == hipSuccess) {
      h->prof_ms[h->ev_kind[p]] += ms;
      h->prof_n[h->ev_kind[p]] += 1;
    }
  }
  h->ev_used = 0;
}

namespace ucp {
// Access to the handle for the entry points defined in other files.
int handle_device(ucp_handle* h) { return h->device; }
int handle_workspace(ucp_handle* h, size_t bytes, void** out) {
  int rc = ensure_ws(h, bytes);
  if (rc == UCP_OK) *out = h->ws;
  return rc;
}
hipError_t handle_events(ucp_handle* h, int kind, hipEvent_t* a, hipEvent_t* b) {
  EvPair p;
  hipError_t e = prof_pair(h, kind, true, p);
  *a = p.a;
  *b = p.b;
  return e;
}
bool handle_profiling(ucp_handle* h) { return h->prof != 0; }
void handle_harvest(ucp_handle* h) { prof_harvest(h); }
}  // namespace ucp

extern "C" {

int ucp_profile(ucp_handle* h, int enable) {
  if (!h) return fail(UCP_EINVAL, "NULL handle");
  if (enable & ~((1 << UCP_PROF_KINDS) - 1)) return fail(UCP_EINVAL, "profile mask has unknown kinds");
  h->prof = enable;
  h->ev_used = 0;
  for (int k = 0; k < UCP_PROF_KINDS; ++k) {
    h->prof_ms[k] = 0.0;
    h->prof_n[k] = 0;
  }
  return UCP_OK;
}

int ucp_profile_read(ucp_handle* h, int kind, double* total_ms, int64_t* launches) {
  if (!h || kind < 0 || kind >= UCP_PROF_KINDS) return fail(UCP_EINVAL, "bad handle or kind");
  if (total_ms) *total_ms = h->prof_ms[kind];
  if (launches) *launches = h->prof_n[kind];
  return UCP_OK;
}

int ucp_last_counts(ucp_handle* h, uint64_t* terms, uint64_t* evaluated, uint64_t* fp64_evals) {
  if (!h) return fail(UCP_EINVAL, "NULL handle");
  if (terms) *terms = h->last_terms;
  if (evaluated) *evaluated = h->last_evaluated;
  if (fp64_evals) *fp64_evals = h->last_evals;
  return UCP_OK;
}

const char* ucp_version(void) { return "ucp-mi355x 0.1 (gfx950)"; }

const char* ucp_last_error(void) { return g_err.c_str(); }

int ucp_create(ucp_handle** out, int device, size_t hbm_budget) {
  if (!out) return fail(UCP_EINVAL, "out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0) return fail(UCP_EHIP, "no HIP device available");
  if (device < 0 || device >= n) return fail(UCP_EINVAL, "device %d out of range (have %d)", device, n);
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  ucp_handle* h = new ucp_handle;
  h->device = device;
  h->budget = hbm_budget;
  *out = h;
  return UCP_OK;
}

void ucp_destroy(ucp_handle* h) {
  if (!h) return;
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  if (h->ws) (void)hipFree(h->ws);
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  for (int k = 0; k < ucp_handle::kStageSlots; ++k) {
    if (h->stage[k]) (void)hipHostFree(h->stage[k]);
    if (h->stage_ev[k]) (void)hipEventDestroy(h->stage_ev[k]);
  }
  delete h;
}

}  // extern "C"

namespace ucp {

// A batch laid out in the handle's workspace: instance table, launch tables
// and per-instance state.
struct Batch {
  std::vector<Inst> insts;
  Inst* d_insts = nullptr;
  int32_t* d_tables = nullptr;  // phases x kinds x (n + 1)
  int n = 0;
  Launch launch(int phase, int kind, const std::vector<int32_t>& host_tab) const {
    Launch L;
    L.insts = d_insts;
    L.n_inst = n;
    const size_t off = ((size_t)phase * kKinds + kind) * (n + 1);
    L.pre = d_tables + off;
    L.total = host_tab[off + n];
    return L;
  }
};

// Lays out the batch in the workspace, lets `fix` set each carved instance's
// call-specific fields (outputs, explicit inputs), and uploads the instance
// and launch tables.
template <typename Fix>
int setup_batch(ucp_handle* h, Batch& B, std::vector<Inst> insts, const std::vector<std::vector<char>>& phases,
                std::vector<int32_t>& host_tab, hipStream_t st, Fix fix, size_t extra = 0, char** extra_out = nullptr) {
  B.n = (int)insts.size();
  size_t bytes = align_up(sizeof(Inst) * B.n) + align_up(sizeof(int32_t) * phases.size() * kKinds * (B.n + 1));
  for (auto& I : insts) bytes += state_bytes(I);
  bytes += align_up(extra);
  int rc = ensure_ws(h, bytes);
  if (rc) return rc;
  char* base = (char*)h->ws;
  if (extra_out) *extra_out = base + bytes - align_up(extra);
  B.d_insts = (Inst*)base;
  base += align_up(sizeof(Inst) * B.n);
  B.d_tables = (int32_t*)base;
  base += align_up(sizeof(int32_t) * phases.size() * kKinds * (B.n + 1));
  for (int b = 0; b < B.n; ++b) {
    carve_state(insts[b], base);
    fix(b, insts[b]);
  }
  host_tab.clear();
  for (auto& run : phases) {
    std::vector<int32_t> t = build_tables(insts, run);
    host_tab.insert(host_tab.end(), t.begin(), t.end());
  }
  B.insts = std::move(insts);
  return stage_upload(h, {{B.d_insts, B.insts.data(), sizeof(Inst) * B.n},
                          {B.d_tables, host_tab.data(), sizeof(int32_t) * host_tab.size()}}, st);
}
int setup_batch(ucp_handle* h, Batch& B, std::vector<Inst> insts, const std::vector<std::vector<char>>& phases,
                std::vector<int32_t>& host_tab, hipStream_t st) {
  return setup_batch(h, B, std::move(insts), phases, host_tab, st, [](int, Inst&) {});
}

#define UCP_TRY(expr, what)                      \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// One round for the running instances of `phase`: the u0 update over all
// levels, the u0 advance, the u1 update and the objective into J[t].
int run_round(ucp_handle* h, const Batch& B, int phase, const std::vector<int32_t>& tab, int prec, int max_levels,
              int t, hipStream_t st) {
  EvPair p;
  // the levels read the moment table of the current u1, built after the
  // u1 update that produced it (previous round, or the set-up)
  for (int l = 0; l < max_levels; ++l) {
    const Launch Lm = B.launch(phase, kKindMc0 + l, tab), Ls = B.launch(phase, kKindSel0 + l, tab),
                 Lt = B.launch(phase, kKindSelT0 + l, tab);
    UCP_TRY(prof_pair(h, UCP_PROF_MC, Lm.total > 0, p), "event");
    UCP_TRY(launch_mc(Lm, l, prec, st, p.a, p.b), "marginal-cost kernel");
    UCP_TRY(prof_pair(h, UCP_PROF_SELECT, Ls.total > 0 || Lt.total > 0, p), "event");
    UCP_TRY(launch_select(Ls, Lt, l, prec, 0, st, p.a, p.b), "selection kernel");
  }
  UCP_TRY(launch_copy_u0(B.launch(phase, kKindCopy, tab), st), "u0 advance kernel");
  const Launch Lp = B.launch(phase, kKindU1p, tab), Lc = B.launch(phase, kKindU1c, tab);
  UCP_TRY(prof_pair(h, UCP_PROF_U1, Lp.total > 0 && Lc.total > 0, p), "event");
  UCP_TRY(launch_u1_partial(B.launch(phase, kKindU1s, tab), Lp, prec, st, p.a), "u1 kernel");
  UCP_TRY(launch_u1_combine(Lc, st, p.b), "u1 combine kernel");
  UCP_TRY(launch_gt_table(B.launch(phase, kKindGt, tab), st), "moment table kernel");
  const Launch Lr = B.launch(phase, kKindJRows, tab), Ld = B.launch(phase, kKindJRed, tab);
  UCP_TRY(prof_pair(h, UCP_PROF_J, Lr.total > 0 && Ld.total > 0, p), "event");
  UCP_TRY(launch_j_rows(Lr, st, p.a), "objective kernel");
  UCP_TRY(launch_j_reduce_t(Ld, t, st, p.b), "objective reduce kernel");
  return UCP_OK;
}

// u1 and J[0] from the initial u0 (after the prior).
int run_init(ucp_handle* h, const Batch& B, int phase, const std::vector<int32_t>& tab, int prec, hipStream_t st) {
  EvPair p;
  UCP_TRY(launch_prior(B.launch(phase, kKindPrior, tab), st), "prior kernel");
  UCP_TRY(launch_gtab(B.launch(phase, kKindGtab, tab), st), "offset table kernel");
  const Launch Lp = B.launch(phase, kKindU1p, tab), Lc = B.launch(phase, kKindU1c, tab);
  UCP_TRY(prof_pair(h, UCP_PROF_U1, Lp.total > 0 && Lc.total > 0, p), "event");
  UCP_TRY(launch_u1_partial(B.launch(phase, kKindU1s, tab), Lp, prec, st, p.a), "u1 kernel");
  UCP_TRY(launch_u1_combine(Lc, st, p.b), "u1 combine kernel");
  UCP_TRY(launch_gt_table(B.launch(phase, kKindGt, tab), st), "moment table kernel");
  const Launch Lr = B.launch(phase, kKindJRows, tab), Ld = B.launch(phase, kKindJRed, tab);
  UCP_TRY(prof_pair(h, UCP_PROF_J, Lr.total > 0 && Ld.total > 0, p), "event");
  UCP_TRY(launch_j_rows(Lr, st, p.a), "objective kernel");
  UCP_TRY(launch_j_reduce_t(Ld, 0, st, p.b), "objective reduce kernel");
  return UCP_OK;
}

}  // namespace ucp

extern "C" {

int ucp_solve_batch(ucp_handle* h, int32_t nb, const ucp_problem* probs, const ucp_search* searches,
                    ucp_prec prec, const int32_t* iters, const double* const* u0_init,
                    double* const* u0_out, double* const* u1_out, double* const* J_hist, void* stream) {
  if (!h) return fail(UCP_EINVAL, "handle is NULL");
  if (nb < 1) return fail(UCP_EINVAL, "batch size must be >= 1");
  if (!probs || !searches || !iters || !u0_init || !u0_out || !u1_out || !J_hist)
    return fail(UCP_EINVAL, "NULL array argument");
  int rc = check_prec(prec);
  if (rc) return rc;
  int max_it = 0, max_lv = 0;
  for (int b = 0; b < nb; ++b) {
    if ((rc = check_problem(&probs[b]))) return fail(rc, "instance %d: %s", b, g_err.c_str());
    if ((rc = check_search(&searches[b]))) return fail(rc, "instance %d: %s", b, g_err.c_str());
    if (iters[b] < 0) return fail(UCP_EINVAL, "instance %d: iters < 0", b);
    if (!u0_init[b] || !u0_out[b] || !u1_out[b] || !J_hist[b]) return fail(UCP_EINVAL, "instance %d: NULL pointer", b);
    max_it = std::max(max_it, (int)iters[b]);
    max_lv = std::max(max_lv, (int)searches[b].levels);
  }
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  std::vector<Inst> insts;
  for (int b = 0; b < nb; ++b) {
    insts.push_back(make_inst(probs[b], &searches[b], prec, 0));
    if ((rc = check_gt(insts.back()))) return fail(rc, "instance %d: %s", b, g_err.c_str());
  }
  // phases: phase t (0..max_it) runs the instances with iters >= t
  std::vector<std::vector<char>> phases(max_it + 1, std::vector<char>(nb, 0));
  std::vector<int> phase_of(max_it + 1, 0);
  for (int t = 0; t <= max_it; ++t)
    for (int b = 0; b < nb; ++b) phases[t][b] = iters[b] >= t;
  Batch B;
  std::vector<int32_t> tab;
  // J_out of each instance is its J_hist
  if ((rc = setup_batch(h, B, insts, phases, tab, st, [&](int b, Inst& I) { I.J_out = J_hist[b]; }))) return rc;
  for (int b = 0; b < nb; ++b) {
    Inst& I = B.insts[b];
    UCP_TRY(hipMemcpyAsync(I.u0, u0_init[b], sizeof(double) * I.n_x, hipMemcpyDeviceToDevice, st), "copy u0_init");
    UCP_TRY(clear_state(I, st), "clear state");
  }
  if ((rc = run_init(h, B, 0, tab, prec, st))) return rc;
  for (int t = 1; t <= max_it; ++t)
    if ((rc = run_round(h, B, t, tab, prec, max_lv, t, st))) return rc;
  std::vector<int32_t> flags(nb, 0);
  std::vector<unsigned long long> counts((size_t)nb * kCountSlots * kCountStride, 0);
  for (int b = 0; b < nb; ++b) {
    Inst& I = B.insts[b];
    UCP_TRY(hipMemcpyAsync(&counts[(size_t)b * kCountSlots * kCountStride], I.terms, kCountBytes, hipMemcpyDeviceToHost, st),
            "read counters");
    UCP_TRY(hipMemcpyAsync(u0_out[b], I.u0, sizeof(double) * I.n_x, hipMemcpyDeviceToDevice, st), "copy u0_out");
    UCP_TRY(hipMemcpyAsync(u1_out[b], I.u1, sizeof(double) * I.n_y, hipMemcpyDeviceToDevice, st), "copy u1_out");
    UCP_TRY(hipMemcpyAsync(&flags[b], I.flags, 4, hipMemcpyDeviceToHost, st), "read flags");
  }
  UCP_TRY(hipStreamSynchronize(st), "synchronise");
  prof_harvest(h);
  h->last_terms = h->last_evals = h->last_evaluated = 0;
  for (int b = 0; b < nb; ++b)
    for (int sl = 0; sl < kCountSlots; ++sl) {
      h->last_terms += counts[((size_t)b * kCountSlots + sl) * kCountStride + kCountTerms];
      h->last_evaluated += counts[((size_t)b * kCountSlots + sl) * kCountStride + kCountEvalTerms];
      h->last_evals += counts[((size_t)b * kCountSlots + sl) * kCountStride + kCountEvals];
    }
  for (int b = 0; b < nb; ++b)
    if (flags[b]) return fail(UCP_ENONFINITE, "instance %d produced non-finite values", b);
  return UCP_OK;
}

int ucp_solve(ucp_handle* h, const ucp_problem* prob, const ucp_search* search, ucp_prec prec, int32_t iters,
              const double* u0_init, double* u0_out, double* u1_out, double* J_hist, void* stream) {
  if (!prob || !search) return fail(UCP_EINVAL, "NULL problem or search");
  return ucp_solve_batch(h, 1, prob, search, prec, &iters, &u0_init, &u0_out, &u1_out, &J_hist, stream);
}

int ucp_argmin_adaptive(ucp_handle* h, const ucp_problem* prob, const ucp_search* search, ucp_prec prec,
                        const double* u1, const double* u0_in, double* u0_out, double* L0_out, void* stream) {
  if (!h) return fail(UCP_EINVAL, "handle is NULL");
  int rc;
  if ((rc = check_problem(prob)) || (rc = check_search(search)) || (rc = check_prec(prec))) return rc;
  if (!u1 || !u0_in || !u0_out) return fail(UCP_EINVAL, "NULL array argument");
  UCP_TRY(hipSetDevice(h->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  std::vector<std::vector<char>> phases(1, std::vector<char>(1, 1));
  Batch B;
  std::vector<int32_t> tab;
  auto fix = [&](int, Inst& I) {
    I.L0_out = L0_out;
    I.terms = nullptr;
  };
  const Inst I0 = make_inst(*prob, search, prec, 0);
  if ((rc = check_gt(I0))) return rc;
  if ((rc = setup_batch(h, B, {I0}, phases, tab, st, fix))) return rc;
  Inst& I = B.insts[0];
  UCP_TRY(hipMemcpyAsync(I.u0, u0_in, sizeof(double) * I.n_x, hipMemcpyDeviceToDevice, st), "copy u0");
  UCP_TRY(hipMemcpyAsync(I.u1, u1, sizeof(double) * I.n_y, hipMemcpyDeviceToDevice, st), "copy u1");
  UCP_TRY(clear_state(I, st), "clear state");
  UCP_TRY(launch_prior(B.launch(0, kKindPrior, tab), st), "prior kernel");
  UCP_TRY(launch_gtab(B.launch(0, kKindGtab, tab), st), "offset table kernel");
  UCP_TRY(launch_v_from_u1(B.launch(0, kKindU1c, tab), st), "residual kernel");
  UCP_TRY(launch_gt_table(B.launch(0, kKindGt, tab), st), "moment table kernel");
  for (int l = 0; l < I.levels; ++l) {
    UCP_TRY(launch_mc(B.launch(0, kKindMc0 + l, tab), l, prec, st), "marginal-cost kernel");
    UCP_TRY(launch_select(B.launch(0, kKindSel0 + l, tab), B.launch(0, kKindSelT0 + l, tab), l, prec,
                          L0_out != nullptr, st),
            "selection kernel");
  }
  UCP_TRY(hipMemcpyAsync(u0_out, I.u0_next, sizeof(double) * I.n_x, hipMemcpyDeviceToDevice, st), "copy u0_out");
  return UCP_OK;
}

int ucp_update_u1(ucp_handle* h, const ucp_problem* prob, ucp_prec prec, const double* u0, double* u1_out,
                  void* stream) {
  if (!h) return fail(UCP_EINVAL, "handle is NULL");
  int rc;
  if ((rc = check_problem(prob)) || (rc = check_prec(prec))) return rc;
  if (!u0 || !u1_out) return fail(UCP_EINVAL, "NULL array argument");
  UCP_TRY(hipSetDevice(h->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  std::vector<std::vector<char>> phases(1, std::vector<char>(1, 1));
  Batch B;
  std::vector<int32_t> tab;
  if ((rc = setup_batch(h, B, {make_inst(*prob, nullptr, prec, 1)}, phases, tab, st))) return rc;
  Inst& I = B.insts[0];
  UCP_TRY(hipMemcpyAsync(I.u0, u0, sizeof(double) * I.n_x, hipMemcpyDeviceToDevice, st), "copy u0");
  UCP_TRY(hipMemsetAsync(I.flags, 0, 128, st), "clear flags");
  UCP_TRY(launch_prior(B.launch(0, kKindPrior, tab), st), "prior kernel");
  UCP_TRY(launch_gtab(B.launch(0, kKindGtab, tab), st), "offset table kernel");
  UCP_TRY(launch_u1_partial(B.launch(0, kKindU1s, tab), B.launch(0, kKindU1p, tab), prec, st), "u1 kernel");
  UCP_TRY(launch_u1_combine(B.launch(0, kKindU1c, tab), st), "u1 combine kernel");
  UCP_TRY(hipMemcpyAsync(u1_out, I.u1, sizeof(double) * I.n_y, hipMemcpyDeviceToDevice, st), "copy u1_out");
  return UCP_OK;
}

int ucp_objective(ucp_handle* h, const ucp_problem* prob, const double* u0, const double* u1, double* J_out,
                  void* stream) {
  if (!h) return fail(UCP_EINVAL, "handle is NULL");
  int rc;
  if ((rc = check_problem(prob))) return rc;
  if (!u0 || !u1 || !J_out) return fail(UCP_EINVAL, "NULL array argument");
  UCP_TRY(hipSetDevice(h->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  std::vector<std::vector<char>> phases(1, std::vector<char>(1, 1));
  Batch B;
  std::vector<int32_t> tab;
  auto fix = [&](int, Inst& I) {
    I.J_out = J_out;
    I.terms = nullptr;
  };
  if ((rc = setup_batch(h, B, {make_inst(*prob, nullptr, UCP_FP64, 1)}, phases, tab, st, fix))) return rc;
  Inst& I = B.insts[0];
  UCP_TRY(hipMemcpyAsync(I.u0, u0, sizeof(double) * I.n_x, hipMemcpyDeviceToDevice, st), "copy u0");
  UCP_TRY(hipMemcpyAsync(I.u1, u1, sizeof(double) * I.n_y, hipMemcpyDeviceToDevice, st), "copy u1");
  UCP_TRY(hipMemsetAsync(I.flags, 0, 128, st), "clear flags");
  UCP_TRY(launch_prior(B.launch(0, kKindPrior, tab), st), "prior kernel");
  UCP_TRY(launch_gtab(B.launch(0, kKindGtab, tab), st), "offset table kernel");
  UCP_TRY(launch_j_rows(B.launch(0, kKindJRows, tab), st), "objective kernel");
  UCP_TRY(launch_j_reduce_t(B.launch(0, kKindJRed, tab), 0, st), "objective reduce kernel");
  return UCP_OK;
}

int ucp_marginal_cost(ucp_handle* h, const ucp_problem* prob, ucp_prec prec, const double* u1, const double* u,
                      int64_t n_cand, double* L0_out, void* stream) {
  if (!h) return fail(UCP_EINVAL, "handle is NULL");
  int rc;
  if ((rc = check_problem(prob)) || (rc = check_prec(prec))) return rc;
  if (!u1 || !u || !L0_out) return fail(UCP_EINVAL, "NULL array argument");
  if (n_cand < 1 || n_cand > 4096) return fail(UCP_EINVAL, "n_cand must be 1..4096");
  if ((int64_t)prob->n_x * n_cand > ((int64_t)1 << 30)) return fail(UCP_EINVAL, "n_x * n_cand too large");
  UCP_TRY(hipSetDevice(h->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  std::vector<std::vector<char>> phases(1, std::vector<char>(1, 1));
  Batch B;
  std::vector<int32_t> tab;
  Inst I0 = make_inst(*prob, nullptr, prec, (int)n_cand);
  I0.free_cands = 1;
  if ((rc = check_gt(I0))) return rc;
  auto fix = [&](int, Inst& I) {
    I.u0 = const_cast<double*>(u);  // the explicit candidates [n_x][n_cand], read only
    I.terms = nullptr;
  };
  if ((rc = setup_batch(h, B, {I0}, phases, tab, st, fix))) return rc;
  Inst& I = B.insts[0];
  UCP_TRY(hipMemcpyAsync(I.u1, u1, sizeof(double) * I.n_y, hipMemcpyDeviceToDevice, st), "copy u1");
  UCP_TRY(launch_prior(B.launch(0, kKindPrior, tab), st), "prior kernel");
  UCP_TRY(launch_gtab(B.launch(0, kKindGtab, tab), st), "offset table kernel");
  UCP_TRY(launch_v_from_u1(B.launch(0, kKindU1c, tab), st), "residual kernel");
  UCP_TRY(launch_gt_table(B.launch(0, kKindGt, tab), st), "moment table kernel");
  UCP_TRY(launch_mc(B.launch(0, kKindFree, tab), -1, prec, st), "marginal-cost kernel");
  Launch Lf = B.launch(0, kKindFin, tab);
  UCP_TRY(launch_finish_free(Lf, L0_out, prec, st), "finish kernel");
  return UCP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// The paper's generic solver (Algorithm 1): local updates and partial
// exhaustion for both controllers, adaptive allocation, precision stop.

namespace ucp {

static int check_alg1(const ucp_alg1_params* a) {
  if (!a) return fail(UCP_EINVAL, "params is NULL");
  if (a->N < 2 || a->N > 1000000) return fail(UCP_EINVAL, "N must be 2..1e6");
  if (a->r != 1 && a->r != 2) return fail(UCP_EINVAL, "the partial-exhaustion radius r must be 1 or 2");
  if (!(a->p >= 0.0) || !std::isfinite(a->p)) return fail(UCP_EINVAL, "p must be finite and >= 0");
  if (!(a->tau > 0.0) || !std::isfinite(a->tau)) return fail(UCP_EINVAL, "tau must be finite and > 0");
  if (!(a->tie_rel64 >= 0.0 && a->tie_rel64 <= 1e-3)) return fail(UCP_EINVAL, "tie_rel64 must be in [0, 1e-3]");
  if (a->max_rounds < 1 || a->max_rounds > 1000000) return fail(UCP_EINVAL, "max_rounds must be 1..1e6");
  return UCP_OK;
}

static double alg1_tie(double t) { return t > 0.0 ? t : kTau64; }

// Partial sums of the u1 partial exhaustion: [slices][n_y][2 r + 2].
static size_t pe_u1_bytes(const Inst& I, int r) { return (size_t)I.u1_slices * I.n_y * (2 * r + 2) * 8; }

}  // namespace ucp

extern "C" {

int ucp_alg1_local_u0(ucp_handle* h, const ucp_problem* prob, double tau, const double* u1, const double* u0_in,
                      double* u0_out, void* stream) {
  if (!h) return fail(UCP_EINVAL, "handle is NULL");
  int rc;
  if ((rc = check_problem(prob))) return rc;
  if (!(tau > 0.0) || !std::isfinite(tau)) return fail(UCP_EINVAL, "tau must be finite and > 0");
  if (!u1 || !u0_in || !u0_out) return fail(UCP_EINVAL, "NULL array argument");
  UCP_TRY(hipSetDevice(h->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  std::vector<std::vector<char>> phases(1, std::vector<char>(1, 1));
  Batch B;
  std::vector<int32_t> tab;
  auto fix = [&](int, Inst& I) {
    I.u1 = const_cast<double*>(u1);  // read only
    I.terms = nullptr;
  };
  if ((rc = setup_batch(h, B, {make_inst(*prob, nullptr, UCP_FP64, 1)}, phases, tab, st, fix))) return rc;
  Inst& I = B.insts[0];
  UCP_TRY(clear_state(I, st), "clear state");
  UCP_TRY(launch_a1_local_u0(B.d_insts, I.n_x, tau, u0_in, I.u0_next, st), "local-update kernel");
  UCP_TRY(hipMemcpyAsync(u0_out, I.u0_next, sizeof(double) * I.n_x, hipMemcpyDeviceToDevice, st), "copy u0_out");
  return UCP_OK;
}

int ucp_alg1_pe_u0(ucp_handle* h, const ucp_problem* prob, double tie_rel64, int32_t r, const double* u1,
                   const double* u0_in, double* u0_out, void* stream) {
  if (!h) return fail(UCP_EINVAL, "handle is NULL");
  int rc;
  if ((rc = check_problem(prob))) return rc;
  if (r != 1 && r != 2) return fail(UCP_EINVAL, "r must be 1 or 2");
  if (!(tie_rel64 >= 0.0 && tie_rel64 <= 1e-3)) return fail(UCP_EINVAL, "tie_rel64 must be in [0, 1e-3]");
  if (!u1 || !u0_in || !u0_out) return fail(UCP_EINVAL, "NULL array argument");
  UCP_TRY(hipSetDevice(h->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  std::vector<std::vector<char>> phases(1, std::vector<char>(1, 1));
  Batch B;
  std::vector<int32_t> tab;
  auto fix = [&](int, Inst& I) {
    I.u1 = const_cast<double*>(u1);  // read only
    I.terms = nullptr;
  };
  if ((rc = setup_batch(h, B, {make_inst(*prob, nullptr, UCP_FP64, 1)}, phases, tab, st, fix))) return rc;
  Inst& I = B.insts[0];
  UCP_TRY(clear_state(I, st), "clear state");
  UCP_TRY(launch_a1_pe_u0(B.d_insts, I.n_x, r, alg1_tie(tie_rel64), u0_in, I.u0_next, st), "exhaustion kernel");
  UCP_TRY(hipMemcpyAsync(u0_out, I.u0_next, sizeof(double) * I.n_x, hipMemcpyDeviceToDevice, st), "copy u0_out");
  return UCP_OK;
}

int ucp_alg1_pe_u1(ucp_handle* h, const ucp_problem* prob, double tie_rel64, int32_t r, const double* u0,
                   const double* u1_in, double* u1_out, void* stream) {
  if (!h) return fail(UCP_EINVAL, "handle is NULL");
  int rc;
  if ((rc = check_problem(prob))) return rc;
  if (r != 1 && r != 2) return fail(UCP_EINVAL, "r must be 1 or 2");
  if (!(tie_rel64 >= 0.0 && tie_rel64 <= 1e-3)) return fail(UCP_EINVAL, "tie_rel64 must be in [0, 1e-3]");
  if (!u0 || !u1_in || !u1_out) return fail(UCP_EINVAL, "NULL array argument");
  UCP_TRY(hipSetDevice(h->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  std::vector<std::vector<char>> phases(1, std::vector<char>(1, 1));
  Batch B;
  std::vector<int32_t> tab;
  auto fix = [&](int, Inst& I) {
    I.u0 = const_cast<double*>(u0);  // read only
    I.terms = nullptr;
  };
  Inst I0 = make_inst(*prob, nullptr, UCP_FP64, 1);
  char* part = nullptr;
  if ((rc = setup_batch(h, B, {I0}, phases, tab, st, fix, pe_u1_bytes(I0, r), &part))) return rc;
  Inst& I = B.insts[0];
  UCP_TRY(clear_state(I, st), "clear state");
  UCP_TRY(launch_prior(B.launch(0, kKindPrior, tab), st), "prior kernel");
  UCP_TRY(launch_a1_pe_u1(I, B.d_insts, r, alg1_tie(tie_rel64), u1_in, (double*)part, I.u1, st), "exhaustion kernels");
  UCP_TRY(hipMemcpyAsync(u1_out, I.u1, sizeof(double) * I.n_y, hipMemcpyDeviceToDevice, st), "copy u1_out");
  return UCP_OK;
}

int ucp_alg1_solve(ucp_handle* h, const ucp_problem* prob, const ucp_alg1_params* a, const double* u0_init,
                   const double* u1_init, double* u0_out, double* u1_out, double* J_log, int32_t* NL_log,
                   int32_t* rounds_out, void* stream) {
  if (!h) return fail(UCP_EINVAL, "handle is NULL");
  int rc;
  if ((rc = check_problem(prob)) || (rc = check_alg1(a))) return rc;
  if (!u0_init || !u1_init || !u0_out || !u1_out || !J_log || !rounds_out) return fail(UCP_EINVAL, "NULL argument");
  UCP_TRY(hipSetDevice(h->device), "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  std::vector<std::vector<char>> phases(1, std::vector<char>(1, 1));
  Batch B;
  std::vector<int32_t> tab;
  Inst I0 = make_inst(*prob, nullptr, UCP_FP64, 1);
  const size_t part_bytes = pe_u1_bytes(I0, a->r);
  auto fix = [&](int, Inst& I) {
    I.J_out = J_log;
    I.terms = nullptr;
  };
  char* extra = nullptr;
  if ((rc = setup_batch(h, B, {I0}, phases, tab, st, fix, part_bytes + (size_t)I0.n_y * 8 + 256, &extra))) return rc;
  Inst& I = B.insts[0];
  double* part = (double*)extra;
  double* u1t = (double*)(extra + ((part_bytes + 255) & ~(size_t)255));
  const double tie = alg1_tie(a->tie_rel64);
  const Inst* dI = B.d_insts;
  UCP_TRY(hipMemcpyAsync(I.u0, u0_init, sizeof(double) * I.n_x, hipMemcpyDeviceToDevice, st), "copy u0_init");
  UCP_TRY(hipMemcpyAsync(I.u1, u1_init, sizeof(double) * I.n_y, hipMemcpyDeviceToDevice, st), "copy u1_init");
  UCP_TRY(clear_state(I, st), "clear state");
  UCP_TRY(launch_prior(B.launch(0, kKindPrior, tab), st), "prior kernel");
  // J into J_log[t], read back for the adaptive allocation
  auto objective = [&](int t, double* Jh) -> int {
    UCP_TRY(launch_j_rows(B.launch(0, kKindJRows, tab), st), "objective kernel");
    UCP_TRY(launch_j_reduce_t(B.launch(0, kKindJRed, tab), t, st), "objective reduce kernel");
    UCP_TRY(hipMemcpyAsync(Jh, J_log + t, sizeof(double), hipMemcpyDeviceToHost, st), "read J");
    UCP_TRY(hipStreamSynchronize(st), "synchronise");
    return UCP_OK;
  };
  double Jc = 0.0;
  if ((rc = objective(0, &Jc))) return rc;
  double IL = a->p, IP = a->p;
  int32_t NL = a->N / 2, NP = a->N - NL;
  int32_t rounds = 0;
  while (IL + IP > a->p && rounds < a->max_rounds) {
    if (NL_log) NL_log[rounds] = NL;
    double Jprev = Jc;
    for (int32_t it = 0; it < NL; ++it) {
      UCP_TRY(launch_a1_local_u0(dI, I.n_x, a->tau, I.u0, I.u0_next, st), "local-update kernel");
      UCP_TRY(launch_copy_u0(B.launch(0, kKindCopy, tab), st), "u0 advance kernel");
      UCP_TRY(launch_u1_partial(B.launch(0, kKindU1s, tab), B.launch(0, kKindU1p, tab), UCP_FP64, st), "u1 kernel");
      UCP_TRY(launch_u1_combine(B.launch(0, kKindU1c, tab), st), "u1 combine kernel");
    }
    if ((rc = objective(1 + 2 * rounds, &Jc))) return rc;
    IL = std::fabs(Jprev - Jc);
    Jprev = Jc;
    for (int32_t it = 0; it < NP; ++it) {
      UCP_TRY(launch_a1_pe_u0(dI, I.n_x, a->r, tie, I.u0, I.u0_next, st), "exhaustion kernel");
      UCP_TRY(launch_copy_u0(B.launch(0, kKindCopy, tab), st), "u0 advance kernel");
      UCP_TRY(launch_a1_pe_u1(I, dI, a->r, tie, I.u1, part, u1t, st), "exhaustion kernels");
      UCP_TRY(hipMemcpyAsync(I.u1, u1t, sizeof(double) * I.n_y, hipMemcpyDeviceToDevice, st), "u1 advance");
    }
    if ((rc = objective(2 + 2 * rounds, &Jc))) return rc;
    IP = std::fabs(Jprev - Jc);
    if (IL + IP > 0.0) {
      int32_t v = (int32_t)std::floor(IL * (double)a->N / (IL + IP));
      NL = std::min(std::max(v, 1), a->N - 1);
    }
    NP = a->N - NL;
    ++rounds;
  }
  *rounds_out = rounds;
  int32_t flags = 0;
  UCP_TRY(hipMemcpyAsync(u0_out, I.u0, sizeof(double) * I.n_x, hipMemcpyDeviceToDevice, st), "copy u0_out");
  UCP_TRY(hipMemcpyAsync(u1_out, I.u1, sizeof(double) * I.n_y, hipMemcpyDeviceToDevice, st), "copy u1_out");
  UCP_TRY(hipMemcpyAsync(&flags, I.flags, 4, hipMemcpyDeviceToHost, st), "read flags");
  UCP_TRY(hipStreamSynchronize(st), "synchronise");
  if (flags) return fail(UCP_ENONFINITE, "the solve produced non-finite values");
  return UCP_OK;
}

}  // extern "C"
