// Continuous-batching server of the marginal-cost solver.
//
// Requests queue on the host.  Each ucp_server_step() admits queued
// requests in arrival order while a slot is free and their device footprint
// fits the memory budget, runs the first-round set-up (prior, u1 of the
// initial u0, J[0]) for the new ones, then one round (u0 update over all
// levels, u0 advance, u1 update, J) for every running request in shared
// launches - one flat work list per kernel over all running instances - and
// retires the requests that reached their iteration count (results copied
// to host).  Kernels depend only on each instance's own data, so a request's
// results are the same alone and in the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <vector>

#include "ucp_internal.h"
#include "ucp_runtime.h"

using namespace ucp;

namespace {

enum State { kQueued, kRunning, kDone, kCancelled };

struct Request {
  int64_t ticket = 0;
  ucp_problem prob;
  ucp_search search;
  int32_t iters = 0;
  std::vector<double> u0_init;
  State state = kQueued;
  int32_t t = 0;          // rounds done
  size_t bytes = 0;       // device footprint
  void* dmem = nullptr;   // device state block
  Inst inst;
  double* d_J = nullptr;  // device J history [iters + 1]
  bool fresh = false;     // admitted in this step: needs the set-up
  std::vector<double> u0_out, u1_out, J_hist;
  int32_t flags = 0;
};

size_t round_up(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

struct ucp_server {
  // device blocks of retired requests kept for reuse (size -> pointer);
  // they count against the memory budget
  std::multimap<size_t, void*> pool;
  size_t pooled = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  size_t budget = 0;  // 0 = unlimited
  int32_t max_slots = 1;
  int prec = UCP_FP32_KAHAN;
  size_t used = 0;
  int64_t next_ticket = 1;
  std::map<int64_t, Request*> reqs;
  std::deque<int64_t> queue;
  std::vector<Request*> running;
  // device launch tables
  Inst* d_insts = nullptr;
  int32_t* d_tab = nullptr;
  size_t cap_insts = 0, cap_tab = 0;
  // pinned host staging of the tables: a step ends by synchronising the
  // stream, so the next step may overwrite it
  char* h_stage = nullptr;
  size_t cap_stage = 0;
};

static size_t footprint(const Inst& I, int32_t iters) {
  return state_bytes(I) + round_up(sizeof(double) * (size_t)(iters + 1));
}

// Return a request's block to the pool (the stream has no work of it left).
static void release(ucp_server* s, Request* r) {
  if (r->dmem) {
    s->pool.emplace(r->bytes, r->dmem);
    s->pooled += r->bytes;
    r->dmem = nullptr;
    s->used -= r->bytes;
  }
}

static void drain_pool(ucp_server* s) {
  for (auto& kv : s->pool) (void)hipFree(kv.second);
  s->pool.clear();
  s->pooled = 0;
}

// A block of exactly `bytes` from the pool, or a new allocation; pooled
// blocks of other sizes are freed first when the budget needs the room.
static void* acquire(ucp_server* s, size_t bytes) {
  auto it = s->pool.find(bytes);
  if (it != s->pool.end()) {
    void* p = it->second;
    s->pool.erase(it);
    s->pooled -= bytes;
    return p;
  }
  if (s->budget && s->used + s->pooled + bytes > s->budget) drain_pool(s);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    drain_pool(s);
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  }
  return p;
}

extern "C" {

int ucp_footprint(const ucp_problem* prob, const ucp_search* search, ucp_prec prec, int32_t iters, size_t* bytes) {
  int rc;
  if (!bytes) return fail(UCP_EINVAL, "bytes is NULL");
  if ((rc = check_problem(prob)) || (rc = check_search(search)) || (rc = check_prec(prec))) return rc;
  if (iters < 0) return fail(UCP_EINVAL, "iters < 0");
  const Inst I = make_inst(*prob, search, prec, 0);
  if ((rc = check_gt(I))) return rc;
  *bytes = footprint(I, iters);
  return UCP_OK;
}

int ucp_server_create(ucp_server** out, int device, size_t hbm_budget, int32_t max_slots, ucp_prec prec) {
  if (!out) return fail(UCP_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_slots < 1 || max_slots > 4096) return fail(UCP_EINVAL, "max_slots must be 1..4096");
  int rc = check_prec(prec);
  if (rc) return rc;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return fail(UCP_EHIP, "no HIP device available");
  if (device < 0 || device >= n) return fail(UCP_EINVAL, "device %d out of range", device);
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  ucp_server* s = new ucp_server;
  s->device = device;
  s->budget = hbm_budget;
  s->max_slots = max_slots;
  s->prec = prec;
  e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "hipStreamCreate");
  }
  *out = s;
  return UCP_OK;
}

void ucp_server_destroy(ucp_server* s) {
  if (!s) return;
  (void)hipSetDevice(s->device);
  (void)hipStreamSynchronize(s->stream);
  for (auto& kv : s->reqs) {
    release(s, kv.second);
    delete kv.second;
  }
  drain_pool(s);
  if (s->d_insts) (void)hipFree(s->d_insts);
  if (s->d_tab) (void)hipFree(s->d_tab);
  if (s->h_stage) (void)hipHostFree(s->h_stage);
  (void)hipStreamDestroy(s->stream);
  delete s;
}

int ucp_server_submit(ucp_server* s, const ucp_problem* prob, const ucp_search* search, int32_t iters,
                      const double* u0_init, int64_t* ticket) {
  if (!s || !ticket || !u0_init) return fail(UCP_EINVAL, "NULL argument");
  int rc;
  if ((rc = check_problem(prob)) || (rc = check_search(search))) return rc;
  if (iters < 0) return fail(UCP_EINVAL, "iters < 0");
  Request* r = new Request;
  r->prob = *prob;
  r->search = *search;
  r->iters = iters;
  r->u0_init.assign(u0_init, u0_init + prob->n_x);
  r->inst = make_inst(*prob, search, s->prec, 0);
  if ((rc = check_gt(r->inst))) {
    delete r;
    return rc;
  }
  r->bytes = footprint(r->inst, iters);
  if (s->budget && r->bytes > s->budget) {
    delete r;
    return fail(UCP_ENOMEM, "request needs %zu bytes, over the budget of %zu", footprint(make_inst(*prob, search, s->prec, 0), iters), s->budget);
  }
  r->ticket = s->next_ticket++;
  s->reqs[r->ticket] = r;
  s->queue.push_back(r->ticket);
  *ticket = r->ticket;
  return UCP_OK;
}

int ucp_server_cancel(ucp_server* s, int64_t ticket) {
  if (!s) return fail(UCP_EINVAL, "NULL server");
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || it->second->state == kCancelled) return fail(UCP_ENOTFOUND, "unknown ticket %lld", (long long)ticket);
  Request* r = it->second;
  if (r->state == kQueued) s->queue.erase(std::find(s->queue.begin(), s->queue.end(), ticket));
  if (r->state == kRunning) {
    // between steps nothing of this request is in flight on the stream
    (void)hipStreamSynchronize(s->stream);
    s->running.erase(std::find(s->running.begin(), s->running.end(), r));
    release(s, r);
  }
  r->state = kCancelled;
  s->reqs.erase(it);
  delete r;
  return UCP_OK;
}

int ucp_server_stats(ucp_server* s, int32_t* queued, int32_t* running, int32_t* done) {
  if (!s) return fail(UCP_EINVAL, "NULL server");
  int32_t d = 0;
  for (auto& kv : s->reqs) d += kv.second->state == kDone;
  if (queued) *queued = (int32_t)s->queue.size();
  if (running) *running = (int32_t)s->running.size();
  if (done) *done = d;
  return UCP_OK;
}

int ucp_server_poll(ucp_server* s, int64_t ticket, double* u0_out, double* u1_out, double* J_hist) {
  if (!s) return fail(UCP_EINVAL, "NULL server");
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(UCP_ENOTFOUND, "unknown ticket %lld", (long long)ticket);
  Request* r = it->second;
  if (r->state != kDone) return fail(UCP_EAGAIN, "ticket %lld not finished", (long long)ticket);
  if (u0_out) std::memcpy(u0_out, r->u0_out.data(), sizeof(double) * r->u0_out.size());
  if (u1_out) std::memcpy(u1_out, r->u1_out.data(), sizeof(double) * r->u1_out.size());
  if (J_hist) std::memcpy(J_hist, r->J_hist.data(), sizeof(double) * r->J_hist.size());
  const int32_t flags = r->flags;
  s->reqs.erase(it);
  delete r;
  if (flags) return fail(UCP_ENONFINITE, "ticket %lld produced non-finite values", (long long)ticket);
  return UCP_OK;
}

}  // extern "C"

#define SRV_TRY(expr, what)                              \
  do {                                                   \
    hipError_t e_ = (expr);                              \
    if (e_ != hipSuccess) return hip_fail(e_, what);     \
  } while (0)

static int admit(ucp_server* s) {
  while (!s->queue.empty() && (int32_t)s->running.size() < s->max_slots) {
    Request* r = s->reqs[s->queue.front()];
    if (s->budget && s->used + r->bytes > s->budget) break;  // arrival order: wait for memory
    void* mem = acquire(s, r->bytes);
    if (!mem) {
      if (s->running.empty()) return fail(UCP_ENOMEM, "cannot allocate %zu bytes for a request", r->bytes);
      break;  // retry once running requests retire
    }
    s->queue.pop_front();
    r->dmem = mem;
    s->used += r->bytes;
    char* base = (char*)mem;
    carve_state(r->inst, base);
    r->d_J = (double*)base;
    r->state = kRunning;
    r->fresh = true;
    r->t = 0;
    s->running.push_back(r);
    SRV_TRY(hipMemcpyAsync(r->inst.u0, r->u0_init.data(), sizeof(double) * r->inst.n_x, hipMemcpyHostToDevice,
                           s->stream), "upload u0_init");
    SRV_TRY(clear_state(r->inst, s->stream), "clear state");
  }
  return UCP_OK;
}

// Upload the instance table of the running requests and the launch tables of
// two sets: the newly admitted (set-up) and those that run a round.
static int upload_tables(ucp_server* s, const std::vector<char>& fresh, const std::vector<char>& round,
                         std::vector<int32_t>& tab) {
  const int n = (int)s->running.size();
  std::vector<Inst> insts(n);
  for (int b = 0; b < n; ++b) {
    Request* r = s->running[b];
    insts[b] = r->inst;
    insts[b].J_out = r->d_J + (r->fresh ? 0 : r->t + 1);  // set-up writes J[0]; a round writes J[t + 1]
  }
  std::vector<int32_t> t0 = build_tables(insts, fresh);
  std::vector<int32_t> t1 = build_tables(insts, round);
  tab = t0;
  tab.insert(tab.end(), t1.begin(), t1.end());
  // the round's J entry differs from the set-up's for fresh requests: a
  // second instance table for the round phase
  std::vector<Inst> insts_round = insts;
  for (int b = 0; b < n; ++b) {
    Request* r = s->running[b];
    insts_round[b].J_out = r->d_J + (r->fresh ? 1 : r->t + 1);
  }
  const size_t need_i = sizeof(Inst) * 2 * (size_t)n;
  const size_t need_t = sizeof(int32_t) * tab.size();
  if (need_i > s->cap_insts) {
    if (s->d_insts) (void)hipFree(s->d_insts);
    s->d_insts = nullptr;
    SRV_TRY(hipMalloc(&s->d_insts, need_i * 2), "allocate instance table");
    s->cap_insts = need_i * 2;
  }
  if (need_t > s->cap_tab) {
    if (s->d_tab) (void)hipFree(s->d_tab);
    s->d_tab = nullptr;
    SRV_TRY(hipMalloc(&s->d_tab, need_t * 2), "allocate launch tables");
    s->cap_tab = need_t * 2;
  }
  // a step that failed part-way may have left uploads in flight
  SRV_TRY(hipStreamSynchronize(s->stream), "synchronise before staging");
  if (need_i + need_t > s->cap_stage) {
    if (s->h_stage) (void)hipHostFree(s->h_stage);
    s->h_stage = nullptr;
    s->cap_stage = 0;
    SRV_TRY(hipHostMalloc((void**)&s->h_stage, 2 * (need_i + need_t), hipHostMallocDefault), "allocate staging");
    s->cap_stage = 2 * (need_i + need_t);
  }
  std::memcpy(s->h_stage, insts.data(), sizeof(Inst) * n);
  std::memcpy(s->h_stage + sizeof(Inst) * n, insts_round.data(), sizeof(Inst) * n);
  std::memcpy(s->h_stage + need_i, tab.data(), need_t);
  SRV_TRY(hipMemcpyAsync(s->d_insts, s->h_stage, need_i, hipMemcpyHostToDevice, s->stream), "upload");
  SRV_TRY(hipMemcpyAsync(s->d_tab, s->h_stage + need_i, need_t, hipMemcpyHostToDevice, s->stream), "upload");
  return UCP_OK;
}

extern "C" int ucp_server_step(ucp_server* s, int32_t* n_running) {
  if (!s) return fail(UCP_EINVAL, "NULL server");
  SRV_TRY(hipSetDevice(s->device), "hipSetDevice");
  int rc = admit(s);
  if (rc) return rc;
  const int n = (int)s->running.size();
  if (n > 0) {
    std::vector<char> fresh(n), round(n);
    int max_lv = 0;
    for (int b = 0; b < n; ++b) {
      Request* r = s->running[b];
      fresh[b] = r->fresh;
      round[b] = r->t < r->iters;
      if (round[b]) max_lv = std::max(max_lv, (int)r->inst.levels);
    }
    std::vector<int32_t> tab;
    if ((rc = upload_tables(s, fresh, round, tab))) return rc;
    auto L = [&](int phase, int kind, int which_insts) {
      Launch l;
      l.insts = s->d_insts + (size_t)which_insts * n;
      l.n_inst = n;
      const size_t off = ((size_t)phase * kKinds + kind) * (n + 1);
      l.pre = s->d_tab + off;
      l.total = tab[off + n];
      return l;
    };
    const int prec = s->prec;
    hipStream_t st = s->stream;
    // set-up of the new requests
    SRV_TRY(launch_prior(L(0, kKindPrior, 0), st), "prior kernel");
    SRV_TRY(launch_gtab(L(0, kKindGtab, 0), st), "offset table kernel");
    SRV_TRY(launch_u1_partial(L(0, kKindU1s, 0), L(0, kKindU1p, 0), prec, st), "u1 kernel");
    SRV_TRY(launch_u1_combine(L(0, kKindU1c, 0), st), "u1 combine kernel");
    SRV_TRY(launch_gt_table(L(0, kKindGt, 0), st), "moment table kernel");
    SRV_TRY(launch_j_rows(L(0, kKindJRows, 0), st), "objective kernel");
    SRV_TRY(launch_j_reduce_t(L(0, kKindJRed, 0), 0, st), "objective reduce kernel");
    // one round for every running request (the levels read the moment
    // table built after the request's last u1 update)
    for (int l = 0; l < max_lv; ++l) {
      SRV_TRY(launch_mc(L(1, kKindMc0 + l, 1), l, prec, st), "marginal-cost kernel");
      SRV_TRY(launch_select(L(1, kKindSel0 + l, 1), L(1, kKindSelT0 + l, 1), l, prec, 0, st), "selection kernel");
    }
    SRV_TRY(launch_copy_u0(L(1, kKindCopy, 1), st), "u0 advance kernel");
    SRV_TRY(launch_u1_partial(L(1, kKindU1s, 1), L(1, kKindU1p, 1), prec, st), "u1 kernel");
    SRV_TRY(launch_u1_combine(L(1, kKindU1c, 1), st), "u1 combine kernel");
    SRV_TRY(launch_gt_table(L(1, kKindGt, 1), st), "moment table kernel");
    SRV_TRY(launch_j_rows(L(1, kKindJRows, 1), st), "objective kernel");
    SRV_TRY(launch_j_reduce_t(L(1, kKindJRed, 1), 0, st), "objective reduce kernel");
    // retire
    std::vector<Request*> keep;
    std::vector<Request*> done;
    for (int b = 0; b < n; ++b) {
      Request* r = s->running[b];
      r->fresh = false;
      if (round[b]) r->t += 1;
      if (r->t >= r->iters) {
        r->u0_out.resize(r->inst.n_x);
        r->u1_out.resize(r->inst.n_y);
        r->J_hist.resize(r->iters + 1);
        SRV_TRY(hipMemcpyAsync(r->u0_out.data(), r->inst.u0, sizeof(double) * r->inst.n_x, hipMemcpyDeviceToHost, st),
                "download u0");
        SRV_TRY(hipMemcpyAsync(r->u1_out.data(), r->inst.u1, sizeof(double) * r->inst.n_y, hipMemcpyDeviceToHost, st),
                "download u1");
        SRV_TRY(hipMemcpyAsync(r->J_hist.data(), r->d_J, sizeof(double) * (r->iters + 1), hipMemcpyDeviceToHost, st),
                "download J");
        SRV_TRY(hipMemcpyAsync(&r->flags, r->inst.flags, 4, hipMemcpyDeviceToHost, st), "download flags");
        done.push_back(r);
      } else {
        keep.push_back(r);
      }
    }
    SRV_TRY(hipStreamSynchronize(st), "synchronise");
    for (Request* r : done) {
      release(s, r);
      r->state = kDone;
    }
    s->running.swap(keep);
  }
  if (n_running) *n_running = (int32_t)s->running.size();
  return UCP_OK;
}
