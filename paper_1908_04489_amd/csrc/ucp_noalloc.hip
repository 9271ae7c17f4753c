// ucp_argmin_adaptive_noalloc: the pointwise u0 update of
// ucp_argmin_adaptive for callers that cannot allocate (code under HIP graph
// capture, serving loops that forbid allocation).  It runs the same kernels
// on the same instance layout, with the instance record, its launch tables
// and its state carved from one file-scope device array instead of the
// handle's workspace.
//
// The array's host-side name is not a device address: each device's copy is
// looked up once with hipGetSymbolAddress (device current) and that address
// is what every kernel argument and copy uses.  Every call on one device
// shares that device's copy, so calls that overlap on one device race; the
// array keeps the last call's contents, and everything a call needs zeroed
// (the non-finite flag) is cleared by the call's own first kernel.  The
// instance record and the launch tables travel as a kernel argument, so no
// host memory is a copy source and no hipMemsetAsync is issued.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <vector>

#include "ucp_internal.h"
#include "ucp_runtime.h"

namespace ucp {
namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {nullptr};

// The device address of `scratch` on `device` (which is current).
int scratch_on(int device, char** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[device] = (char*)p;
  }
  *out = g_scratch_ptr[device];
  return UCP_OK;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// The state the u0 update uses, carved from `base`: the update reads the
// caller's u0 and u1 in place, and never touches the u1 partial sums, the
// objective rows or the work counters.  The moment table (FP32 modes on
// grids fine enough for it) is rebuilt from u1 by every call.
size_t update_bytes(const Inst& I) {
  const size_t nx = (size_t)I.n_x, ny = (size_t)I.n_y;
  return 7 * align256(nx * 8) + align256(ny * 4) + align256((size_t)(2 * I.nw32 + 1 + kGtabPad) * 4) +
         align256(part_doubles(I) * 8) + 256 +
         (I.gts ? align256((size_t)I.gtr * 3 * (kGtN + 1) * 8) : 0);
}
void carve_update(Inst& I, char* base) {
  const size_t nx = (size_t)I.n_x, ny = (size_t)I.n_y;
  auto take = [&](size_t bytes) {
    char* p = base;
    base += align256(bytes);
    return p;
  };
  I.u0_next = (double*)take(nx * 8);
  I.f = (double*)take(nx * 8);
  I.logf = (double*)take(nx * 8);
  I.cbest = (double*)take(nx * 8);
  I.b32best = (double*)take(nx * 8);
  I.b64best = (double*)take(nx * 8);
  I.b32inc = (double*)take(nx * 8);
  I.v = (float*)take(ny * 4);
  I.gtab = (float*)take((size_t)(2 * I.nw32 + 1 + kGtabPad) * 4);
  I.part = (double*)take(part_doubles(I) * 8);
  I.flags = (int32_t*)take(256);
  I.gt = I.gts ? (double*)take((size_t)I.gtr * 3 * (kGtN + 1) * 8) : nullptr;
  I.u1part = nullptr;
  I.u1stat = nullptr;
  I.jrow = nullptr;
  I.terms = nullptr;
}

// The instance record and its launch tables (one phase), passed by value.
struct Header {
  Inst inst;
  int32_t pre[kKinds * 2];
};
static_assert(sizeof(Header) <= 2048, "the header travels as a kernel argument");

constexpr size_t kHeaderBytes = (sizeof(Header) + 255) & ~(size_t)255;

// Writes the header into the scratch array and clears the instance's flags.
__global__ void k_put_header(Header h, Header* dst, int32_t* flags) {
  const int t = threadIdx.x;
  const int32_t* src = (const int32_t*)&h;
  int32_t* out = (int32_t*)dst;
  for (int k = t; k < (int)(sizeof(Header) / 4); k += blockDim.x) out[k] = src[k];
  if (t < 64) flags[t] = 0;
}

}  // namespace
}  // namespace ucp

using namespace ucp;

extern "C" int ucp_argmin_adaptive_noalloc(ucp_handle* h, const ucp_problem* prob, const ucp_search* search,
                                           ucp_prec prec, const double* u1, const double* u0_in, double* u0_out,
                                           double* L0_out, void* stream) {
  if (!h) return fail(UCP_EINVAL, "handle is NULL");
  int rc;
  if ((rc = check_problem(prob)) || (rc = check_search(search)) || (rc = check_prec(prec))) return rc;
  if (prec == UCP_FP64_GT) return fail(UCP_EINVAL, "the allocation-free update does not take UCP_FP64_GT");
  if (!u1 || !u0_in || !u0_out) return fail(UCP_EINVAL, "NULL array argument");
  const int device = handle_device(h);
  if (device < 0 || device >= kMaxDevices) return fail(UCP_EINVAL, "device %d beyond the supported range", device);
  Inst I = make_inst(*prob, search, prec, 0);
  const size_t need = kHeaderBytes + update_bytes(I);
  if (need > kScratchBytes)
    return fail(UCP_EINVAL,
                "this problem needs %zu bytes of scratch, above the allocation-free limit of %zu "
                "(use ucp_argmin_adaptive)",
                need, kScratchBytes);
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  char* base = nullptr;
  if ((rc = scratch_on(device, &base))) return rc;
  hipStream_t st = (hipStream_t)stream;
  Header* dh = (Header*)base;
  carve_update(I, base + kHeaderBytes);
  // the caller's arrays are read in place: the update reads u0 (the
  // incumbents) and u1 only, and writes u0_next, copied out at the end
  I.u0 = const_cast<double*>(u0_in);
  I.u1 = const_cast<double*>(u1);
  I.L0_out = L0_out;
  Header hd;
  std::memset(&hd, 0, sizeof hd);
  hd.inst = I;
  std::vector<char> run(1, 1);
  std::vector<int32_t> tab = build_tables({I}, run);
  std::memcpy(hd.pre, tab.data(), sizeof(hd.pre));
  hipLaunchKernelGGL(k_put_header, dim3(1), dim3(256), 0, st, hd, dh, I.flags);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "header kernel");
  auto L = [&](int kind) {
    Launch l;
    l.insts = &dh->inst;
    l.n_inst = 1;
    l.pre = dh->pre + (size_t)kind * 2;
    l.total = tab[(size_t)kind * 2 + 1];
    return l;
  };
#define NA_TRY(expr, what)                           \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)
  NA_TRY(launch_prior(L(kKindPrior), st), "prior kernel");
  NA_TRY(launch_gtab(L(kKindGtab), st), "offset table kernel");
  NA_TRY(launch_v_from_u1(L(kKindU1c), st), "residual kernel");
  NA_TRY(launch_gt_table(L(kKindGt), st), "moment table kernel");
  for (int l = 0; l < I.levels; ++l) {
    NA_TRY(launch_mc(L(kKindMc0 + l), l, prec, st), "marginal-cost kernel");
    NA_TRY(launch_select(L(kKindSel0 + l), L(kKindSelT0 + l), l, prec, L0_out != nullptr, st), "selection kernel");
  }
  NA_TRY(hipMemcpyAsync(u0_out, I.u0_next, sizeof(double) * I.n_x, hipMemcpyDeviceToDevice, st), "copy u0_out");
#undef NA_TRY
  return UCP_OK;
}
