// Issue-rate probes of the VALU operations the marginal-cost kernels are
// built from: FP32 FMA, the FP32 base-2 exponential (v_exp_f32) and FP64
// FMA.  They fix the peak the roofline of the bench line is taken against
// on the GPU at hand: lane-operations per second for each kind, with every
// wave slot of the chip busy and enough independent chains per lane to hide
// the pipeline latency.  Not part of the solver.
#include <hip/hip_runtime.h>

#include "ucp_internal.h"
#include "ucp_runtime.h"

namespace ucp {
namespace {

constexpr int kProbeChains = 8;   // independent chains per lane
constexpr int kProbeBlock = 256;

__global__ __launch_bounds__(kProbeBlock) void k_probe_fma32(int iters, float* out) {
  float a[kProbeChains];
  const float m = 1.0f + 1e-7f * (float)threadIdx.x, c = 1e-9f;
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) a[k] = (float)(k + 1) * 1e-3f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) a[k] = fmaf(a[k], m, c);
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) s += a[k];
  out[blockIdx.x * kProbeBlock + threadIdx.x] = s;
}

__global__ __launch_bounds__(kProbeBlock) void k_probe_exp32(int iters, float* out) {
  float a[kProbeChains];
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) a[k] = -1e-3f * (float)(k + 1 + threadIdx.x % 7);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) a[k] = -__builtin_amdgcn_exp2f(a[k]);  // stays in (-1, 0)
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) s += a[k];
  out[blockIdx.x * kProbeBlock + threadIdx.x] = s;
}

__global__ __launch_bounds__(kProbeBlock) void k_probe_fma64(int iters, double* out) {
  double a[kProbeChains];
  const double m = 1.0 + 1e-12 * (double)threadIdx.x, c = 1e-15;
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) a[k] = (double)(k + 1) * 1e-3;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) a[k] = fma(a[k], m, c);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) s += a[k];
  out[blockIdx.x * kProbeBlock + threadIdx.x] = s;
}

}  // namespace
}  // namespace ucp

using namespace ucp;

// kind 0: FP32 FMA, 1: v_exp_f32, 2: FP64 FMA, on `device`.  Launches
// `blocks` blocks of 256 lanes, each lane running kProbeChains chains of
// `iters` operations,
// times the launch with HIP events on `stream` (synchronising it) and
// returns the lane-operations per second.
extern "C" int ucp_peak_probe(int device, int kind, int32_t blocks, int32_t iters, double* lane_ops_per_s,
                              void* stream) {
  if (kind < 0 || kind > 2 || blocks < 1 || iters < 1 || !lane_ops_per_s)
    return fail(UCP_EINVAL, "kind must be 0..2, blocks and iters >= 1, output not NULL");
  int ndev = 0;
  hipError_t e0_ = hipGetDeviceCount(&ndev);
  if (e0_ != hipSuccess || ndev <= 0) return fail(UCP_EHIP, "no HIP device available");
  if (device < 0 || device >= ndev) return fail(UCP_EINVAL, "device %d out of range (have %d)", device, ndev);
  if ((e0_ = hipSetDevice(device)) != hipSuccess) return hip_fail(e0_, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  void* buf = nullptr;
  const size_t n = (size_t)blocks * kProbeBlock;
  hipError_t e = hipMalloc(&buf, n * 8);
  if (e != hipSuccess) return fail(UCP_ENOMEM, "probe buffer: %s", hipGetErrorString(e));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float ms = 0.0f;
  int rc = UCP_OK;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
    rc = hip_fail(e, "event");
  } else {
    for (int rep = 0; rep < 2 && rc == UCP_OK; ++rep) {  // the first launch warms up
      (void)hipEventRecord(e0, st);
      if (kind == 0) hipLaunchKernelGGL(k_probe_fma32, dim3(blocks), dim3(kProbeBlock), 0, st, iters, (float*)buf);
      if (kind == 1) hipLaunchKernelGGL(k_probe_exp32, dim3(blocks), dim3(kProbeBlock), 0, st, iters, (float*)buf);
      if (kind == 2) hipLaunchKernelGGL(k_probe_fma64, dim3(blocks), dim3(kProbeBlock), 0, st, iters, (double*)buf);
      (void)hipEventRecord(e1, st);
      if ((e = hipGetLastError()) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
          (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
        rc = hip_fail(e, "probe launch");
    }
  }
  if (rc == UCP_OK) *lane_ops_per_s = (double)n * kProbeChains * (double)iters / (ms * 1e-3);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(buf);
  return rc;
}
