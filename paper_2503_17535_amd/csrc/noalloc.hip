// Device-wide static workspace of the allocation-free solve (hps_solve_noalloc).
//
// The solve's per-level vectors (boundary data g and outgoing fluxes h of
// every tree level, leaf particular solutions v, interface data of every
// merge, split-K partial products) normally live in memory the operator
// allocates at build time.  The allocation-free entry point places them in
// `scratch` instead: a file-scope device array that the code object brings
// with it, one copy per GPU, alive until the process ends.
//
// In host code `scratch` names a host-side stand-in, not device memory: a
// kernel handed that name would fault.  Its device address is therefore
// looked up once per device with hipGetSymbolAddress (with that device
// current) and only that address is used (kernel arguments, descriptor
// tables).  Every call on one GPU shares its copy; calls that overlap on one
// GPU race on it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.hpp"
#include "../../include/hps.h"

namespace hps {

static __device__ __align__(256) char scratch[HPS_STATIC_WS_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of the current device's copy of `scratch` (looked up on the
// first call per device).  Returns HPS_EDEVICE if the lookup fails.
int static_ws_ptr(void** out) {
  *out = nullptr;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return HPS_EDEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HPS_EDEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return HPS_OK;
}

// x[0 .. n) = 0 by a kernel (not hipMemsetAsync, so that a caller may capture
// the solve in a HIP graph).
constexpr int ZF_THREADS = 256;
__global__ __launch_bounds__(ZF_THREADS) void zero_fill_kernel(double* __restrict__ x, long long n) {
  const long long step = (long long)gridDim.x * ZF_THREADS;
  for (long long i = (long long)blockIdx.x * ZF_THREADS + threadIdx.x; i < n; i += step) x[i] = 0.0;
}

int zero_fill_launch(double* x, long long n, hipStream_t st) {
  if (n <= 0) return HPS_OK;
  long long nb = (n + ZF_THREADS - 1) / ZF_THREADS;
  if (nb > 2048) nb = 2048;
  hipLaunchKernelGGL(zero_fill_kernel, dim3((unsigned)nb), dim3(ZF_THREADS), 0, st, x, n);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

}  // namespace hps
