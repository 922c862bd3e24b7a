// Accuracy guard of the merge inverses (Algorithm "Merge stage": "Invert D").
//
// A merge matrix D inverted by block elimination around its zero interface
// blocks is only as accurate as its diagonal blocks and their Schur
// complement are well conditioned, and for Helmholtz operators those blocks
// (Dirichlet problems of two-leaf sub-rectangles) can sit near resonance while
// D itself is benign.  Every merge inverse Z is therefore probed with a fixed
// vector x:  rho = |Z (D x) - x|_inf / |x|_inf  (the probe's D x is formed
// before the inversion overwrites D).  Nodes whose rho exceeds a threshold
// are switched on in a per-node gate that the Newton-Schulz GEMMs
// Z <- 2 Z - (Z D) Z of the block-eliminated levels read on the device; each
// step squares the residual I - Z D.  The kernels here are the probe's
// reduction and the gated copy of the refined inverse.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "../../include/hps.h"

namespace hps {

constexpr int PR_THREADS = 256;

__device__ __forceinline__ double nanmax(double a, double b) { return (a > b || a != a) ? a : b; }

// rho[b] = max_i |r_b(i)| * inv_xmax;  gate[b] = 1 unless rho[b] <= tau
// (a NaN residual keeps the gate on).  One workgroup per node.
__global__ __launch_bounds__(PR_THREADS) void probe_reduce_kernel(const double* __restrict__ r, long long stride,
                                                                  int m, double inv_xmax, double tau,
                                                                  double* __restrict__ rho, int* __restrict__ gate) {
  __shared__ double s[PR_THREADS];
  const long long b = blockIdx.x;
  const double* rb = r + b * stride;
  double mx = 0.0;
  for (int i = threadIdx.x; i < m; i += PR_THREADS) mx = nanmax(fabs(rb[i]), mx);
  s[threadIdx.x] = mx;
  __syncthreads();
  for (int w = PR_THREADS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] = nanmax(s[threadIdx.x + w], s[threadIdx.x]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double v = s[0] * inv_xmax;
    rho[b] = v;
    gate[b] = (v <= tau) ? 0 : 1;
  }
}

int probe_reduce_launch(const double* r, long long stride, int m, double inv_xmax, double tau, double* rho,
                        int* gate, long long nodes, hipStream_t st) {
  if (nodes <= 0) return HPS_OK;
  hipLaunchKernelGGL(probe_reduce_kernel, dim3((unsigned)nodes), dim3(PR_THREADS), 0, st, r, stride, m, inv_xmax,
                     tau, rho, gate);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

// dst[b] = src[b] (n doubles per node) for the nodes whose gate is on.
constexpr int GC_THREADS = 256;
__global__ __launch_bounds__(GC_THREADS) void gated_copy_kernel(double* __restrict__ dst,
                                                                const double* __restrict__ src, long long n,
                                                                const int* __restrict__ gate) {
  const long long b = blockIdx.y;
  if (gate[b] == 0) return;
  double* d = dst + b * n;
  const double* s = src + b * n;
  const long long step = (long long)GC_THREADS * gridDim.x;
  for (long long i = (long long)blockIdx.x * GC_THREADS + threadIdx.x; i < n; i += step) d[i] = s[i];
}

int gated_copy_launch(double* dst, const double* src, long long n, const int* gate, long long nodes,
                      hipStream_t st) {
  if (nodes <= 0 || n <= 0) return HPS_OK;
  long long gx = (n + GC_THREADS - 1) / GC_THREADS;
  const long long cap = std::max(1LL, 4096LL / nodes);  // about 4096 workgroups in all
  if (gx > cap) gx = cap;
  hipLaunchKernelGGL(gated_copy_kernel, dim3((unsigned)gx, (unsigned)nodes), dim3(GC_THREADS), 0, st, dst, src, n,
                     gate);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

}  // namespace hps
