// Device pieces of the adaptive 3D path (Section 4.2): row permutations
// between the caller's depth-first leaf order and the level-grouped leaf
// slots, and the refinement criterion of eq. (refinement_check).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.hpp"
#include "../../include/hps.h"

namespace hps {

// dst[r][i][e] = src[r][idx[i]][e]  (rows of len doubles; r < nrhs)
__global__ __launch_bounds__(256) void adaptive_permute_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                                               const int* __restrict__ idx, long long len, long long n,
                                                               long long src_rstride, long long dst_rstride) {
  const int r = blockIdx.y;
  const long long total = n * len;
  const double* s = src + (long long)r * src_rstride;
  double* d = dst + (long long)r * dst_rstride;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    const long long i = e / len, k = e - i * len;
    d[e] = s[(long long)idx[i] * len + k];
  }
}

int adaptive_permute_launch(const double* src, double* dst, const int* idx, long long len, long long n, int nrhs,
                            long long src_rstride, long long dst_rstride, hipStream_t st) {
  if (n <= 0 || len <= 0 || nrhs <= 0) return HPS_OK;
  if (nrhs > 65535) { set_error("permute: too many right-hand sides"); return HPS_EINVAL; }
  const long long total = n * len;
  const unsigned gx = (unsigned)std::min<long long>(4096, (total + 255) / 256);
  hipLaunchKernelGGL(adaptive_permute_kernel, dim3(gx, (unsigned)nrhs), dim3(256), 0, st, src, dst, idx, len, n,
                     src_rstride, dst_rstride);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

// Refinement check of one leaf per workgroup.  f0 [leaf][p^3] are the samples
// at the leaf's Chebyshev points, f1 [leaf][8][p^3] those at its children's
// (children in the merge's child order: offsets (x, y, z) = 000, 100, 110,
// 010, 001, 101, 111, 011), E [2][p][p] row-major the 1D interpolation from
// the leaf's nodes to the lower / upper child's nodes.  The tensor
// interpolation runs one axis at a time through LDS.
// err[leaf] = max |f1 - L_8f1 f0|, fabsmax[leaf] = max |f0|.
constexpr int CHK_MAXP = 16;
__global__ __launch_bounds__(256) void adaptive_check_kernel(const double* __restrict__ f0, const double* __restrict__ f1,
                                                             const double* __restrict__ E, int p,
                                                             double* __restrict__ err, double* __restrict__ fabsmax) {
  __shared__ double a[CHK_MAXP * CHK_MAXP * CHK_MAXP];
  __shared__ double b[CHK_MAXP * CHK_MAXP * CHK_MAXP];
  __shared__ double red[2][256];
  static constexpr int off[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0},
                                    {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};
  const long long leaf = blockIdx.x;
  const int np = p * p * p, tid = threadIdx.x;
  const double* x0 = f0 + leaf * np;
  double e_max = 0.0, f_max = 0.0;
  for (int j = tid; j < np; j += blockDim.x) f_max = fmax(f_max, fabs(x0[j]));
  for (int c = 0; c < 8; ++c) {
    const double* Ex = E + off[c][0] * p * p;
    const double* Ey = E + off[c][1] * p * p;
    const double* Ez = E + off[c][2] * p * p;
    for (int j = tid; j < np; j += blockDim.x) a[j] = x0[j];
    __syncthreads();
    for (int j = tid; j < np; j += blockDim.x) {  // along x
      const int ix = j % p, rest = j - ix;
      double s = 0.0;
      for (int k = 0; k < p; ++k) s += Ex[ix * p + k] * a[rest + k];
      b[j] = s;
    }
    __syncthreads();
    for (int j = tid; j < np; j += blockDim.x) {  // along y
      const int ix = j % p, iy = (j / p) % p, iz = j / (p * p);
      double s = 0.0;
      for (int k = 0; k < p; ++k) s += Ey[iy * p + k] * b[ix + p * k + p * p * iz];
      a[j] = s;
    }
    __syncthreads();
    const double* x1 = f1 + (leaf * 8 + c) * np;
    for (int j = tid; j < np; j += blockDim.x) {  // along z, compared with the children's samples
      const int ixy = j % (p * p), iz = j / (p * p);
      double s = 0.0;
      for (int k = 0; k < p; ++k) s += Ez[iz * p + k] * a[ixy + p * p * k];
      e_max = fmax(e_max, fabs(x1[j] - s));
    }
    __syncthreads();
  }
  red[0][tid] = e_max;
  red[1][tid] = f_max;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) {
      red[0][tid] = fmax(red[0][tid], red[0][tid + s]);
      red[1][tid] = fmax(red[1][tid], red[1][tid + s]);
    }
    __syncthreads();
  }
  if (tid == 0) {
    err[leaf] = red[0][0];
    fabsmax[leaf] = red[1][0];
  }
}

int adaptive_check_launch(const double* f0, const double* f1, const double* E, int p, long long nl, double* err,
                          double* fmax_out, hipStream_t st) {
  if (p > CHK_MAXP || p < 2) { set_error("refinement check: p out of range"); return HPS_EINVAL; }
  if (nl <= 0) return HPS_OK;
  hipLaunchKernelGGL(adaptive_check_kernel, dim3((unsigned)nl), dim3(256), 0, st, f0, f1, E, p, err, fmax_out);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

}  // namespace hps
