// 3D leaf stage (Appendix C.1: the 2D local solve with 3D P, Q, I_i, I_e).
//
// n_i = (p-2)^3 interior unknowns per leaf (1000 at p = 12) is too large for a
// register-resident factorization, so the 3D leaf stage is split:
//   leaf3d_assemble   L_ii (n_i x n_i) and R = L_ie P (n_i x n_b) per leaf,
//                     column-major, written to HBM;
//   blocked Gauss-Jordan (gj.hip) on the batch of L_ii  ->  L_ii^{-1};
//   GEMMs             Y_int = -L_ii^{-1} R,   T = Q_e P + Q_i Y_int.
// The explicit inverse also serves the sources at solve time (a GEMM).
//
// leaf_gather_int: f at the interior points of every leaf, into the
// [leaf][rhs][n_i] layout the source GEMM reads.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "../../include/hps.h"

namespace hps {

__global__ void leaf3d_assemble_kernel(const double* __restrict__ coeffs,  // [nl][10][p^3]
                                       const double* __restrict__ D1, const double* __restrict__ D2,  // [p*p]
                                       const double* __restrict__ Mt,  // [10][n_i x n_b]
                                       int p, double* __restrict__ Lii, double* __restrict__ R) {
  const int q = p - 2, ni = q * q * q, nb = 6 * q * q, np = p * p * p;
  const long long leaf = blockIdx.y;
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;  // element of [L_ii | R]
  if (e >= (long long)ni * (ni + nb)) return;
  const int row = (int)(e % ni);
  const int col = (int)(e / ni);
  const int ixr = 1 + row % q, iyr = 1 + (row / q) % q, izr = 1 + row / (q * q);
  const int pr = ixr + p * iyr + p * p * izr;
  const double* c = coeffs + leaf * 10 * np + pr;
  if (col < ni) {
    const int ixc = 1 + col % q, iyc = 1 + (col / q) % q, izc = 1 + col / (q * q);
    const bool sx = ixr == ixc, sy = iyr == iyc, sz = izr == izc;
    double v = 0.0;
    if (sy && sz) v += c[0 * np] * D2[ixr * p + ixc] + c[6 * np] * D1[ixr * p + ixc];
    if (sx && sz) v += c[1 * np] * D2[iyr * p + iyc] + c[7 * np] * D1[iyr * p + iyc];
    if (sx && sy) v += c[2 * np] * D2[izr * p + izc] + c[8 * np] * D1[izr * p + izc];
    if (sz && c[3 * np] != 0.0) v += c[3 * np] * D1[iyr * p + iyc] * D1[ixr * p + ixc];
    if (sy && c[4 * np] != 0.0) v += c[4 * np] * D1[izr * p + izc] * D1[ixr * p + ixc];
    if (sx && c[5 * np] != 0.0) v += c[5 * np] * D1[izr * p + izc] * D1[iyr * p + iyc];
    if (row == col) v += c[9 * np];
    Lii[leaf * (long long)ni * ni + e] = v;
  } else {
    const long long j = col - ni;
    double v = 0.0;
#pragma unroll
    for (int t = 0; t < 9; ++t) {  // the zeroth-order term has no L_ie part
      const double ct = c[t * np];
      if (ct != 0.0) v += ct * Mt[(long long)t * ni * nb + row + j * ni];
    }
    R[leaf * (long long)ni * nb + row + j * ni] = v;
  }
}

int leaf3d_assemble_launch(const double* coeffs, const double* D1, const double* D2, const double* Mt, int p,
                           double* Lii, double* R, long long nl, hipStream_t st) {
  const int q = p - 2, ni = q * q * q, nb = 6 * q * q;
  const long long n = (long long)ni * (ni + nb);
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)nl);
  hipLaunchKernelGGL(leaf3d_assemble_kernel, grid, dim3(256), 0, st, coeffs, D1, D2, Mt, p, Lii, R);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

// fint[leaf][r][k] = src[r][leaf][Ii[k]] for r < nrhs
__global__ void leaf_gather_int_kernel(const double* __restrict__ src, const int* __restrict__ Ii, int ni, int npts,
                                       long long nl, int nrhs, int NRcap, double* __restrict__ fint) {
  const long long leaf = blockIdx.y;
  const int r = blockIdx.z;
  if (r >= nrhs) return;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < ni; k += gridDim.x * blockDim.x)
    fint[(leaf * NRcap + r) * ni + k] = src[((long long)r * nl + leaf) * npts + Ii[k]];
}

int leaf_gather_int_launch(const double* src, const int* Ii, int ni, int npts, long long nl, int nrhs, int NRcap,
                           double* fint, hipStream_t st) {
  dim3 grid((unsigned)((ni + 255) / 256), (unsigned)nl, (unsigned)nrhs);
  hipLaunchKernelGGL(leaf_gather_int_kernel, grid, dim3(256), 0, st, src, Ii, ni, npts, nl, nrhs, NRcap, fint);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

}  // namespace hps
