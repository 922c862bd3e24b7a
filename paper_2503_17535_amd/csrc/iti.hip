// Leaf stage of the ItI variant (Appendix B.1, Algorithm "2D ItI local
// solve"): assembly of B = [G; L(I_i, :)] for every leaf.
//
// Complex quantities are carried in their real representation with the real
// and imaginary parts interleaved: a complex vector of length n is the real
// vector [Re x_0, Im x_0, Re x_1, ...] (the memory layout of a complex128
// array), and a complex r x c matrix M is the real 2r x 2c matrix whose 2 x 2
// block (i, j) is [[Re M_ij, -Im M_ij], [Im M_ij, Re M_ij]].  Products,
// inverses and block copies of these real matrices are those of the complex
// ones, so the library's fp64 GEMM, Gauss-Jordan and block-copy kernels run
// the ItI method unchanged with every size doubled.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.hpp"
#include "../../include/hps.h"

namespace hps {

// L_{ij} = sum_t c_t(x_i) (D_t)_{ij} on a leaf (real coefficients; term
// order xx, xy, yy, x, y, 0; point index ix + p iy)
__device__ inline double iti_lval(const double* __restrict__ ci, const double* __restrict__ D1,
                                  const double* __restrict__ D2, int p, int np, int i, int jc) {
  const int ix = i % p, iy = i / p, jx = jc % p, jy = jc / p;
  const double dx1 = D1[ix * p + jx], dy1 = D1[iy * p + jy];
  double val = ci[np] * dx1 * dy1;  // c_xy d_x d_y
  if (iy == jy) val += ci[0] * D2[ix * p + jx] + ci[3 * np] * dx1;
  if (ix == jx) val += ci[2 * np] * D2[iy * p + jy] + ci[4 * np] * dy1;
  if (i == jc) val += ci[5 * np];
  return val;
}

// Row equilibration of the interior rows: scale[leaf][2a + s] = 1 / max_j
// |L(Ii[a], j)| (the Robin rows are scaled on the host; their G is the same on
// every leaf).  Gauss-Jordan with partial pivoting on B as assembled (row
// magnitudes from ~1/r to ~p^4/r^2) leaves residuals |B B^{-1} - I| about a
// hundred times larger than on the equilibrated matrix.
__global__ __launch_bounds__(64) void iti_row_scale_kernel(const double* __restrict__ coeffs,
                                                            const double* __restrict__ D1,
                                                            const double* __restrict__ D2,
                                                            const int* __restrict__ Ii, int p, int ni,
                                                            double* __restrict__ scale) {
  const long long leaf = blockIdx.y;
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= ni) return;
  const int np = p * p, i = Ii[a];
  const double* ci = coeffs + leaf * 6 * np + i;
  double mx = 0.0;
  for (int jc = 0; jc < np; ++jc) mx = fmax(mx, fabs(iti_lval(ci, D1, D2, p, np, i, jc)));
  const double s = mx > 0.0 ? 1.0 / mx : 1.0;
  scale[leaf * 2 * ni + 2 * a] = s;
  scale[leaf * 2 * ni + 2 * a + 1] = s;
}

// B (real representation, 2p^2 x 2p^2, column-major) of every leaf:
//   rows 0 .. 2nr - 1: the Robin rows G (the same on every leaf; Gr given in
//   the real representation, column-major with leading dimension 2nr);
//   rows 2nr + 2a + s: interior point Ii[a], part s, times scale[leaf][2a+s];
//   the operator L = sum_t c_t D_t has real coefficients, so its 2 x 2
//   blocks are diag(L_ij, L_ij).
// D1 / D2: first / second derivative on the leaf, p x p row-major; the point
// index is ix + p iy.
__global__ __launch_bounds__(256) void iti_leaf_assemble_kernel(const double* __restrict__ coeffs,
                                                                 const double* __restrict__ D1,
                                                                 const double* __restrict__ D2,
                                                                 const double* __restrict__ Gr,
                                                                 const int* __restrict__ Ii,
                                                                 const double* __restrict__ scale, int p, int nr,
                                                                 double* __restrict__ B) {
  const long long leaf = blockIdx.y;
  const int np = p * p, m = 2 * np, nr2 = 2 * nr, ni2 = m - nr2;
  const double* c = coeffs + leaf * 6 * np;
  const double* sc = scale + leaf * ni2;
  double* Bl = B + leaf * (long long)m * m;
  const long long total = (long long)m * m;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(e % m), j = (int)(e / m);  // row, column
    double val;
    if (k < nr2) {
      val = Gr[(long long)j * nr2 + k];
    } else {
      const int kr = k & 1, jr = j & 1;
      val = 0.0;
      if (kr == jr) {
        const int i = Ii[(k - nr2) >> 1];
        val = sc[k - nr2] * iti_lval(c + i, D1, D2, p, np, i, j >> 1);
      }
    }
    Bl[e] = val;
  }
}

// scale: [leaf][2 (p-2)^2] interior row scales (written here)
int iti_leaf_assemble_launch(const double* coeffs, const double* D1, const double* D2, const double* Gr,
                             const int* Ii, int p, long long nl, double* scale, double* B, hipStream_t st) {
  if (nl <= 0) return HPS_OK;
  const long long m = 2LL * p * p;
  const int ni = (p - 2) * (p - 2);
  const unsigned gx = (unsigned)std::min<long long>(256, (m * m + 255) / 256);
  for (long long l0 = 0; l0 < nl; l0 += 65535) {
    const long long cnt = std::min<long long>(65535, nl - l0);
    const double* cl = coeffs + l0 * 6 * p * p;
    double* sl = scale + l0 * 2 * ni;
    hipLaunchKernelGGL(iti_row_scale_kernel, dim3((unsigned)((ni + 63) / 64), (unsigned)cnt), dim3(64), 0, st, cl, D1,
                       D2, Ii, p, ni, sl);
    HPS_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(iti_leaf_assemble_kernel, dim3(gx, (unsigned)cnt), dim3(256), 0, st, cl, D1, D2, Gr, Ii, sl, p,
                       4 * p - 4, B + l0 * m * m);
    HPS_HIP_TRY(hipGetLastError());
  }
  return HPS_OK;
}

// fint[leaf][r][k] = src[r][leaf][Iir[k]] * scale[leaf][k] for r < nrhs: the
// interior source values in the real representation, with the row scales of
// the equilibrated B (B^{-1}(:, I_i) f = (D B)^{-1}(:, I_i) (D f))
__global__ __launch_bounds__(256) void iti_gather_src_kernel(const double* __restrict__ src,
                                                              const int* __restrict__ Iir,
                                                              const double* __restrict__ scale, int ni2, int m,
                                                              long long nl, int NRcap, double* __restrict__ fint) {
  const long long leaf = blockIdx.y;
  const int r = blockIdx.z;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < ni2; k += gridDim.x * blockDim.x)
    fint[(leaf * NRcap + r) * ni2 + k] = src[((long long)r * nl + leaf) * m + Iir[k]] * scale[leaf * ni2 + k];
}

int iti_gather_src_launch(const double* src, const int* Iir, const double* scale, int ni2, int m, long long nl,
                          int nrhs, int NRcap, double* fint, hipStream_t st) {
  if (nl <= 0 || nrhs <= 0) return HPS_OK;
  if (nl > 65535) {
    set_error("ItI source gather: more than 65535 leaves");
    return HPS_EINVAL;
  }
  dim3 grid((unsigned)((ni2 + 255) / 256), (unsigned)nl, (unsigned)nrhs);
  hipLaunchKernelGGL(iti_gather_src_kernel, grid, dim3(256), 0, st, src, Iir, scale, ni2, m, nl, NRcap, fint);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

}  // namespace hps
