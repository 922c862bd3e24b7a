// Gradient of a scalar misfit with respect to the coefficient fields.
//
// The coefficients c_t enter the discrete system only through the collocation
// rows at interior leaf points (Section 2: boundary bordering replaces the
// rows at the leaf boundary points).  With K u = b and lam = K^{-T} grad_u J,
//   dJ/dc_t(x) = -lam(x) (d_t u)(x)   at interior points,   0 elsewhere,
// where d_t is the leaf's spectral derivative of term t (tensor products of
// the 1D Chebyshev derivative D).  One workgroup per leaf; u of one
// right-hand side at a time is staged in LDS, the sum over right-hand sides
// accumulates in the output (each point is owned by one thread).
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "../../include/hps.h"

namespace hps {

constexpr int GRAD_THREADS = 256;

template <int D>
__global__ __launch_bounds__(GRAD_THREADS) void coeff_grad_kernel(const double* __restrict__ u,
                                                                  const double* __restrict__ lam,
                                                                  const double* __restrict__ D1g,
                                                                  const double* __restrict__ D2g, int p,
                                                                  long long nl, int nrhs,
                                                                  double* __restrict__ grad) {
  constexpr int NT = D == 2 ? 6 : 10;
  extern __shared__ double sm[];
  double* sD1 = sm;
  double* sD2 = sm + p * p;
  double* su = sm + 2 * p * p;
  const int npts = D == 2 ? p * p : p * p * p;
  const long long leaf = blockIdx.x;
  const int tid = threadIdx.x;
  for (int i = tid; i < p * p; i += GRAD_THREADS) {
    sD1[i] = D1g[i];
    sD2[i] = D2g[i];
  }
  for (int r = 0; r < nrhs; ++r) {
    __syncthreads();  // the previous right-hand side is done with su
    const double* ur = u + ((long long)r * nl + leaf) * npts;
    for (int i = tid; i < npts; i += GRAD_THREADS) su[i] = ur[i];
    __syncthreads();
    const double* lr = lam + ((long long)r * nl + leaf) * npts;
    for (int pt = tid; pt < npts; pt += GRAD_THREADS) {
      const int ix = pt % p, iy = (pt / p) % p, iz = pt / (p * p);
      const bool inner = ix > 0 && ix < p - 1 && iy > 0 && iy < p - 1 && (D == 2 || (iz > 0 && iz < p - 1));
      double g[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) g[t] = 0.0;
      if (inner) {
        const double* d1x = sD1 + ix * p;
        const double* d1y = sD1 + iy * p;
        const double* d2x = sD2 + ix * p;
        const double* d2y = sD2 + iy * p;
        const int base = p * p * iz;
        double dx = 0.0, dy = 0.0, dxx = 0.0, dyy = 0.0, dxy = 0.0;
        for (int a = 0; a < p; ++a) {
          const double ux = su[a + p * iy + base], uy = su[ix + p * a + base];
          dx += d1x[a] * ux;
          dxx += d2x[a] * ux;
          dy += d1y[a] * uy;
          dyy += d2y[a] * uy;
          double s = 0.0;
          for (int b = 0; b < p; ++b) s += d1x[b] * su[b + p * a + base];
          dxy += d1y[a] * s;
        }
        const double l = -lr[pt];
        if (D == 2) {
          g[0] = l * dxx; g[1] = l * dxy; g[2] = l * dyy;
          g[3] = l * dx;  g[4] = l * dy;  g[5] = l * su[pt];
        } else {
          const double* d1z = sD1 + iz * p;
          const double* d2z = sD2 + iz * p;
          double dz = 0.0, dzz = 0.0, dxz = 0.0, dyz = 0.0;
          for (int c = 0; c < p; ++c) {
            const double uz = su[ix + p * iy + p * p * c];
            dz += d1z[c] * uz;
            dzz += d2z[c] * uz;
            double sx = 0.0, sy = 0.0;
            for (int b = 0; b < p; ++b) {
              sx += d1x[b] * su[b + p * iy + p * p * c];
              sy += d1y[b] * su[ix + p * b + p * p * c];
            }
            dxz += d1z[c] * sx;
            dyz += d1z[c] * sy;
          }
          g[0] = l * dxx; g[1] = l * dyy; g[2] = l * dzz;
          g[3] = l * dxy; g[4] = l * dxz; g[5] = l * dyz;
          g[6] = l * dx;  g[7] = l * dy;  g[8] = l * dz;
          g[NT - 1] = l * su[pt];
        }
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        double* o = grad + (leaf * NT + t) * (long long)npts + pt;
        *o = r == 0 ? g[t] : *o + g[t];
      }
    }
  }
}

int coeff_grad_launch(int d, int p, const double* u, const double* lam, const double* D1, const double* D2,
                      long long nl, int nrhs, double* grad, hipStream_t st) {
  const int npts = d == 2 ? p * p : p * p * p;
  const size_t shm = sizeof(double) * (2 * p * p + npts);
  if (d == 2)
    hipLaunchKernelGGL(coeff_grad_kernel<2>, dim3((unsigned)nl), dim3(GRAD_THREADS), shm, st, u, lam, D1, D2, p, nl,
                       nrhs, grad);
  else
    hipLaunchKernelGGL(coeff_grad_kernel<3>, dim3((unsigned)nl), dim3(GRAD_THREADS), shm, st, u, lam, D1, D2, p, nl,
                       nrhs, grad);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

}  // namespace hps
