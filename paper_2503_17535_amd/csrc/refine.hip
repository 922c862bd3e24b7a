// Kernels of the mixed-precision (fp32 apply, fp64 residual) solve, 2D.
//
// The iterate is kept in fp64 as (gamma, u_int): gamma = Gauss boundary values
// of every leaf face (the two leaves of a shared panel hold the same values,
// domain-boundary panels hold g exactly) and u_int = u at interior leaf
// points; u at exterior points is always P gamma, so the bordering equations
// of the composite collocation system hold exactly.  One sweep:
//   residual  r1 = f - L u at interior points (collocation rows) and the
//             outgoing flux Q u of every leaf face, in fp64;
//   flux      r3 = Q u_a + Q u_b on every shared panel (flux balance rows),
//             handed to the panel's lower-index leaf as an extra outgoing flux;
//   solve     an fp32 HPS solve of (r1, r3) with zero Dirichlet data, using
//             fp32 copies of the stored operators;
//   update    gamma += delta gamma, u_int += Y delta gamma + v, in fp64.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "../../include/hps.h"

namespace hps {

constexpr int RF_THREADS = 256;
constexpr int RF_MAXP = 16;
constexpr int RF_MAXR = 16;

__global__ void to_f32_kernel(const double* __restrict__ src, float* __restrict__ dst, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

int to_f32_launch(const double* src, float* dst, long long n, hipStream_t st) {
  if (n <= 0) return HPS_OK;
  const long long blocks = std::min<long long>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(to_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, src, dst, n);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

// gamma[leaf][r][face*q + j] = g[r][bidx + j] on domain-boundary faces, 0 elsewhere
__global__ void refine_init_kernel(const double* __restrict__ bdry, const long long* __restrict__ bidx, int q,
                                   int nb0, long long nl, int nrhs, int NRcap, double* __restrict__ gam) {
  const long long leaf = blockIdx.x;
  const int nb = 4 * q;
  for (int e = threadIdx.x; e < nrhs * nb; e += blockDim.x) {
    const int r = e / nb, c = e % nb, f = c / q, j = c % q;
    const long long b = bidx[leaf * 4 + f];
    gam[(leaf * NRcap + r) * nb + c] = b >= 0 ? bdry[(long long)r * nb0 + b + j] : 0.0;
  }
}

int refine_init_launch(const double* bdry, const long long* bidx, int q, int nb0, long long nl, int nrhs, int NRcap,
                       double* gam, hipStream_t st) {
  hipLaunchKernelGGL(refine_init_kernel, dim3((unsigned)nl), dim3(RF_THREADS), 0, st, bdry, bidx, q, nb0, nl, nrhs,
                     NRcap, gam);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

// One workgroup per leaf, all right-hand sides at once (thread work items
// are (rhs, point) pairs):
//   u(I_e) = P gamma (written to u), r1 = f - L u at interior points,
//   Qu = outgoing normal derivative at the Gauss points of every face.
// D1, D2 row-major p x p (scaled to the leaf), P column-major n_e x n_b,
// C2G row-major q x p, coef [leaf][6][p^2].  The mixed derivative is formed
// separably: ux = D1 along x on the whole grid (LDS), then D1 along y of ux.
// D1 and D2 are kept transposed (DxT[a * p + i] = D(i, a)) so that lanes of
// consecutive x index read consecutive LDS words.
struct RfShared {
  double D1[RF_MAXP * RF_MAXP], D2[RF_MAXP * RF_MAXP], D1T[RF_MAXP * RF_MAXP], D2T[RF_MAXP * RF_MAXP];
  double C2G[RF_MAXP * RF_MAXP];
  double u[RF_MAXR][RF_MAXP * RF_MAXP];
  double ux[RF_MAXR][RF_MAXP * RF_MAXP];
  double uy[RF_MAXR][RF_MAXP * RF_MAXP];
  double g[RF_MAXR][4 * RF_MAXP];
  double P[(4 * RF_MAXP - 4) * 4 * (RF_MAXP - 2)];  // Gauss -> Chebyshev boundary interpolation
};

__global__ __launch_bounds__(RF_THREADS) void refine_residual_kernel(
    const double* __restrict__ coef, const double* __restrict__ src, const double* __restrict__ gam,
    const double* __restrict__ D1g, const double* __restrict__ D2g, const double* __restrict__ P,
    const double* __restrict__ C2G, const int* __restrict__ Ii, const int* __restrict__ Ie, int p, long long nl,
    int nrhs, int NRcap, double* __restrict__ u, double* __restrict__ r1, double* __restrict__ Qu) {
  extern __shared__ double smem[];
  RfShared& S = *reinterpret_cast<RfShared*>(smem);
  const int q = p - 2, npts = p * p, ni = q * q, ne = npts - ni, nb = 4 * q;
  const long long leaf = blockIdx.x;
  const int tid = threadIdx.x;
  for (int i = tid; i < p * p; i += RF_THREADS) {
    S.D1[i] = D1g[i];
    S.D2[i] = D2g[i];
    S.D1T[(i % p) * p + i / p] = D1g[i];
    S.D2T[(i % p) * p + i / p] = D2g[i];
  }
  for (int i = tid; i < q * p; i += RF_THREADS) S.C2G[i] = C2G[i];
  for (int i = tid; i < ne * nb; i += RF_THREADS) S.P[i] = P[i];
  for (int e = tid; e < nrhs * nb; e += RF_THREADS) {
    const int r = e / nb, k = e % nb;
    S.g[r][k] = gam[(leaf * NRcap + r) * nb + k];
  }
  // point outer, rhs inner: one index load per point, then the rhs loads together
  for (int k = tid; k < ni; k += RF_THREADS) {
    const int pt = Ii[k];
    double uv[RF_MAXR];
#pragma unroll
    for (int r = 0; r < RF_MAXR; ++r) uv[r] = u[((long long)(r < nrhs ? r : 0) * nl + leaf) * npts + pt];
#pragma unroll
    for (int r = 0; r < RF_MAXR; ++r)
      if (r < nrhs) S.u[r][pt] = uv[r];
  }
  __syncthreads();
  // exterior points: u = P gamma
  for (int e = tid; e < nrhs * ne; e += RF_THREADS) {
    const int r = e / ne, k = e % ne;
    double v = 0.0;
    for (int b = 0; b < nb; ++b) v += S.P[k + b * ne] * S.g[r][b];
    S.u[r][Ie[k]] = v;
    u[((long long)r * nl + leaf) * npts + Ie[k]] = v;
  }
  __syncthreads();
  // ux and uy on the whole grid
  for (int e = tid; e < nrhs * npts; e += RF_THREADS) {
    const int r = e / npts, pt = e % npts, ix = pt % p, iy = pt / p;
    double vx = 0.0, vy = 0.0;
    for (int a = 0; a < p; ++a) {
      vx += S.D1T[a * p + ix] * S.u[r][a + p * iy];
      vy += S.D1[iy * p + a] * S.u[r][ix + p * a];
    }
    S.ux[r][pt] = vx;
    S.uy[r][pt] = vy;
  }
  __syncthreads();
  // collocation residual at interior points: point outer (its coefficients
  // loaded once), rhs inner (the sources loaded together)
  const double* c = coef + leaf * 6 * (long long)npts;
  for (int k = tid; k < ni; k += RF_THREADS) {
    const int pt = Ii[k], ix = pt % p, iy = pt / p;
    const double cxx = c[pt], cxy = c[npts + pt], cyy = c[2 * npts + pt], cx = c[3 * npts + pt],
                 cy = c[4 * npts + pt], c0 = c[5 * npts + pt];
    double fv[RF_MAXR];
#pragma unroll
    for (int r = 0; r < RF_MAXR; ++r) fv[r] = src ? src[((long long)(r < nrhs ? r : 0) * nl + leaf) * npts + pt] : 0.0;
#pragma unroll
    for (int r = 0; r < RF_MAXR; ++r) {
      if (r >= nrhs) continue;
      double dxx = 0.0, dyy = 0.0, dxy = 0.0;
      for (int a = 0; a < p; ++a) {
        dxx += S.D2T[a * p + ix] * S.u[r][a + p * iy];
        dyy += S.D2[iy * p + a] * S.u[r][ix + p * a];
        dxy += S.D1[iy * p + a] * S.ux[r][ix + p * a];
      }
      const double Lu = cxx * dxx + cxy * dxy + cyy * dyy + cx * S.ux[r][pt] + cy * S.uy[r][pt] + c0 * S.u[r][pt];
      r1[(leaf * NRcap + r) * ni + k] = fv[r] - Lu;
    }
  }
  // outgoing fluxes: normal derivative at the face's Chebyshev points (faces
  // S, E, N, W; tangential coordinate ascending), then Chebyshev -> Gauss
  for (int e = tid; e < nrhs * nb; e += RF_THREADS) {
    const int r = e / nb, cg = e % nb, f = cg / q, j = cg % q;
    const int axis = (f == 1 || f == 3) ? 0 : 1;
    const int side = (f == 1 || f == 2) ? 1 : 0;
    const int in = side ? p - 1 : 0;
    double v = 0.0;
    for (int t = 0; t < p; ++t) {
      const double d = axis == 0 ? S.ux[r][in + p * t] : S.uy[r][t + p * in];
      v += S.C2G[j * p + t] * d;
    }
    Qu[(leaf * NRcap + r) * nb + cg] = side ? v : -v;
  }
}

int refine_residual_launch(const double* coef, const double* src, const double* gam, const double* D1,
                           const double* D2, const double* P, const double* C2G, const int* Ii, const int* Ie, int p,
                           long long nl, int nrhs, int NRcap, double* u, double* r1, double* Qu, hipStream_t st) {
  if (p > RF_MAXP || nrhs > RF_MAXR) {
    set_error("refined solve: p <= 16 and at most 16 right-hand sides per pass");
    return HPS_EUNSUPPORTED;
  }
  const size_t shm = sizeof(RfShared);
  static bool attr = false;
  if (!attr) {
    HPS_HIP_TRY(hipFuncSetAttribute((const void*)refine_residual_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)shm));
    attr = true;
  }
  hipLaunchKernelGGL(refine_residual_kernel, dim3((unsigned)nl), dim3(RF_THREADS), shm, st, coef, src, gam, D1, D2, P,
                     C2G, Ii, Ie, p, nl, nrhs, NRcap, u, r1, Qu);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

// Flux imbalance of every shared panel, handed to its lower-index leaf:
// hx[leaf][r][f*q + j] = Qu[leaf][r][f*q + j] + Qu[nbr][r][f'*q + j] (owner) or 0.
__global__ void refine_flux_kernel(const double* __restrict__ Qu, const int* __restrict__ nbr, int q, long long nl,
                                   int nrhs, int NRcap, float* __restrict__ hx) {
  const long long leaf = blockIdx.x;
  const int nb = 4 * q;
  for (int e = threadIdx.x; e < nrhs * nb; e += blockDim.x) {
    const int r = e / nb, c = e % nb, f = c / q, j = c % q;
    const int o = nbr[leaf * 4 + f];  // neighbour leaf * 4 + its face, or -1
    double v = 0.0;
    if (o >= 0 && (long long)(o / 4) > leaf)
      v = Qu[(leaf * NRcap + r) * nb + c] + Qu[((long long)(o / 4) * NRcap + r) * nb + (o % 4) * q + j];
    hx[(leaf * NRcap + r) * nb + c] = (float)v;
  }
}

int refine_flux_launch(const double* Qu, const int* nbr, int q, long long nl, int nrhs, int NRcap, float* hx,
                       hipStream_t st) {
  hipLaunchKernelGGL(refine_flux_kernel, dim3((unsigned)nl), dim3(RF_THREADS), 0, st, Qu, nbr, q, nl, nrhs, NRcap, hx);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

// gamma += dg;  u(I_i) += Y dg + v   (dg = fp32 leaf boundary data of the
// correction solve, Y fp32 [leaf][n_i x n_b] column-major, v fp32 [leaf][r][n_i])
__global__ __launch_bounds__(RF_THREADS) void refine_update_kernel(const float* __restrict__ dg_all,
                                                                   const float* __restrict__ Y32,
                                                                   const float* __restrict__ v32,
                                                                   const int* __restrict__ Ii, int ni, int nb,
                                                                   int npts, long long nl, int nrhs, int NRcap,
                                                                   double* __restrict__ gam, double* __restrict__ u) {
  __shared__ float sdg[4 * RF_MAXP * RF_MAXR];  // [nb][RF_MAXR]
  const long long leaf = blockIdx.x;
  const int tid = threadIdx.x;
  const float* dg = dg_all + leaf * (long long)NRcap * nb;
  for (int e = tid; e < nb * RF_MAXR; e += RF_THREADS) {
    const int c = e / RF_MAXR, j = e % RF_MAXR;
    const float x = j < nrhs ? dg[(long long)j * nb + c] : 0.0f;
    sdg[e] = x;
    if (j < nrhs) gam[(leaf * NRcap + j) * nb + c] += (double)x;
  }
  __syncthreads();
  const float* Y = Y32 + leaf * (long long)ni * nb;
  const float* v = v32 + leaf * (long long)NRcap * ni;
  for (int k = tid; k < ni; k += RF_THREADS) {
    float acc[RF_MAXR];
#pragma unroll
    for (int j = 0; j < RF_MAXR; ++j) acc[j] = 0.0f;
    // Y columns in batches of 8, all loads in flight before their FMAs
    for (int c0 = 0; c0 < nb; c0 += 8) {
      float yv[8];
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) yv[cc] = c0 + cc < nb ? Y[k + (long long)(c0 + cc) * ni] : 0.0f;
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) {
        const int c = min(c0 + cc, nb - 1);
#pragma unroll
        for (int j = 0; j < RF_MAXR; ++j) acc[j] += yv[cc] * sdg[c * RF_MAXR + j];
      }
    }
    const int pt = Ii[k];
    // loads of v and u (clamped to a valid rhs) together, then the updates
    float vv[RF_MAXR];
    double uo[RF_MAXR];
#pragma unroll
    for (int j = 0; j < RF_MAXR; ++j) {
      const int jj = j < nrhs ? j : 0;
      vv[j] = v[(long long)jj * ni + k];
      uo[j] = u[((long long)jj * nl + leaf) * npts + pt];
    }
#pragma unroll
    for (int j = 0; j < RF_MAXR; ++j)
      if (j < nrhs) u[((long long)j * nl + leaf) * npts + pt] = uo[j] + (double)(acc[j] + vv[j]);
  }
}

int refine_update_launch(const float* dg, const float* Y32, const float* v32, const int* Ii, int ni, int nb, int npts,
                         long long nl, int nrhs, int NRcap, double* gam, double* u, hipStream_t st) {
  if (nb > 4 * RF_MAXP || nrhs > RF_MAXR) {
    set_error("refined solve: leaf boundary too large");
    return HPS_EUNSUPPORTED;
  }
  hipLaunchKernelGGL(refine_update_kernel, dim3((unsigned)nl), dim3(RF_THREADS), 0, st, dg, Y32, v32, Ii, ni, nb, npts,
                     nl, nrhs, NRcap, gam, u);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

}  // namespace hps
