// Gathers and leaf-level kernels of the build and the solve.
//
// * block_copy: a table of (rows x cols) block copies / two-block sums between
//   per-node buffers.  It assembles the merge matrices D (sums of child DtN
//   blocks on shared interfaces, Appendix A.2 / C.2), the A-part of the parent
//   DtN matrix, the nonzero blocks of B kept for the solve, and in the solve
//   the interface data h_int (sums of the two children's outgoing data) and the
//   children's incoming data cut from [g_ext; g_int] (Algorithm "Downward
//   pass").
// * leaf_src: the particular solution of each leaf, v_int = L_ii^{-1} f_int,
//   by forward/back substitution with the stored LU factors (implicit row
//   order), for several right-hand sides at once.
// * leaf_out: u = Y g + v at the leaves (Algorithm "Downward pass", last loop),
//   with Y = [I; Y_int] P written out as  u(I_e) = P g,  u(I_i) = Y_int g + v.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "../../include/hps.h"

namespace hps {

constexpr int BC_THREADS = 256;

__global__ __launch_bounds__(BC_THREADS) void block_copy_kernel(const BlockOp* __restrict__ ops,
                                                                const CopyItem* __restrict__ items,
                                                                const CopyTask* __restrict__ tasks, int ncols_rt,
                                                                double* __restrict__ dst, long long dst_stride,
                                                                const double* __restrict__ src0, long long s0_stride,
                                                                const double* __restrict__ src1, long long s1_stride) {
  const CopyTask task = tasks[blockIdx.x];
  const long long b = blockIdx.y;
  for (int it = task.begin; it < task.end; ++it) {
    const CopyItem item = items[it];
    const BlockOp op = ops[item.op];
    const int c0 = item.c0, c1 = item.c1 < 0 ? ncols_rt : item.c1;
    double* D = dst + b * dst_stride + op.dst_off;
    const double* S0 = nullptr;
    const double* S1 = nullptr;
    if (op.nsrc > 0) S0 = (op.src_buf[0] == 0 ? src0 + b * s0_stride : src1 + b * s1_stride) + op.src_off[0];
    if (op.nsrc > 1) S1 = (op.src_buf[1] == 0 ? src0 + b * s0_stride : src1 + b * s1_stride) + op.src_off[1];
    const int rows = op.rows;
    const int n = rows * (c1 - c0);
    for (int e = threadIdx.x; e < n; e += BC_THREADS) {
      const int r = e % rows, c = c0 + e / rows;
      double v = 0.0;
      if (S0) v = S0[r + (long long)c * op.src_ld[0]];
      if (S1) v += S1[r + (long long)c * op.src_ld[1]];
      D[r + (long long)c * op.dst_ld] = v;
    }
  }
}

int block_copy_launch(const BlockOp* dev_ops, const CopyItem* dev_items, const CopyTask* dev_tasks, int ntasks,
                      int ncols_rt, double* dst, long long dst_stride, const double* src0, long long s0_stride,
                      const double* src1, long long s1_stride, long long batch, hipStream_t st) {
  if (ntasks <= 0 || batch <= 0) return HPS_OK;
  dim3 grid((unsigned)ntasks, (unsigned)batch);
  hipLaunchKernelGGL(block_copy_kernel, grid, dim3(BC_THREADS), 0, st, dev_ops, dev_items, dev_tasks, ncols_rt, dst,
                     dst_stride, src0, s0_stride, src1, s1_stride);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

// ---------------------------------------------------------------------------
// leaf_src: v_int[leaf][r][k] = (L_ii^{-1} f_int)[k] for rhs r < nrhs.
// LU is stored with rows in original order: row perm[s] is the pivot row of
// step s; a row r with pos[r] > s holds L(r, s) in column s, a row with
// pos[r] <= s holds U(pos[r], s).
// ---------------------------------------------------------------------------
constexpr int SRC_THREADS = 256;
constexpr int SRC_MAXR = 16;

template <int RPT>
__global__ __launch_bounds__(SRC_THREADS) void leaf_src_kernel(const double* __restrict__ LUall,
                                                               const int* __restrict__ permall,
                                                               const int* __restrict__ posall,
                                                               const double* __restrict__ src, const int* __restrict__ Ii,
                                                               int NI, int npts, long long nl, int nrhs,
                                                               double* __restrict__ vout, int NRcap) {
  __shared__ double s_y[2][SRC_MAXR];
  extern __shared__ int s_int[];  // perm[NI], pos[NI]
  int* s_perm = s_int;
  int* s_pos = s_int + NI;
  const long long leaf = blockIdx.x;
  const double* LU = LUall + leaf * (long long)NI * NI;
  const int tid = threadIdx.x;
  for (int i = tid; i < NI; i += SRC_THREADS) {
    s_perm[i] = permall[leaf * NI + i];
    s_pos[i] = posall[leaf * NI + i];
  }
  double b[RPT][SRC_MAXR];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int row = tid + SRC_THREADS * i;
#pragma unroll
    for (int j = 0; j < SRC_MAXR; ++j)
      b[i][j] = (row < NI && j < nrhs) ? src[(long long)j * nl * npts + leaf * npts + Ii[row]] : 0.0;
  }
  __syncthreads();
  int mypos[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int row = tid + SRC_THREADS * i;
    mypos[i] = row < NI ? s_pos[row] : -1;
  }
  // forward: y_s = b[perm[s]];  b[r] -= L(r, s) y_s for pos[r] > s
  for (int s = 0; s < NI; ++s) {
    const int buf = s & 1;
    const int pr = __builtin_amdgcn_readfirstlane(s_perm[s]);  // uniform: scalar branches below
    if (tid == pr % SRC_THREADS) {
      const int ip = pr / SRC_THREADS;
#pragma unroll
      for (int i = 0; i < RPT; ++i)
        if (i == ip)
#pragma unroll
          for (int j = 0; j < SRC_MAXR; ++j) s_y[buf][j] = b[i][j];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int row = tid + SRC_THREADS * i;
      if (row < NI && mypos[i] > s) {
        const double l = LU[row + (long long)s * NI];
#pragma unroll
        for (int j = 0; j < SRC_MAXR; ++j) b[i][j] -= l * s_y[buf][j];
      }
    }
  }
  // backward: x_s = b[perm[s]] / U(s, s);  b[r] -= U(pos[r], s) x_s for pos[r] < s
  for (int s = NI - 1; s >= 0; --s) {
    const int buf = s & 1;
    const int pr = __builtin_amdgcn_readfirstlane(s_perm[s]);  // uniform: scalar branches below
    if (tid == pr % SRC_THREADS) {
      const int ip = pr / SRC_THREADS;
      const double dinv = 1.0 / LU[pr + (long long)s * NI];
#pragma unroll
      for (int i = 0; i < RPT; ++i)
        if (i == ip)
#pragma unroll
          for (int j = 0; j < SRC_MAXR; ++j) {
            b[i][j] *= dinv;
            s_y[buf][j] = b[i][j];
          }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int row = tid + SRC_THREADS * i;
      if (row < NI && mypos[i] < s) {
        const double u = LU[row + (long long)s * NI];
#pragma unroll
        for (int j = 0; j < SRC_MAXR; ++j) b[i][j] -= u * s_y[buf][j];
      }
    }
  }
  // unknown pos[r] sits in row r
  double* v = vout + leaf * (long long)NRcap * NI;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int row = tid + SRC_THREADS * i;
    if (row >= NI) continue;
#pragma unroll
    for (int j = 0; j < SRC_MAXR; ++j)
      if (j < nrhs) v[(long long)j * NI + mypos[i]] = b[i][j];
  }
}

int leaf_src_launch(const double* LU, const int* perm, const int* pos, const double* src, const int* Ii, int NI,
                    int npts, long long nl, int nrhs, double* v, int NRcap, hipStream_t st) {
  if (nrhs > SRC_MAXR) {
    set_error("leaf_src: at most 16 right-hand sides per pass");
    return HPS_EINVAL;
  }
  const size_t shm = 2 * NI * sizeof(int);
  const int rpt = (NI + SRC_THREADS - 1) / SRC_THREADS;
  dim3 grid((unsigned)nl), block(SRC_THREADS);
  switch (rpt) {
    case 1: hipLaunchKernelGGL(leaf_src_kernel<1>, grid, block, shm, st, LU, perm, pos, src, Ii, NI, npts, nl, nrhs, v, NRcap); break;
    case 2: hipLaunchKernelGGL(leaf_src_kernel<2>, grid, block, shm, st, LU, perm, pos, src, Ii, NI, npts, nl, nrhs, v, NRcap); break;
    case 3: hipLaunchKernelGGL(leaf_src_kernel<3>, grid, block, shm, st, LU, perm, pos, src, Ii, NI, npts, nl, nrhs, v, NRcap); break;
    case 4: hipLaunchKernelGGL(leaf_src_kernel<4>, grid, block, shm, st, LU, perm, pos, src, Ii, NI, npts, nl, nrhs, v, NRcap); break;
    default:
      set_error("leaf_src: too many interior points");
      return HPS_EUNSUPPORTED;
  }
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

// ---------------------------------------------------------------------------
// leaf_out: u[r][leaf][pt] for rhs r < nrhs
// ---------------------------------------------------------------------------
constexpr int OUT_THREADS = 256;
constexpr int OUT_MAXR = 16;

__global__ __launch_bounds__(OUT_THREADS) void leaf_out_kernel(const double* __restrict__ Yall, const double* __restrict__ P,
                                                               const double* __restrict__ gall, const double* __restrict__ vall,
                                                               const int* __restrict__ Ii, const int* __restrict__ Ie,
                                                               int NI, int NE, int NB, int npts, long long nl, int nrhs,
                                                               int NRcap, double* __restrict__ u) {
  extern __shared__ double s_g[];  // [NB][OUT_MAXR]
  const long long leaf = blockIdx.x;
  const int tid = threadIdx.x;
  const double* g = gall + leaf * (long long)NRcap * NB;
  for (int e = tid; e < NB * OUT_MAXR; e += OUT_THREADS) {
    const int c = e / OUT_MAXR, j = e % OUT_MAXR;
    s_g[e] = j < nrhs ? g[(long long)j * NB + c] : 0.0;
  }
  __syncthreads();
  const double* Y = Yall + leaf * (long long)NI * NB;
  const double* v = vall ? vall + leaf * (long long)NRcap * NI : nullptr;
  for (int k = tid; k < npts; k += OUT_THREADS) {
    double acc[OUT_MAXR];
#pragma unroll
    for (int j = 0; j < OUT_MAXR; ++j) acc[j] = 0.0;
    int pt;
    if (k < NI) {
      pt = Ii[k];
      for (int c = 0; c < NB; ++c) {
        const double y = Y[k + (long long)c * NI];
#pragma unroll
        for (int j = 0; j < OUT_MAXR; ++j) acc[j] += y * s_g[c * OUT_MAXR + j];
      }
      if (v)
#pragma unroll
        for (int j = 0; j < OUT_MAXR; ++j)
          if (j < nrhs) acc[j] += v[(long long)j * NI + k];
    } else {
      const int e = k - NI;
      pt = Ie[e];
      for (int c = 0; c < NB; ++c) {
        const double pv = P[e + (long long)c * NE];
#pragma unroll
        for (int j = 0; j < OUT_MAXR; ++j) acc[j] += pv * s_g[c * OUT_MAXR + j];
      }
    }
#pragma unroll
    for (int j = 0; j < OUT_MAXR; ++j)
      if (j < nrhs) u[(long long)j * nl * npts + leaf * npts + pt] = acc[j];
  }
}

int leaf_out_launch(const double* Y, const double* P, const double* g, const double* v, const int* Ii, const int* Ie,
                    int NI, int NE, int NB, int npts, long long nl, int nrhs, int NRcap, double* u, hipStream_t st) {
  if (nrhs > OUT_MAXR) {
    set_error("leaf_out: at most 16 right-hand sides per pass");
    return HPS_EINVAL;
  }
  const size_t shm = (size_t)NB * OUT_MAXR * sizeof(double);
  if (shm > 65536) {
    if (shm > 160 * 1024) {
      set_error("leaf_out: boundary too large for LDS staging");
      return HPS_EUNSUPPORTED;
    }
    HPS_HIP_TRY(hipFuncSetAttribute((const void*)leaf_out_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
  }
  hipLaunchKernelGGL(leaf_out_kernel, dim3((unsigned)nl), dim3(OUT_THREADS), shm, st, Y, P, g, v, Ii, Ie, NI, NE, NB,
                     npts, nl, nrhs, NRcap, u);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

}  // namespace hps
