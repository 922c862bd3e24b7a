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

#include <algorithm>
#include <type_traits>

#include "common.hpp"
#include "../../include/hps.h"

namespace hps {

constexpr int BC_THREADS = 256;
constexpr int BC_UNROLL = 8;  // elements per thread whose loads are in flight together

// Copy (or add) one item: the (row, column) pairs of the item are walked by
// nthr threads, thread t starting at pair t, with one division up front and
// BC_UNROLL elements at a time (all their loads go out before the stores).
template <typename T>
__device__ __forceinline__ void copy_item(const BlockOp* __restrict__ ops, const CopyItem item, long long b,
                                          int ncols_rt, T* __restrict__ dst, long long dst_stride,
                                          const T* __restrict__ src0, long long s0_stride,
                                          const T* __restrict__ src1, long long s1_stride, int nthr, int t) {
  const BlockOp op = ops[item.op];
  const int c0 = item.c0, c1 = item.c1 < 0 ? ncols_rt : item.c1;
  T* D = dst + b * dst_stride + op.dst_off;
  const T* S0 = nullptr;
  const T* S1 = nullptr;
  if (op.nsrc > 0) S0 = (op.src_buf[0] == 0 ? src0 + b * s0_stride : src1 + b * s1_stride) + op.src_off[0];
  if (op.nsrc > 1) S1 = (op.src_buf[1] == 0 ? src0 + b * s0_stride : src1 + b * s1_stride) + op.src_off[1];
  const int rows = item.r1 - item.r0;
  if (rows <= 0 || c1 <= c0) return;
  const int dq = nthr / rows, dr = nthr % rows;
  int r = t % rows, c = c0 + t / rows;
  while (c < c1) {
    int er[BC_UNROLL], ec[BC_UNROLL];
#pragma unroll
    for (int u = 0; u < BC_UNROLL; ++u) {
      er[u] = item.r0 + r;
      ec[u] = c;
      r += dr;
      c += dq;
      if (r >= rows) {
        r -= rows;
        ++c;
      }
    }
    T v[BC_UNROLL];
#pragma unroll
    for (int u = 0; u < BC_UNROLL; ++u) {
      const bool ok = ec[u] < c1;
      const int cu = ok ? ec[u] : c0;  // a valid column for the unused tail
      T x = T(0);
      if (S0) x = S0[er[u] + (long long)cu * op.src_ld[0]];
      if (S1) x += S1[er[u] + (long long)cu * op.src_ld[1]];
      v[u] = x;
    }
#pragma unroll
    for (int u = 0; u < BC_UNROLL; ++u)
      if (ec[u] < c1) D[er[u] + (long long)ec[u] * op.dst_ld] = v[u];
  }
}

// One task: its items one after the other by the whole workgroup, or (small
// items) every fourth item by each wavefront.
template <typename T>
__device__ __forceinline__ void block_copy_body(const BlockOp* __restrict__ ops, const CopyItem* __restrict__ items,
                                                const CopyTask task, long long b, int ncols_rt, T* __restrict__ dst,
                                                long long dst_stride, const T* __restrict__ src0,
                                                long long s0_stride, const T* __restrict__ src1,
                                                long long s1_stride) {
  constexpr int NWAVE = BC_THREADS / 64;
  if (task.per_wave) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int it = task.begin + wave; it < task.end; it += NWAVE)
      copy_item(ops, items[it], b, ncols_rt, dst, dst_stride, src0, s0_stride, src1, s1_stride, 64, lane);
  } else {
    for (int it = task.begin; it < task.end; ++it)
      copy_item(ops, items[it], b, ncols_rt, dst, dst_stride, src0, s0_stride, src1, s1_stride, BC_THREADS,
                (int)threadIdx.x);
  }
}

template <typename T>
__global__ __launch_bounds__(BC_THREADS) void block_copy_kernel(const BlockOp* __restrict__ ops,
                                                                const CopyItem* __restrict__ items,
                                                                const CopyTask* __restrict__ tasks, int ncols_rt,
                                                                T* __restrict__ dst, long long dst_stride,
                                                                const T* __restrict__ src0, long long s0_stride,
                                                                const T* __restrict__ src1, long long s1_stride) {
  block_copy_body(ops, items, tasks[blockIdx.x], blockIdx.y, ncols_rt, dst, dst_stride, src0, s0_stride, src1,
                  s1_stride);
}

int block_copy_launch(const BlockOp* dev_ops, const CopyItem* dev_items, const CopyTask* dev_tasks, int ntasks,
                      int ncols_rt, double* dst, long long dst_stride, const double* src0, long long s0_stride,
                      const double* src1, long long s1_stride, long long batch, hipStream_t st) {
  if (ntasks <= 0 || batch <= 0) return HPS_OK;
  dim3 grid((unsigned)ntasks, (unsigned)batch);
  hipLaunchKernelGGL(block_copy_kernel<double>, grid, dim3(BC_THREADS), 0, st, dev_ops, dev_items, dev_tasks, ncols_rt,
                     dst, dst_stride, src0, s0_stride, src1, s1_stride);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

int block_copy_launch_f32(const BlockOp* dev_ops, const CopyItem* dev_items, const CopyTask* dev_tasks, int ntasks,
                          int ncols_rt, float* dst, long long dst_stride, const float* src0, long long s0_stride,
                          const float* src1, long long s1_stride, long long batch, hipStream_t st) {
  if (ntasks <= 0 || batch <= 0) return HPS_OK;
  dim3 grid((unsigned)ntasks, (unsigned)batch);
  hipLaunchKernelGGL(block_copy_kernel<float>, grid, dim3(BC_THREADS), 0, st, dev_ops, dev_items, dev_tasks, ncols_rt,
                     dst, dst_stride, src0, s0_stride, src1, s1_stride);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

// ---------------------------------------------------------------------------
// leaf_src: v_int[leaf][r][k] = (L_ii^{-1} f_int)[k] for rhs r < nrhs.
// Factor layout (implicit pivoting: row perm[s] is the pivot row of step s,
// pos = perm^{-1}): column s of LU holds, at positions 0 .. s, the U entries
// U(j, s) in pivot order j, and at positions s+1 .. NI-1 the L entries of the
// rows not yet pivoted after step s, in increasing row order.  Row r's L entry
// sits at s + 1 + r - cnt_s(r), cnt_s(r) = #{j <= s : perm[j] < r}.  The
// forward pass reads only the L part of each column and the backward pass only
// the U part, so a solve reads the factor once.
// ---------------------------------------------------------------------------
constexpr int SRC_THREADS = 256;
constexpr int SRC_MAXR = 16;

// Body shared by the single-operator, the batched (cross-operator) and the
// fp32 launches: one wavefront solves one leaf in precision T, so the
// column-by-column substitution needs no workgroup barrier.  Lane l owns rows
// l + 64 i; src(j, k) is the source of rhs j at interior point k (as double);
// the result for rhs j goes to v[j * NI + k].  The LU columns (and pivot
// rows / diagonal entries) of the next PF steps are in flight in a register
// ring, so the step chain does not wait on HBM.
constexpr int SRCW_THREADS = 64;
constexpr int SRC_PF = 2;
constexpr int SRC_STAGE = 8;  // right-hand sides per pass of the pivot-order staging
// src_key(row) gives a row's source key (loaded once per row), src(j, key)
// the source of rhs j.
// MAXR: right-hand-side capacity of the wave (registers b[RPT][MAXR])
template <int RPT, typename T, int MAXR = SRC_MAXR, class SrcKey, class Src>
__device__ __forceinline__ void leaf_src_wave(const T* __restrict__ LU, const int* __restrict__ perm_g,
                                              const int* __restrict__ pos_g, SrcKey src_key, Src src, int NI,
                                              int nrhs, T* __restrict__ v, T* s_y, T* s_stage) {
  constexpr int PF = SRC_PF;
  constexpr int STAGE = MAXR < SRC_STAGE ? MAXR : SRC_STAGE;
  const int lane = threadIdx.x;
  T b[RPT][MAXR];
  int mypos[RPT];
  int permv[RPT];  // perm[lane + 64 i]: any perm entry by readlane, without memory
  int key[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int row = lane + SRCW_THREADS * i;
    mypos[i] = row < NI ? pos_g[row] : -1;
    permv[i] = row < NI ? perm_g[row] : 0;
    key[i] = row < NI ? src_key(row) : 0;
  }
  // the value loads depend only on the keys: all of them go out together
  if constexpr (std::is_same<T, double>::value) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int row = lane + SRCW_THREADS * i;
#pragma unroll
      for (int j = 0; j < MAXR; ++j) b[i][j] = (row < NI && j < nrhs) ? src(j, key[i]) : 0.0;
    }
    // every load above completes here: otherwise the compiler cannot tell,
    // in the step loops, whether b still has loads pending and waits for all
    // outstanding loads (the ring prefetches included) at every step
    __builtin_amdgcn_s_waitcnt(0);
  } else {
    // fp64 values first; the narrowing conversion comes after one wait for
    // all of them (the empty asm keeps it from moving next to each load)
    double b0[RPT][MAXR];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int row = lane + SRCW_THREADS * i;
#pragma unroll
      for (int j = 0; j < MAXR; ++j) b0[i][j] = (row < NI && j < nrhs) ? (double)src(j, key[i]) : 0.0;
    }
    __builtin_amdgcn_s_waitcnt(0);
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
      for (int j = 0; j < MAXR; ++j) {
        __asm__ volatile("" : "+v"(b0[i][j]));
        b[i][j] = (T)b0[i][j];
      }
  }
  auto perm_at = [&](int s) {  // s uniform: readlane of every slot, then a scalar select
    const int l = s % SRCW_THREADS;
    int r = __builtin_amdgcn_readlane(permv[0], l);
#pragma unroll
    for (int i = 1; i < RPT; ++i) {
      const int ri = __builtin_amdgcn_readlane(permv[i], l);
      r = s >= SRCW_THREADS * i ? ri : r;
    }
    return r;
  };
  // The step loops are straight-line code: prefetch loads are unconditional
  // (addresses clamped into the factor) and masked where they are used, and
  // the LDS broadcast relies on the in-order LDS queue of one wavefront, so
  // the compiler can keep the ring's loads in flight across steps.
  T ring[PF][RPT];
  int pring[PF];
  T dring[PF];
  // ---- forward: y_s = b[perm[s]];  b[r] -= L(r, s) y_s for pos[r] > s
  // lidx[i] = sp + 1 + row - #{j <= sp : perm[j] < row}: row i's slot in
  // column sp of the step sp being prefetched (advances by [perm[sp] >= row])
  int lidx[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) lidx[i] = lane + SRCW_THREADS * i;
  auto fetch_l = [&](int u, int sp) {
    const int spc = sp < NI ? sp : NI - 1;
    const int p = perm_at(spc);
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int row = lane + SRCW_THREADS * i;
      lidx[i] += (sp < NI && p >= row) ? 1 : 0;
      ring[u][i] = LU[(long long)spc * NI + min(max(lidx[i], 0), NI - 1)];
    }
    pring[u] = p;
  };
#pragma unroll
  for (int u = 0; u < PF; ++u) fetch_l(u, u);
  for (int s0 = 0; s0 < NI; s0 += PF) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int s = s0 + u;
      const int pr = pring[u];
      if (lane == pr % SRCW_THREADS) {
        const int ip = pr / SRCW_THREADS;
#pragma unroll
        for (int i = 0; i < RPT; ++i)
          if (i == ip)
#pragma unroll
            for (int j = 0; j < MAXR; ++j) s_y[j] = b[i][j];
      }
      __builtin_amdgcn_wave_barrier();
      const bool live = s < NI;  // uniform: the tail of the last group does nothing
      T y[MAXR];
#pragma unroll
      for (int j = 0; j < MAXR; ++j) y[j] = live ? s_y[j] : T(0);
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const T l = mypos[i] > s ? ring[u][i] : T(0);
#pragma unroll
        for (int j = 0; j < MAXR; ++j) b[i][j] -= l * y[j];
      }
      __builtin_amdgcn_wave_barrier();  // s_y is rewritten next step
      fetch_l(u, s + PF);  // refill this slot
    }
  }
  // ---- to pivot order: lane l takes unknowns k = l + 64 i (value of row
  // perm[k]), staged through LDS STAGE right-hand sides at a time
#pragma unroll
  for (int h = 0; h < MAXR; h += STAGE) {
#pragma unroll
    for (int i = 0; i < RPT; ++i)
      if (mypos[i] >= 0)
#pragma unroll
        for (int jj = 0; jj < STAGE; ++jj) s_stage[mypos[i] * STAGE + jj] = b[i][h + jj];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int k = lane + SRCW_THREADS * i;
#pragma unroll
      for (int jj = 0; jj < STAGE; ++jj) b[i][h + jj] = k < NI ? s_stage[k * STAGE + jj] : T(0);
    }
    __builtin_amdgcn_wave_barrier();  // s_stage is rewritten by the next pass
  }
  // ---- backward in pivot order: x_s = b_s / U(s, s);  b_k -= U(k, s) x_s for k < s
  auto fetch_u = [&](int u, int s) {
    const int sc = s >= 0 ? s : 0;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int k = lane + SRCW_THREADS * i;
      ring[u][i] = LU[(long long)sc * NI + min(k, NI - 1)];
    }
    dring[u] = LU[(long long)sc * NI + sc];
  };
#pragma unroll
  for (int u = 0; u < PF; ++u) fetch_u(u, NI - 1 - u);
  for (int s0 = 0; s0 < NI; s0 += PF) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int s = NI - 1 - (s0 + u);
      const bool live = s >= 0;  // uniform
      const int sc = live ? s : 0;
      const T dinv = T(1) / dring[u];
      if (live && lane == sc % SRCW_THREADS) {
        const int ip = sc / SRCW_THREADS;
#pragma unroll
        for (int i = 0; i < RPT; ++i)
          if (i == ip)
#pragma unroll
            for (int j = 0; j < MAXR; ++j) {
              b[i][j] *= dinv;
              s_y[j] = b[i][j];
            }
      }
      __builtin_amdgcn_wave_barrier();
      T y[MAXR];
#pragma unroll
      for (int j = 0; j < MAXR; ++j) y[j] = live ? s_y[j] : T(0);
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int k = lane + SRCW_THREADS * i;
        const T uu = k < s ? ring[u][i] : T(0);
#pragma unroll
        for (int j = 0; j < MAXR; ++j) b[i][j] -= uu * y[j];
      }
      __builtin_amdgcn_wave_barrier();
      fetch_u(u, s - PF);
    }
  }
  // unknown k = lane + 64 i
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int k = lane + SRCW_THREADS * i;
    if (k >= NI) continue;
#pragma unroll
    for (int j = 0; j < MAXR; ++j)
      if (j < nrhs) v[(long long)j * NI + k] = b[i][j];
  }
}

// at least WPE wavefronts per SIMD: the step loop's latency is hidden by
// occupancy more than by a deeper prefetch ring (a ring of 4-8 columns at one
// wavefront per SIMD measured 25 % slower); solves of at most 4 right-hand
// sides use a narrow instance with fewer registers and more waves
template <int RPT, int MAXR, int WPE>
__global__ __launch_bounds__(SRCW_THREADS) __attribute__((amdgpu_waves_per_eu(WPE))) void leaf_src_kernel(const double* __restrict__ LUall,
                                                                const int* __restrict__ permall,
                                                                const int* __restrict__ posall,
                                                                const double* __restrict__ src, const int* __restrict__ Ii,
                                                                int NI, int npts, long long rstride, int nrhs,
                                                                double* __restrict__ vout, int NRcap) {
  constexpr int STAGE = MAXR < SRC_STAGE ? MAXR : SRC_STAGE;
  __shared__ double s_y[MAXR];
  __shared__ double s_stage[RPT * SRCW_THREADS * STAGE];
  const long long leaf = blockIdx.x;
  const double* f = src + leaf * npts;
  auto key = [=](int k) { return Ii[k]; };
  auto at = [=](int j, int ik) { return f[(long long)j * rstride + ik]; };
  leaf_src_wave<RPT, double, MAXR>(LUall + leaf * (long long)NI * NI, permall + leaf * NI, posall + leaf * NI, key, at, NI, nrhs,
                             vout + leaf * (long long)NRcap * NI, s_y, s_stage);
}

// src[r] starts rstride doubles after src[r - 1] (nl * npts for a whole
// operator's sources; larger when the leaves are a slice of a bigger field).
// max_wg_per_cu > 0 caps the workgroups resident per CU (by reserving unused
// LDS), leaving registers and LDS on those CUs for work on another stream.
int leaf_src_launch(const double* LU, const int* perm, const int* pos, const double* src, const int* Ii, int NI,
                    int npts, long long nl, int nrhs, double* v, int NRcap, hipStream_t st, long long rstride,
                    int max_wg_per_cu) {
  constexpr long long kLdsPerCu = 160 * 1024;
  if (rstride <= 0) rstride = nl * npts;
  if (nrhs > SRC_MAXR) {
    set_error("leaf_src: at most 16 right-hand sides per pass");
    return HPS_EINVAL;
  }
  const int rpt = (NI + SRCW_THREADS - 1) / SRCW_THREADS;
  dim3 grid((unsigned)nl), block(SRCW_THREADS);
#define HPS_SRC_LAUNCH(R, M, W)                                                                              \
  do {                                                                                                       \
    size_t shm = 0;                                                                                          \
    hipFuncAttributes fa;                                                                                    \
    if (max_wg_per_cu > 0 && hipFuncGetAttributes(&fa, (const void*)leaf_src_kernel<R, M, W>) == hipSuccess) { \
      const long long want = kLdsPerCu / (max_wg_per_cu + 1) + 256 - (long long)fa.sharedSizeBytes;         \
      shm = want > 0 ? (size_t)want : 0;                                                                     \
    }                                                                                                        \
    hipLaunchKernelGGL((leaf_src_kernel<R, M, W>), grid, block, shm, st, LU, perm, pos, src, Ii, NI, npts,    \
                       rstride, nrhs, v, NRcap);                                                             \
  } while (0)
  if (rpt < 1 || rpt > 4) {
    set_error("leaf_src: too many interior points");
    return HPS_EUNSUPPORTED;
  }
  if (nrhs <= 4) {
    switch (rpt) {
      case 1: HPS_SRC_LAUNCH(1, 4, 4); break;
      case 2: HPS_SRC_LAUNCH(2, 4, 4); break;
      case 3: HPS_SRC_LAUNCH(3, 4, 4); break;
      default: HPS_SRC_LAUNCH(4, 4, 4); break;
    }
  } else {
    switch (rpt) {
      case 1: HPS_SRC_LAUNCH(1, SRC_MAXR, 2); break;
      case 2: HPS_SRC_LAUNCH(2, SRC_MAXR, 2); break;
      case 3: HPS_SRC_LAUNCH(3, SRC_MAXR, 2); break;
      default: HPS_SRC_LAUNCH(4, SRC_MAXR, 2); break;
    }
  }
#undef HPS_SRC_LAUNCH
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

// ---------------------------------------------------------------------------
// leaf_out: u[r][leaf][pt] for rhs r < nrhs
// ---------------------------------------------------------------------------
constexpr int OUT_THREADS = 256;
constexpr int OUT_MAXR = 16;

// Body shared by the single-operator and the batched launches: one
// workgroup per leaf; g holds the leaf's boundary data [rhs][NB] (NRcap
// stride), out(j, pt, value) stores u of rhs j at leaf point pt.
constexpr int OUT_KB = 8;  // Y columns loaded together
template <class Out>
__device__ __forceinline__ void leaf_out_body(const double* __restrict__ Y, const double* __restrict__ P,
                                              const double* __restrict__ g, const double* __restrict__ v,
                                              const int* __restrict__ Ii, const int* __restrict__ Ie, int NI, int NE,
                                              int NB, int npts, int nrhs, Out out, double* s_g) {
  const int tid = threadIdx.x;
  for (int e = tid; e < NB * OUT_MAXR; e += OUT_THREADS) {
    const int c = e / OUT_MAXR, j = e % OUT_MAXR;
    s_g[e] = j < nrhs ? g[(long long)j * NB + c] : 0.0;
  }
  __syncthreads();
  for (int k = tid; k < npts; k += OUT_THREADS) {
    double acc[OUT_MAXR];
#pragma unroll
    for (int j = 0; j < OUT_MAXR; ++j) acc[j] = 0.0;
    int pt;
    if (k < NI) {
      pt = Ii[k];
      // Y loads in batches of OUT_KB, all in flight before their FMAs
      for (int c0 = 0; c0 < NB; c0 += OUT_KB) {
        double yv[OUT_KB];
#pragma unroll
        for (int cc = 0; cc < OUT_KB; ++cc) yv[cc] = c0 + cc < NB ? Y[k + (long long)(c0 + cc) * NI] : 0.0;
#pragma unroll
        for (int cc = 0; cc < OUT_KB; ++cc) {
          const int c = min(c0 + cc, NB - 1);
#pragma unroll
          for (int j = 0; j < OUT_MAXR; ++j) acc[j] += yv[cc] * s_g[c * OUT_MAXR + j];
        }
      }
      if (v) {
        double vv[OUT_MAXR];  // all loads first, then the adds
#pragma unroll
        for (int j = 0; j < OUT_MAXR; ++j) vv[j] = j < nrhs ? v[(long long)j * NI + k] : 0.0;
#pragma unroll
        for (int j = 0; j < OUT_MAXR; ++j) acc[j] += vv[j];
      }
    } else {
      const int e = k - NI;
      pt = Ie[e];
      for (int c0 = 0; c0 < NB; c0 += OUT_KB) {
        double pvv[OUT_KB];
#pragma unroll
        for (int cc = 0; cc < OUT_KB; ++cc) pvv[cc] = c0 + cc < NB ? P[e + (long long)(c0 + cc) * NE] : 0.0;
#pragma unroll
        for (int cc = 0; cc < OUT_KB; ++cc) {
          const int c = min(c0 + cc, NB - 1);
#pragma unroll
          for (int j = 0; j < OUT_MAXR; ++j) acc[j] += pvv[cc] * s_g[c * OUT_MAXR + j];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < OUT_MAXR; ++j)
      if (j < nrhs) out(j, pt, acc[j]);
  }
}

__global__ __launch_bounds__(OUT_THREADS) void leaf_out_kernel(const double* __restrict__ Yall, const double* __restrict__ P,
                                                               const double* __restrict__ gall, const double* __restrict__ vall,
                                                               const int* __restrict__ Ii, const int* __restrict__ Ie,
                                                               int NI, int NE, int NB, int npts, long long rstride, int nrhs,
                                                               int NRcap, double* __restrict__ u) {
  extern __shared__ double s_g[];  // [NB][OUT_MAXR]
  const long long leaf = blockIdx.x;
  double* ul = u + leaf * npts;
  auto out = [=](int j, int pt, double val) { ul[(long long)j * rstride + pt] = val; };
  leaf_out_body(Yall + leaf * (long long)NI * NB, P, gall + leaf * (long long)NRcap * NB,
                vall ? vall + leaf * (long long)NRcap * NI : nullptr, Ii, Ie, NI, NE, NB, npts, nrhs, out, s_g);
}

// u[r] starts rstride doubles after u[r - 1] (0: nl * npts)
int leaf_out_launch(const double* Y, const double* P, const double* g, const double* v, const int* Ii, const int* Ie,
                    int NI, int NE, int NB, int npts, long long nl, int nrhs, int NRcap, double* u, hipStream_t st,
                    long long rstride) {
  if (rstride <= 0) rstride = nl * npts;
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
                     npts, rstride, nrhs, NRcap, u);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}


// ---------------------------------------------------------------------------
// Adjoint (transposed) solve pieces.
// ---------------------------------------------------------------------------
// out[leaf][r][k] = w[r][leaf][idx[k]]  (k < n)
// w[r] starts rstride doubles after w[r - 1] (0: nl * npts)
__global__ void leaf_gather_pts_kernel(const double* __restrict__ w, const int* __restrict__ idx, int n, int npts,
                                       long long rstride, int nrhs, int NRcap, double* __restrict__ out) {
  const long long leaf = blockIdx.y;
  const int r = blockIdx.z;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
    out[(leaf * NRcap + r) * n + k] = w[(long long)r * rstride + leaf * npts + idx[k]];
}

int leaf_gather_pts_launch(const double* w, const int* idx, int n, int npts, long long nl, int nrhs, int NRcap,
                           double* out, hipStream_t st, long long rstride) {
  if (rstride <= 0) rstride = nl * npts;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)nl, (unsigned)nrhs);
  hipLaunchKernelGGL(leaf_gather_pts_kernel, grid, dim3(256), 0, st, w, idx, n, npts, rstride, nrhs, NRcap, out);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

// lam[r][leaf][pt] = interior value fint[leaf][r][k] at pt = Ii[k], 0 at exterior points
// lam[r] starts rstride doubles after lam[r - 1] (0: nl * npts)
__global__ void leaf_scatter_int_kernel(const double* __restrict__ fint, const int* __restrict__ pos_i, int ni,
                                        int npts, long long rstride, int nrhs, int NRcap, double* __restrict__ lam) {
  const long long leaf = blockIdx.y;
  const int r = blockIdx.z;
  for (int pt = blockIdx.x * blockDim.x + threadIdx.x; pt < npts; pt += gridDim.x * blockDim.x) {
    const int k = pos_i[pt];
    lam[(long long)r * rstride + leaf * npts + pt] = k >= 0 ? fint[(leaf * NRcap + r) * ni + k] : 0.0;
  }
}

int leaf_scatter_int_launch(const double* fint, const int* pos_i, int ni, int npts, long long nl, int nrhs, int NRcap,
                            double* lam, hipStream_t st, long long rstride) {
  if (rstride <= 0) rstride = nl * npts;
  dim3 grid((unsigned)((npts + 255) / 256), (unsigned)nl, (unsigned)nrhs);
  hipLaunchKernelGGL(leaf_scatter_int_kernel, grid, dim3(256), 0, st, fint, pos_i, ni, npts, rstride, nrhs, NRcap,
                     lam);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

// Transposed leaf solve  x = L_ii^{-T} b  with the stored factors
// (A = P^T L U,  A^T = U^T L^T P):  U^T y = b (forward), L^T z = y (backward),
// x[perm[k]] = z_k.  b: [leaf][NRcap][NI] in natural interior order (read
// from `bin`); x written to `xout` in the same layout.
template <int RPT>
__global__ __launch_bounds__(SRC_THREADS) void leaf_src_t_kernel(const double* __restrict__ LUall,
                                                                 const int* __restrict__ permall,
                                                                 const double* __restrict__ bin, int NI, int nrhs,
                                                                 int NRcap, double* __restrict__ xout) {
  __shared__ double s_y[2][SRC_MAXR];
  extern __shared__ int s_perm[];
  const long long leaf = blockIdx.x;
  const double* LU = LUall + leaf * (long long)NI * NI;
  const int tid = threadIdx.x;
  for (int i = tid; i < NI; i += SRC_THREADS) s_perm[i] = permall[leaf * NI + i];
  const double* b = bin + leaf * (long long)NRcap * NI;
  double y[RPT][SRC_MAXR];  // thread owns natural indices m = tid + 256 i
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int mm = tid + SRC_THREADS * i;
#pragma unroll
    for (int j = 0; j < SRC_MAXR; ++j) y[i][j] = (mm < NI && j < nrhs) ? b[(long long)j * NI + mm] : 0.0;
  }
  // rows pivoted at steps <= m, as a bit mask over rows, for the thread's
  // natural indices m: L(k, m) sits at m + 1 + rank_m(perm[k]) in column m,
  // rank_m(r) = r - #{pivoted rows below r}
  constexpr int MW = 8;  // NI <= 256
  unsigned pmask[RPT][MW];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int mm = tid + SRC_THREADS * i;
#pragma unroll
    for (int w = 0; w < MW; ++w) pmask[i][w] = 0u;
    for (int j = 0; j <= mm && j < NI; ++j) {
      const int r = s_perm[j];
#pragma unroll
      for (int w = 0; w < MW; ++w)
        if (w == (r >> 5)) pmask[i][w] |= 1u << (r & 31);
    }
  }
  // U^T y = b:  y_k = b_k / U(k,k);  b_m -= U(k, m) y_k  for m > k,  U(k, m) = LU[m * NI + k]
  for (int k = 0; k < NI; ++k) {
    const int buf = k & 1;
    if (tid == k % SRC_THREADS) {
      const double dinv = 1.0 / LU[(long long)k * NI + k];
      const int ik = k / SRC_THREADS;
#pragma unroll
      for (int i = 0; i < RPT; ++i)
        if (i == ik)
#pragma unroll
          for (int j = 0; j < SRC_MAXR; ++j) {
            y[i][j] *= dinv;
            s_y[buf][j] = y[i][j];
          }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int mm = tid + SRC_THREADS * i;
      if (mm > k && mm < NI) {
        const double u = LU[(long long)mm * NI + k];
#pragma unroll
        for (int j = 0; j < SRC_MAXR; ++j) y[i][j] -= u * s_y[buf][j];
      }
    }
  }
  // L^T z = y:  z_k = y_k;  y_m -= L(k, m) z_k  for m < k (L(k, m): row perm[k] in column m)
  for (int k = NI - 1; k >= 0; --k) {
    const int buf = k & 1;
    const int pk = __builtin_amdgcn_readfirstlane(s_perm[k]);
    if (tid == k % SRC_THREADS) {
      const int ik = k / SRC_THREADS;
#pragma unroll
      for (int i = 0; i < RPT; ++i)
        if (i == ik)
#pragma unroll
          for (int j = 0; j < SRC_MAXR; ++j) s_y[buf][j] = y[i][j];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int mm = tid + SRC_THREADS * i;
      if (mm < k) {
        int below = 0;
#pragma unroll
        for (int w = 0; w < MW; ++w) {
          const unsigned bits = w < (pk >> 5) ? pmask[i][w]
                                : (w == (pk >> 5) ? (pmask[i][w] & ((1u << (pk & 31)) - 1u)) : 0u);
          below += __popc(bits);
        }
        const int idx = min(mm + 1 + pk - below, NI - 1);
        const double l = LU[(long long)mm * NI + idx];
#pragma unroll
        for (int j = 0; j < SRC_MAXR; ++j) y[i][j] -= l * s_y[buf][j];
      }
    }
  }
  // x[perm[k]] = z_k (thread of index k holds z_k)
  double* x = xout + leaf * (long long)NRcap * NI;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int k = tid + SRC_THREADS * i;
    if (k >= NI) continue;
    const int pk = s_perm[k];
#pragma unroll
    for (int j = 0; j < SRC_MAXR; ++j)
      if (j < nrhs) x[(long long)j * NI + pk] = y[i][j];
  }
}

int leaf_src_t_launch(const double* LU, const int* perm, const double* b, int NI, long long nl, int nrhs, int NRcap,
                      double* x, hipStream_t st) {
  if (nrhs > SRC_MAXR) {
    set_error("leaf_src_t: at most 16 right-hand sides per pass");
    return HPS_EINVAL;
  }
  if (NI > 256) {
    set_error("leaf_src_t: at most 256 interior points per leaf");
    return HPS_EUNSUPPORTED;
  }
  const size_t shm = NI * sizeof(int);
  const int rpt = (NI + SRC_THREADS - 1) / SRC_THREADS;
  dim3 grid((unsigned)nl), block(SRC_THREADS);
  switch (rpt) {
    case 1: hipLaunchKernelGGL(leaf_src_t_kernel<1>, grid, block, shm, st, LU, perm, b, NI, nrhs, NRcap, x); break;
    case 2: hipLaunchKernelGGL(leaf_src_t_kernel<2>, grid, block, shm, st, LU, perm, b, NI, nrhs, NRcap, x); break;
    default:
      set_error("leaf_src_t: too many interior points");
      return HPS_EUNSUPPORTED;
  }
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

// ---------------------------------------------------------------------------
// Batched solve over several operators (one launch per pass stage).
// ---------------------------------------------------------------------------
template <class J>
__device__ __forceinline__ int find_job(const J* __restrict__ jobs, int njobs, long long blk) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].first_block <= blk) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(BC_THREADS) void block_copy_multi_kernel(const CopyJob* __restrict__ jobs, int njobs) {
  const CopyJob& J = jobs[find_job(jobs, njobs, blockIdx.x)];
  const long long local = blockIdx.x - J.first_block;
  const int task = (int)(local % J.ntasks);
  const long long b = local / J.ntasks;
  block_copy_body(J.ops, J.items, J.tasks[task], b, J.ncols_rt, J.dst, J.dst_stride, J.src0, J.s0_stride, J.src1,
                  J.s1_stride);
}

// root boundary data of every job: g0[j][i] = bdry[j][i]
__global__ __launch_bounds__(BC_THREADS) void root_gather_multi_kernel(const LeafJob* __restrict__ jobs) {
  const LeafJob& J = jobs[blockIdx.z];
  const int j = blockIdx.y;
  if (j >= J.nrhs) return;
  const double* src = J.bdry[0];
#pragma unroll
  for (int k = 1; k < kBatchMaxRhs; ++k)
    if (k == j) src = J.bdry[k];
  for (int i = blockIdx.x * BC_THREADS + threadIdx.x; i < J.nb0; i += gridDim.x * BC_THREADS)
    J.g0[(long long)j * J.nb0 + i] = src[i];
}

__global__ __launch_bounds__(SRCW_THREADS) __attribute__((amdgpu_waves_per_eu(2))) void leaf_src_multi_kernel(const LeafJob* __restrict__ jobs, int njobs) {
  __shared__ double s_y[SRC_MAXR];
  __shared__ double s_stage[4 * SRCW_THREADS * SRC_STAGE];
  const LeafJob& J = jobs[find_job(jobs, njobs, blockIdx.x)];
  const long long leaf = blockIdx.x - J.first_block;
  const int NI = J.NI, npts = J.npts;
  const int* Ii = J.Ii;
  auto key = [&](int k) { return Ii[k]; };
  auto at = [&](int j, int ik) {
    const double* f = J.src[j];
    return f ? f[leaf * npts + ik] : 0.0;
  };
  leaf_src_wave<4, double>(J.LU + leaf * (long long)NI * NI, J.perm + leaf * NI, J.pos + leaf * NI, key, at, NI, J.nrhs,
                           J.v + leaf * (long long)J.NRcap * NI, s_y, s_stage);
}

__global__ __launch_bounds__(OUT_THREADS) void leaf_out_multi_kernel(const LeafJob* __restrict__ jobs, int njobs) {
  extern __shared__ double s_g[];
  const LeafJob& J = jobs[find_job(jobs, njobs, blockIdx.x)];
  const long long leaf = blockIdx.x - J.first_block;
  const int NI = J.NI, NB = J.NB, npts = J.npts;
  auto out = [&](int j, int pt, double val) { J.u[j][leaf * npts + pt] = val; };
  leaf_out_body(J.Y + leaf * (long long)NI * NB, J.P, J.g + leaf * (long long)J.NRcap * NB,
                J.v ? J.v + leaf * (long long)J.NRcap * NI : nullptr, J.Ii, J.Ie, NI, J.NE, NB, npts, J.nrhs, out,
                s_g);
}

int block_copy_multi_launch(const CopyJob* dev_jobs, int njobs, long long nblocks, hipStream_t st) {
  if (njobs <= 0 || nblocks <= 0) return HPS_OK;
  hipLaunchKernelGGL(block_copy_multi_kernel, dim3((unsigned)nblocks), dim3(BC_THREADS), 0, st, dev_jobs, njobs);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

int root_gather_multi_launch(const LeafJob* dev_jobs, int njobs, int max_nb0, hipStream_t st) {
  if (njobs <= 0) return HPS_OK;
  dim3 grid((unsigned)std::min(64, (max_nb0 + BC_THREADS - 1) / BC_THREADS), kBatchMaxRhs, (unsigned)njobs);
  hipLaunchKernelGGL(root_gather_multi_kernel, grid, dim3(BC_THREADS), 0, st, dev_jobs);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

int leaf_src_multi_launch(const LeafJob* dev_jobs, int njobs, long long nblocks, int max_ni, hipStream_t st) {
  if (njobs <= 0 || nblocks <= 0) return HPS_OK;
  if (max_ni > 4 * SRCW_THREADS) {
    set_error("batched solve: at most 256 interior points per leaf");
    return HPS_EUNSUPPORTED;
  }
  hipLaunchKernelGGL(leaf_src_multi_kernel, dim3((unsigned)nblocks), dim3(SRCW_THREADS), 0, st, dev_jobs, njobs);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

int leaf_out_multi_launch(const LeafJob* dev_jobs, int njobs, long long nblocks, int max_nb, hipStream_t st) {
  if (njobs <= 0 || nblocks <= 0) return HPS_OK;
  const size_t shm = (size_t)max_nb * OUT_MAXR * sizeof(double);
  if (shm > 65536) {
    set_error("batched solve: leaf boundary too large");
    return HPS_EUNSUPPORTED;
  }
  hipLaunchKernelGGL(leaf_out_multi_kernel, dim3((unsigned)nblocks), dim3(OUT_THREADS), shm, st, dev_jobs, njobs);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

// ---------------------------------------------------------------------------
// fp32 leaf solve of the refined (mixed-precision) solve: v = L_ii^{-1} r with
// fp32 copies of the LU factors; r is an fp64 interior-point residual
// [leaf][NRcap][NI].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(SRCW_THREADS) __attribute__((amdgpu_waves_per_eu(2))) void leaf_src_f32_kernel(const float* __restrict__ LUall,
                                                                    const int* __restrict__ permall,
                                                                    const int* __restrict__ posall,
                                                                    const double* __restrict__ r, int NI, int nrhs,
                                                                    int NRcap, float* __restrict__ vout) {
  __shared__ float s_y[SRC_MAXR];
  __shared__ float s_stage[4 * SRCW_THREADS * SRC_STAGE];
  const long long leaf = blockIdx.x;
  const double* rl = r + leaf * (long long)NRcap * NI;
  auto key = [](int k) { return k; };
  auto at = [=](int j, int k) { return rl[(long long)j * NI + k]; };
  leaf_src_wave<4, float>(LUall + leaf * (long long)NI * NI, permall + leaf * NI, posall + leaf * NI, key, at, NI, nrhs,
                          vout + leaf * (long long)NRcap * NI, s_y, s_stage);
}

int leaf_src_f32_launch(const float* LU, const int* perm, const int* pos, const double* r, int NI, long long nl,
                        int nrhs, int NRcap, float* v, hipStream_t st) {
  if (nrhs > SRC_MAXR || NI > 4 * SRCW_THREADS) {
    set_error("leaf_src_f32: at most 16 right-hand sides and 256 interior points");
    return HPS_EUNSUPPORTED;
  }
  hipLaunchKernelGGL(leaf_src_f32_kernel, dim3((unsigned)nl), dim3(SRCW_THREADS), 0, st, LU, perm, pos, r, NI, nrhs,
                     NRcap, v);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

}  // namespace hps
