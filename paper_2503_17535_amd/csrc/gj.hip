// Inversion of the merge matrices D (Algorithm "Merge stage": "Invert D").
//
// Gauss-Jordan elimination with implicit partial pivoting: rows never move;
// at step k the pivot of column k is the unused row p_k of largest |D(r, k)|
// (ties: lowest row), and the in-place update replaces column k by the k-th
// column of the accumulated elimination operator.  With R the in-place result
// and pos = p^{-1}, the inverse is  D^{-1}(a, b) = R(p_a, pos_b).
//
// Two forms:
//  * gj_small: one workgroup per matrix, the whole matrix in registers
//    (cyclic TR x TC thread grid, the pivot column rotated into slot 0), for
//    m <= 224 (used for the many small merges near the leaves, and for large
//    batches such as 3D leaves);
//  * blocked: per panel of NB columns one workgroup per matrix factors the
//    panel with the panel's rows in registers, while the other workgroups of
//    the same launch apply the previous panel's rank-NB update to every other
//    column (each workgroup owns whole columns); a final gather unscrambles
//    rows and columns.  Used for the few large merges near the root.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "common.hpp"
#include "dpp.hpp"
#include "../../include/hps.h"

namespace hps {

// ---------------------------------------------------------------------------
// gj_small
// ---------------------------------------------------------------------------
template <int TR, int TC, int RI, int RJ>
__global__ __launch_bounds__(TR* TC) void gj_small_kernel(const double* __restrict__ Din, double* __restrict__ Zout,
                                                           int m, int* __restrict__ flag) {
  constexpr int NT = TR * TC;
  // the pivot chain is the critical path: its waves win instruction issue over
  // other work resident on the same SIMD (another stream's kernels)
  __builtin_amdgcn_s_setprio(3);
  static_assert(64 % TR == 0, "a column group of TR lanes lies inside one wavefront");
  static_assert(RI * TR <= 255, "row rank codes fit in the 8 low bits of a pivot key");
  __shared__ double s_lcol[2][RI * TR];
  __shared__ double s_urow[2][RJ * TC];
  __shared__ int s_perm[RJ * TC], s_pos[RI * TR];
  __shared__ int s_piv[2];
  __shared__ double s_pinv[2];

  const long long b = blockIdx.x;
  const double* D = Din + b * (long long)m * m;
  double* Z = Zout + b * (long long)m * m;
  const int tid = threadIdx.x;
  const int tr = tid % TR, tc = tid / TR;
  const int lane = tid & 63;
  const int gbase = lane - tr;

  for (int i = tid; i < RI * TR; i += NT) s_pos[i] = -1;
  double a[RI][RJ];
#pragma unroll
  for (int ri = 0; ri < RI; ++ri)
#pragma unroll
    for (int s = 0; s < RJ; ++s) {
      const int row = tr + TR * ri, col = tc + TC * s;
      a[ri][s] = (row < m && col < m) ? D[row + (long long)col * m] : 0.0;
    }
  unsigned used = 0;
#pragma unroll
  for (int ri = 0; ri < RI; ++ri)
    if (tr + TR * ri >= m) used |= 1u << ri;
  __syncthreads();

  // slot s holds column block (kb + s) mod RJ during block kb
  for (int kb = 0; kb < RJ; ++kb) {
    for (int t = 0; t < TC; ++t) {
      const int k = kb * TC + t;
      if (k >= m) break;
      const int buf = k & 1;
      if (tc == t) {
        // pivot search: unsigned max of packed keys (pivot_key32_c8), ties
        // to the lower row; the pivot value comes from its lane by readlane
        unsigned key = 0;
#pragma unroll
        for (int ri = 0; ri < RI; ++ri) {
          const unsigned kk = pivot_key32_c8(a[ri][0], 255 - tr - TR * ri);
          key = max(key, ((used >> ri) & 1u) ? 0u : kk);
        }
        key = group_max<TR>(key);
        const int brow = __builtin_amdgcn_readfirstlane(255 - (int)(key & 255u));  // uniform in the group
        const int bri = brow / TR, btr = brow % TR;
        double v = 0.0;
#pragma unroll
        for (int ri = 0; ri < RI; ++ri)
          if (ri == bri) v = a[ri][0];
        const double pv = readlane_d(v, __builtin_amdgcn_readfirstlane(gbase) + btr);
        const double pinv = recip_nr(pv);
#pragma unroll
        for (int ri = 0; ri < RI; ++ri)
          s_lcol[buf][tr + TR * ri] = (ri == bri && tr == btr) ? 0.0 : a[ri][0];
        if (tr == 0) {
          s_piv[buf] = brow;
          s_pinv[buf] = pinv;
          s_perm[k] = brow;
          s_pos[brow] = k;
          if (!(pv != 0.0) || !isfinite(pv) || !isfinite(pinv)) atomicOr(flag, 2);
        }
      }
      __syncthreads();
      const int pr = __builtin_amdgcn_readfirstlane(s_piv[buf]);  // uniform: scalar branches below
      if (tr == pr % TR) {
        const int rip = pr / TR;  // uniform: one scalar branch is taken
        used |= 1u << rip;
        const double pinv = s_pinv[buf];
#pragma unroll
        for (int ri = 0; ri < RI; ++ri)
          if (ri == rip) {
#pragma unroll
            for (int s = 0; s < RJ; ++s) {
              const double v = ((s == 0 && tc == t) ? 1.0 : a[ri][s]) * pinv;
              a[ri][s] = v;
              s_urow[buf][tc + TC * s] = v;
            }
          }
      }
      // s_urow entries of column tc + TC*s are read only by this thread's
      // column group (TR lanes of one wavefront): a wavefront-level barrier
      // orders the owner's LDS write before their reads
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // multipliers of this thread's rows, read once per step (the pivot
      // row's entry is 0, so the update leaves that row unchanged)
      double lc[RI];
#pragma unroll
      for (int ri = 0; ri < RI; ++ri) lc[ri] = s_lcol[buf][tr + TR * ri];
#pragma unroll
      for (int s = 0; s < RJ; ++s) {
        const double u = s_urow[buf][tc + TC * s];
        if (s == 0 && tc == t) {
          // column k becomes the k-th column of the elimination operator
#pragma unroll
          for (int ri = 0; ri < RI; ++ri)
            if (tr + TR * ri != pr) a[ri][0] = -lc[ri] * u;
        } else {
#pragma unroll
          for (int ri = 0; ri < RI; ++ri) a[ri][s] -= lc[ri] * u;
        }
      }
    }
    // rotate slots left cyclically
#pragma unroll
    for (int ri = 0; ri < RI; ++ri) {
      const double first = a[ri][0];
#pragma unroll
      for (int s = 0; s + 1 < RJ; ++s) a[ri][s] = a[ri][s + 1];
      a[ri][RJ - 1] = first;
    }
  }
  __syncthreads();
  // Z(pos[row], perm[col]) = R(row, col)
#pragma unroll
  for (int ri = 0; ri < RI; ++ri) {
    const int row = tr + TR * ri;
    if (row >= m) continue;
    const int zr = s_pos[row];
#pragma unroll
    for (int s = 0; s < RJ; ++s) {
      const int col = tc + TC * s;
      if (col < m) Z[zr + (long long)s_perm[col] * m] = a[ri][s];
    }
  }
}

template <int RI>
static void launch_gj_small_ri(const double* D, double* Z, int m, int* flag, long long batch, hipStream_t st) {
  constexpr int RJ = (RI + 1) / 2;
  hipLaunchKernelGGL((gj_small_kernel<16, 32, RI, RJ>), dim3((unsigned)batch), dim3(512), 0, st, D, Z, m, flag);
}

int gj_small_max() { return 224; }

int gj_small_launch(const double* D, double* Z, int m, int* flag, long long batch, hipStream_t st) {
  const int ri = (m + 15) / 16;
  switch (ri) {
    case 1: launch_gj_small_ri<1>(D, Z, m, flag, batch, st); break;
    case 2: launch_gj_small_ri<2>(D, Z, m, flag, batch, st); break;
    case 3: launch_gj_small_ri<3>(D, Z, m, flag, batch, st); break;
    case 4: launch_gj_small_ri<4>(D, Z, m, flag, batch, st); break;
    case 5: launch_gj_small_ri<5>(D, Z, m, flag, batch, st); break;
    case 6: launch_gj_small_ri<6>(D, Z, m, flag, batch, st); break;
    case 7: launch_gj_small_ri<7>(D, Z, m, flag, batch, st); break;
    case 8: launch_gj_small_ri<8>(D, Z, m, flag, batch, st); break;
    case 9: launch_gj_small_ri<9>(D, Z, m, flag, batch, st); break;
    case 10: launch_gj_small_ri<10>(D, Z, m, flag, batch, st); break;
    case 11: launch_gj_small_ri<11>(D, Z, m, flag, batch, st); break;
    case 12: launch_gj_small_ri<12>(D, Z, m, flag, batch, st); break;
    case 13: launch_gj_small_ri<13>(D, Z, m, flag, batch, st); break;
    case 14: launch_gj_small_ri<14>(D, Z, m, flag, batch, st); break;
    default:
      set_error("gj_small: m too large");
      return HPS_EUNSUPPORTED;
  }
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

// ---------------------------------------------------------------------------
// blocked form
// ---------------------------------------------------------------------------
constexpr int PANEL_THREADS = 512;
constexpr int PANEL_MAX_NB = 16;
constexpr int GU_COLS = 8;  // columns per workgroup of the update
constexpr int GU_KC = 8;    // panel columns per chunk of W loads in the update

// Initialize the pivot bookkeeping of a batch (pos = -1).
__global__ void gj_init_kernel(int* pos, long long n) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) pos[i] = -1;
}

// Compile-time loop: f(integral_constant<int, I>) for I = B .. E-1.
template <int B, int E, class F>
__device__ __forceinline__ void gj_static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    gj_static_for<B + 1, E>(f);
  }
}

// bits of a row rank code for n rows: codes 2^b - 1 - row stay >= 1
constexpr int rank_code_bits(int n) { return n < 256 ? 8 : 1 + rank_code_bits(n / 2); }

// One Gauss-Jordan panel: columns [j0, j0+nbw) of every row, rows
// distributed cyclically over the workgroup (row = tid + 512 i), in registers.
// The column loop is expanded at compile time, so panel column c stays in
// register slot c.  Per column: each wavefront finds its best unused row
// (packed keys, pivot_key32) and publishes that row's panel entries already
// scaled by its own reciprocal pivot; one barrier; every thread takes the
// best of the NW candidates and applies the rank-1 Gauss-Jordan update.
template <int RPT, int NB>
__device__ __forceinline__ void gj_panel_body(double* __restrict__ A, int m, int j0, int nbw, int* __restrict__ pos,
                                              int* __restrict__ piv, double* __restrict__ W, int* __restrict__ flag,
                                              const double* __restrict__ Wp = nullptr, int jp = 0, int wp = 0) {
  constexpr int NW = PANEL_THREADS / 64;
  constexpr int CB = rank_code_bits(RPT * PANEL_THREADS);
  constexpr int CMAX = (1 << CB) - 1;
  static_assert(CB <= 16, "row codes fit a pivot key");
  __shared__ unsigned s_key[2][NW];
  __shared__ double s_cpinv[2][NW];
  __shared__ double s_cand[2][NW][NB];  // each wavefront's candidate pivot row, scaled
  __shared__ int s_piv[NB];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  // With Wp: the previous panel's update of this panel's columns is applied
  // here, in registers, in the same order of operations as the update of the
  // other columns (gj_update_body), instead of a store and reload.  Its
  // factors are the previous panel's pivot rows of these columns (old
  // values), which this workgroup already holds: the row whose pos is jp + k
  // publishes row k.  The panel, pos and the first chunk of W are loaded
  // together, so the step waits for memory once before its first pivot.
  __shared__ double s_pp[PANEL_MAX_NB][PANEL_MAX_NB];  // old pivot rows of the previous panel
  constexpr int KC = RPT >= 16 ? 1 : (RPT >= 8 ? 2 : (RPT >= 4 ? 4 : GU_KC));  // W rows per chunk
  static_assert(GU_KC % KC == 0, "W chunks tile the padded panel width");
  const int wpad = Wp ? (wp + GU_KC - 1) / GU_KC * GU_KC : 0;
  double a[RPT][NB];
  int pv[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int row = tid + PANEL_THREADS * i;
#pragma unroll
    for (int c = 0; c < NB; ++c)
      a[i][c] = (row < m && c < nbw) ? A[row + (long long)(j0 + c) * m] : 0.0;
    pv[i] = row < m ? pos[row] : -1;
  }
  double w[KC][RPT];
  if (Wp) {
#pragma unroll
    for (int k = 0; k < KC; ++k)
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int row = tid + PANEL_THREADS * i;
        w[k][i] = (row < m && k < wp) ? Wp[row + (long long)k * m] : 0.0;
      }
  }
  unsigned used = 0;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int row = tid + PANEL_THREADS * i;
    if (row >= m || pv[i] >= 0) used |= 1u << i;
  }
  if (Wp) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int row = tid + PANEL_THREADS * i;
      const int k = pv[i] - jp;
      if (row < m && k >= 0 && k < wp) {
#pragma unroll
        for (int c = 0; c < NB; ++c) s_pp[k][c] = a[i][c];
      }
    }
    for (int e = tid; e < (wpad - wp) * NB; e += PANEL_THREADS) s_pp[wp + e / NB][e % NB] = 0.0;
    __syncthreads();
    for (int k0 = 0; k0 < wpad; k0 += KC) {
      if (k0 > 0) {
#pragma unroll
        for (int k = 0; k < KC; ++k)
#pragma unroll
          for (int i = 0; i < RPT; ++i) {
            const int row = tid + PANEL_THREADS * i;
            w[k][i] = (row < m && k0 + k < wp) ? Wp[row + (long long)(k0 + k) * m] : 0.0;
          }
      }
#pragma unroll
      for (int k = 0; k < KC; ++k)
#pragma unroll
        for (int c = 0; c < NB; ++c) {
          const double pc = s_pp[k0 + k][c];
#pragma unroll
          for (int i = 0; i < RPT; ++i) a[i][c] += w[k][i] * pc;
        }
    }
  }

  gj_static_for<0, NB>([&](auto cc_) __attribute__((always_inline)) {
    constexpr int c = decltype(cc_)::value;
    if (c >= nbw) return;
    constexpr int buf = c & 1;
    unsigned key = 0;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const unsigned kk = pivot_key32<CB>(a[i][c], CMAX - (tid + PANEL_THREADS * i));
      key = max(key, ((used >> i) & 1u) ? 0u : kk);
    }
    const unsigned wkey = wave_max(key);  // uniform
    const int crow = CMAX - (int)(wkey & (unsigned)CMAX);
    if (lane == 0) s_key[buf][wave] = wkey;
    if (tid == crow % PANEL_THREADS) {
      const int ip = crow / PANEL_THREADS;  // uniform: one scalar branch is taken
#pragma unroll
      for (int i = 0; i < RPT; ++i)
        if (i == ip) {
          const double cpinv = recip_nr(a[i][c]);
          s_cpinv[buf][wave] = cpinv;
#pragma unroll
          for (int cc = 0; cc < NB; ++cc) s_cand[buf][wave][cc] = a[i][cc] * cpinv;
          // a distinct marker closing each branch keeps the compiler from
          // sinking the branches into one dynamically indexed access, which
          // would move the register array to scratch memory
          __asm__ volatile("; candidate row slot %0" ::"n"(i));
        }
    }
    __syncthreads();
    unsigned best = s_key[buf][0];
#pragma unroll
    for (int w = 1; w < NW; ++w) best = max(best, s_key[buf][w]);
    const int pr = __builtin_amdgcn_readfirstlane(CMAX - (int)(best & (unsigned)CMAX));  // uniform
    const int wb = (pr % PANEL_THREADS) / 64;
    const double pinv = s_cpinv[buf][wb];
    const bool owner = tid == pr % PANEL_THREADS;
    if (owner) {
      used |= 1u << (pr / PANEL_THREADS);
      s_piv[c] = pr;  // pos / piv go to global memory after the panel
      if (!(pinv != 0.0) || !isfinite(pinv)) atomicOr(flag, 2);
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const double l = a[i][c];
#pragma unroll
      for (int cc = 0; cc < NB; ++cc) {
        if (cc == c)
          a[i][cc] = -l * pinv;  // column k becomes the k-th column of the elimination operator
        else
          a[i][cc] -= l * s_cand[buf][wb][cc];
      }
    }
    if (owner) {
      const int ip = pr / PANEL_THREADS;  // uniform: one scalar branch is taken
#pragma unroll
      for (int i = 0; i < RPT; ++i)
        if (i == ip) {
#pragma unroll
          for (int cc = 0; cc < NB; ++cc) a[i][cc] = cc == c ? pinv : s_cand[buf][wb][cc];
          __asm__ volatile("; pivot row slot %0" ::"n"(i));
        }
    }
  });
  __syncthreads();
  if (tid < nbw) {
    pos[s_piv[tid]] = j0 + tid;
    piv[j0 + tid] = s_piv[tid];
  }
  // write the panel back (its columns are final for this panel) and W = panel - E_P
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int row = tid + PANEL_THREADS * i;
    if (row >= m) continue;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      if (c < nbw) {
        A[row + (long long)(j0 + c) * m] = a[i][c];
        W[row + (long long)c * m] = a[i][c] - (row == s_piv[c] ? 1.0 : 0.0);
      } else {
        W[row + (long long)c * m] = 0.0;
      }
    }
  }
}

template <int RPT, int NB>
__global__ __launch_bounds__(PANEL_THREADS) void gj_panel_kernel(double* __restrict__ Aall, int m, int j0, int nbw,
                                                                  int* __restrict__ posall, int* __restrict__ pivall,
                                                                  double* __restrict__ Wall, int* __restrict__ flag) {
  __builtin_amdgcn_s_setprio(3);  // critical path (see gj_small_kernel)
  const long long b = blockIdx.x;
  gj_panel_body<RPT, NB>(Aall + b * (long long)m * m, m, j0, nbw, posall + b * (long long)m,
                         pivall + b * (long long)m, Wall + b * (long long)m * PANEL_MAX_NB, flag);
}

// Gauss-Jordan update by the panel at jp of width w:
//   A(:, j) += W A(piv[jp .. jp+w), j)   (W = panel - E_P, written by the panel kernel)
// for the nout columns j = cbase + q (q < jx) and j = cbase + q + wx (q >= jx), q < nout: all
// columns outside [jx, jx + wx) = [jp, jp + w) or a wider range, or (jx = 0)
// the nout columns from wx on.  A workgroup owns GU_COLS whole columns (the
// qblk-th group): it first stages the (old) pivot-row entries of its columns
// in LDS, then rewrites its columns, so no other workgroup can overwrite a
// pivot row before it is read.
template <int THREADS, int ROWS>
__device__ __forceinline__ void gj_update_body(double* __restrict__ A, const double* __restrict__ W,
                                               const int* __restrict__ piv, int m, int jp, int w, int jx, int wx,
                                               int nout, int qblk, int cbase = 0) {
  static_assert(THREADS >= PANEL_MAX_NB * GU_COLS, "one staged pivot-row entry per thread at most");
  __shared__ double s_p[PANEL_MAX_NB][GU_COLS];
  const int tid = threadIdx.x;
  const int q0 = qblk * GU_COLS;         // first column index q of this workgroup
  auto colof = [&](int q) { return cbase + (q < jx ? q : q + wx); };
  double* colp[GU_COLS];
#pragma unroll
  for (int jj = 0; jj < GU_COLS; ++jj) colp[jj] = A + (long long)colof(q0 + jj < nout ? q0 + jj : q0) * m;
  double acc[ROWS][GU_COLS];
  double wr[GU_KC][ROWS];
  auto load_cols = [&](int r0) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
      const int r = r0 + tid + THREADS * i;
#pragma unroll
      for (int jj = 0; jj < GU_COLS; ++jj) acc[i][jj] = (r < m && q0 + jj < nout) ? colp[jj][r] : 0.0;
    }
  };
  auto load_w = [&](int r0, int c0) __attribute__((always_inline)) {
#pragma unroll
    for (int cc = 0; cc < GU_KC; ++cc)
#pragma unroll
      for (int i = 0; i < ROWS; ++i) {
        const int r = r0 + tid + THREADS * i;
        wr[cc][i] = (r < m && c0 + cc < w) ? W[r + (long long)(c0 + cc) * m] : 0.0;
      }
  };
  // the pivot index first, then the first row chunk's columns and W, then the
  // (dependent) pivot-row entry: two memory round trips before the barrier
  const int sc = tid / GU_COLS, sjj = tid % GU_COLS, sq = q0 + sjj;
  const bool stage = tid < PANEL_MAX_NB * GU_COLS && sc < w && sq < nout;
  const int prow = stage ? piv[jp + sc] : 0;
  load_cols(0);
  if (w > 0) load_w(0, 0);
  const double pval = stage ? A[prow + (long long)colof(sq) * m] : 0.0;
  if (tid < PANEL_MAX_NB * GU_COLS) s_p[sc][sjj] = pval;
  __syncthreads();
  for (int r0 = 0; r0 < m; r0 += THREADS * ROWS) {
    if (r0 > 0) load_cols(r0);
    // K loop in chunks of GU_KC with every W load of a chunk issued first
    for (int c0 = 0; c0 < w; c0 += GU_KC) {
      if (r0 > 0 || c0 > 0) load_w(r0, c0);
#pragma unroll
      for (int cc = 0; cc < GU_KC; ++cc)
#pragma unroll
        for (int jj = 0; jj < GU_COLS; ++jj) {
          const double pc = s_p[c0 + cc][jj];
#pragma unroll
          for (int i = 0; i < ROWS; ++i) acc[i][jj] += wr[cc][i] * pc;
        }
    }
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
      const int r = r0 + tid + THREADS * i;
      if (r >= m) continue;
#pragma unroll
      for (int jj = 0; jj < GU_COLS; ++jj)
        if (q0 + jj < nout) colp[jj][r] = acc[i][jj];
    }
  }
}

constexpr int GU_THREADS = 256;
// (columns restricted to [cb, cb + cw))
__global__ __launch_bounds__(GU_THREADS) void gj_update_kernel(double* __restrict__ Aall, const double* __restrict__ Wall,
                                                               const int* __restrict__ pivall, int m, int j0, int w,
                                                               int cb, int cw) {
  const long long b = blockIdx.y;
  gj_update_body<GU_THREADS, 4>(Aall + b * (long long)m * m, Wall + b * (long long)m * PANEL_MAX_NB,
                                pivall + b * (long long)m, m, j0, w, j0 - cb, w, cw - w, blockIdx.x, cb);
}

// One step of the blocked elimination in a single launch: workgroup 0 of each
// matrix applies the previous panel's update to the panel's own columns in
// registers (same order of operations as the other columns' update), then
// factors the panel at j0; the other workgroups apply the previous panel's update to
// every column of [cb, cb + cw) outside both panels (the whole matrix, or the
// column block of the two-level form).  The two parts touch disjoint columns;
// the panel writes its W into the other buffer of the pair.
template <int RPT, int NB>
__global__ __launch_bounds__(PANEL_THREADS) void gj_step_kernel(double* __restrict__ Aall, int m, int j0, int nbw,
                                                                 int* __restrict__ posall, int* __restrict__ pivall,
                                                                 double* __restrict__ Wall, const double* __restrict__ Wpall,
                                                                 int wp, int* __restrict__ flag, int cb, int cw) {
  __builtin_amdgcn_s_setprio(3);  // critical path (see gj_small_kernel)
  const long long b = blockIdx.y;
  double* A = Aall + b * (long long)m * m;
  int* piv = pivall + b * (long long)m;
  const double* Wp = Wpall + b * (long long)m * PANEL_MAX_NB;
  const int jp = j0 - wp;
  if (blockIdx.x == 0) {
    gj_panel_body<RPT, NB>(A, m, j0, nbw, posall + b * (long long)m, piv, Wall + b * (long long)m * PANEL_MAX_NB,
                           flag, Wp, jp, wp);
  } else {
    gj_update_body<PANEL_THREADS, 2>(A, Wp, piv, m, jp, wp, jp - cb, wp + nbw, cw - wp - nbw, blockIdx.x - 1, cb);
  }
}

int gj_update_launch(double* A, const double* W, const int* piv, int m, int j0, int w, long long batch,
                     hipStream_t st, int cb, int cw) {
  if (cw <= 0) { cb = 0; cw = m; }
  const int nout = cw - w;
  if (nout <= 0) return HPS_OK;
  if (cb < 0 || cb + cw > m || j0 < cb || j0 + w > cb + cw) {
    set_error("Gauss-Jordan update: column range out of bounds");
    return HPS_EINVAL;
  }
  dim3 grid((unsigned)((nout + GU_COLS - 1) / GU_COLS), (unsigned)batch);
  hipLaunchKernelGGL(gj_update_kernel, grid, dim3(GU_THREADS), 0, st, A, W, piv, m, j0, w, cb, cw);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

// Panel widths: a narrower panel shortens the serial chain of the panel
// workgroup (each pivot step updates m x nb register entries), a wider one
// needs fewer launches.  With the next panel's factorization running beside
// the previous panel's update, 8 columns measured fastest for m = 448 and 896
// (16 and 4 slower).
int gj_panel_width(int m) {
  if (m <= 1024) return 8;
  if (m <= 2048) return 16;
  if (m <= 4096) return 8;
  if (m <= 8192) return 4;
  if (m <= 16384) return 2;
  return 0;
}
int gj_panel_max_nb() { return PANEL_MAX_NB; }

int gj_panel_launch(double* A, int m, int j0, int nbw, int* pos, int* piv, double* W, int* flag, long long batch,
                    hipStream_t st) {
  dim3 grid((unsigned)batch), block(PANEL_THREADS);
  if (m <= 512)
    hipLaunchKernelGGL((gj_panel_kernel<1, 8>), grid, block, 0, st, A, m, j0, nbw, pos, piv, W, flag);
  else if (m <= 1024)
    hipLaunchKernelGGL((gj_panel_kernel<2, 8>), grid, block, 0, st, A, m, j0, nbw, pos, piv, W, flag);
  else if (m <= 2048)
    hipLaunchKernelGGL((gj_panel_kernel<4, 16>), grid, block, 0, st, A, m, j0, nbw, pos, piv, W, flag);
  else if (m <= 4096)
    hipLaunchKernelGGL((gj_panel_kernel<8, 8>), grid, block, 0, st, A, m, j0, nbw, pos, piv, W, flag);
  else if (m <= 8192)
    hipLaunchKernelGGL((gj_panel_kernel<16, 4>), grid, block, 0, st, A, m, j0, nbw, pos, piv, W, flag);
  else if (m <= 16384)
    hipLaunchKernelGGL((gj_panel_kernel<32, 2>), grid, block, 0, st, A, m, j0, nbw, pos, piv, W, flag);
  else {
    set_error("blocked Gauss-Jordan: matrix larger than 16384 not supported");
    return HPS_EUNSUPPORTED;
  }
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

int gj_step_launch(double* A, int m, int j0, int nbw, int* pos, int* piv, double* W, const double* Wp, int wp,
                   int* flag, long long batch, hipStream_t st, int cb, int cw) {
  if (cw <= 0) { cb = 0; cw = m; }
  const int nout = cw - wp - nbw;
  // the first panel (wp = 0) has no previous update to apply: panel workgroups only
  const int nupd = (wp > 0 && nout > 0) ? (nout + GU_COLS - 1) / GU_COLS : 0;
  dim3 grid((unsigned)(1 + nupd), (unsigned)batch), block(PANEL_THREADS);
  if (batch > 65535 || wp > PANEL_MAX_NB || j0 < wp || j0 - wp < cb || cb < 0 || cb + cw > m || j0 + nbw > cb + cw) {
    set_error("blocked Gauss-Jordan step: batch or panel layout out of range");
    return HPS_EINVAL;
  }
  if (m <= 512)
    hipLaunchKernelGGL((gj_step_kernel<1, 8>), grid, block, 0, st, A, m, j0, nbw, pos, piv, W, Wp, wp, flag, cb, cw);
  else if (m <= 1024)
    hipLaunchKernelGGL((gj_step_kernel<2, 8>), grid, block, 0, st, A, m, j0, nbw, pos, piv, W, Wp, wp, flag, cb, cw);
  else if (m <= 2048)
    hipLaunchKernelGGL((gj_step_kernel<4, 16>), grid, block, 0, st, A, m, j0, nbw, pos, piv, W, Wp, wp, flag, cb, cw);
  else if (m <= 4096)
    hipLaunchKernelGGL((gj_step_kernel<8, 8>), grid, block, 0, st, A, m, j0, nbw, pos, piv, W, Wp, wp, flag, cb, cw);
  else if (m <= 8192)
    hipLaunchKernelGGL((gj_step_kernel<16, 4>), grid, block, 0, st, A, m, j0, nbw, pos, piv, W, Wp, wp, flag, cb, cw);
  else if (m <= 16384)
    hipLaunchKernelGGL((gj_step_kernel<32, 2>), grid, block, 0, st, A, m, j0, nbw, pos, piv, W, Wp, wp, flag, cb, cw);
  else {
    set_error("blocked Gauss-Jordan: matrix larger than 16384 not supported");
    return HPS_EUNSUPPORTED;
  }
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

// Two-level form, per column block [b0, b0 + w) after its inner panels:
// Wk(:, c) = A(:, b0 + c) - e_{piv[b0 + c]} (the block's combined elimination
// operator minus the pivot-row identity) and Pk(c, j) = A(piv[b0 + c], j) for
// every column j (the pivot rows' values before the block's update of the
// other columns); then A(:, j) += Wk Pk(:, j) for every j outside the block,
// as two grouped GEMMs.
__global__ __launch_bounds__(256) void gj_block_w_kernel(const double* __restrict__ Aall, const int* __restrict__ pivall,
                                                         int m, int b0, int w, int ob, double* __restrict__ Wkall) {
  const long long b = blockIdx.y;
  const double* A = Aall + b * (long long)m * m;
  const int* piv = pivall + b * (long long)m;
  double* Wk = Wkall + b * (long long)m * ob;
  const long long n = (long long)m * w;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e % m), c = (int)(e / m);
    Wk[e] = A[r + (long long)(b0 + c) * m] - (r == piv[b0 + c] ? 1.0 : 0.0);
  }
}

__global__ __launch_bounds__(256) void gj_pivot_rows_kernel(const double* __restrict__ Aall,
                                                            const int* __restrict__ pivall, int m, int b0, int w,
                                                            int ob, double* __restrict__ Pkall) {
  const long long b = blockIdx.y;
  const double* A = Aall + b * (long long)m * m;
  const int* piv = pivall + b * (long long)m;
  double* Pk = Pkall + b * (long long)ob * m;
  const long long n = (long long)w * m;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(e % w), j = (int)(e / w);
    Pk[c + (long long)j * ob] = A[piv[b0 + c] + (long long)j * m];
  }
}

int gj_block_prep_launch(const double* A, const int* piv, int m, int b0, int w, int ob, double* Wk, double* Pk,
                         long long batch, hipStream_t st) {
  if (batch > 65535 || w > ob || b0 < 0 || b0 + w > m) {
    set_error("Gauss-Jordan block preparation: layout out of range");
    return HPS_EINVAL;
  }
  const long long n = (long long)m * w;
  const unsigned gx = (unsigned)std::min<long long>(2048, (n + 255) / 256);
  hipLaunchKernelGGL(gj_block_w_kernel, dim3(gx, (unsigned)batch), dim3(256), 0, st, A, piv, m, b0, w, ob, Wk);
  HPS_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(gj_pivot_rows_kernel, dim3(gx, (unsigned)batch), dim3(256), 0, st, A, piv, m, b0, w, ob, Pk);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

int gj_init_launch(int* pos, long long n, hipStream_t st) {
  hipLaunchKernelGGL(gj_init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pos, n);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

// Z(a, b) = R(piv[a], pos[b])
__global__ void gj_unscramble_kernel(const double* __restrict__ Rall, double* __restrict__ Zall, int m,
                                     const int* __restrict__ posall, const int* __restrict__ pivall) {
  const long long b = blockIdx.y;
  const int col = blockIdx.x;
  const double* R = Rall + b * (long long)m * m;
  double* Z = Zall + b * (long long)m * m;
  const int* pos = posall + b * (long long)m;
  const int* piv = pivall + b * (long long)m;
  const long long src_col = (long long)pos[col] * m;
  for (int a = threadIdx.x; a < m; a += blockDim.x) Z[a + (long long)col * m] = R[piv[a] + src_col];
}

int gj_unscramble_launch(const double* R, double* Z, int m, const int* pos, const int* piv, long long batch,
                         hipStream_t st) {
  hipLaunchKernelGGL(gj_unscramble_kernel, dim3((unsigned)m, (unsigned)batch), dim3(256), 0, st, R, Z, m, pos, piv);
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

}  // namespace hps
