// 2D leaf stage, fused: one workgroup per leaf.
//
// For each leaf (Algorithm "2D DtN local solve", Appendix A.1) the kernel
//   1. assembles in registers the augmented matrix  [ L_ii | L_ie P ]
//      (n_i x (n_i + n_b)) from the coefficient samples: L_ii from the 1D
//      Chebyshev derivative matrices, L_ie P as sum_t c_t(x) M_t with the
//      precomputed M_t = D_t(I_i, I_e) P,
//   2. factors L_ii by Gaussian elimination with partial pivoting, carrying the
//      augmented columns along (forward elimination),
//   3. back-substitutes the augmented columns:  X = L_ii^{-1} L_ie P,
// and writes the LU factors (for sources at solve time; column s holds the U
// entries in pivot order, then the L entries of the rows not yet pivoted, in
// row order), the pivot order, and Y_int = -X (the interior rows of
// Y = [I; -L_ii^{-1} L_ie] P).
// T = Q Y is one batched GEMM after this kernel.
//
// Layout: the threads form a TR x TC grid (thread id = tc * TR + tr); thread
// (tr, tc) owns rows tr + TR*ri and columns tc + TC*rj (cyclic), all in
// registers.  Pivoting is implicit: rows never move; a row that has served as
// pivot is marked used, the pivot order is recorded (perm[k] = row of step k,
// pos[row] = k), and the factors are stored with rows in their original
// positions.  The pivot search of column k runs inside the TR lanes that own
// the column (one wavefront, DPP lane exchanges); ties go to the lowest row.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "common.hpp"
#include "dpp.hpp"
#include "../../include/hps.h"

namespace hps {

// Compile-time loop: f(integral_constant<int, I>) for I = B .. E-1.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

template <int P>
struct Leaf2DCfg {
  static constexpr int NI = (P - 2) * (P - 2);
  static constexpr int NB = 4 * (P - 2);
  static constexpr int NC = NI + NB;                  // augmented columns
  static constexpr int TR = NI > 16 ? 16 : 8;
  static constexpr int TC = NI > 64 ? 32 : 16;
  static constexpr int NT = TR * TC;
  static constexpr int RI = (NI + TR - 1) / TR;
  static constexpr int RJALL = (NC + TC - 1) / TC;    // column blocks in total
  static constexpr int RJ = RJALL > 7 ? 7 : RJALL;    // register slots
  static constexpr int EXTRA = RJALL > RJ ? 1 : 0;    // one block enters late
  static constexpr int NBLK = RJ + EXTRA;
  static constexpr int RJP = (NI + TC - 1) / TC;      // blocks holding pivot columns
  static constexpr int NPTS = P * P;
  // augmented columns held in the register slots / entering late; both are
  // staged through LDS (SAUG columns at a time)
  static constexpr int AUG_IN_SLOTS = RJ * TC - NI < NB ? RJ * TC - NI : NB;
  static constexpr int AUG_LATE = EXTRA ? NC - RJ * TC : 0;
  static constexpr int SAUG = AUG_IN_SLOTS > AUG_LATE ? AUG_IN_SLOTS : AUG_LATE;
  static_assert(RJALL <= RJ + 1, "at most one late column block");
  static_assert(64 % TR == 0, "a column group of TR lanes lies inside one wavefront");
  static_assert(RI * TR <= 255, "row rank codes fit in the 8 low bits of a pivot key");
  static_assert(!EXTRA || RJP >= 2, "late block needs a first pivot block to replay");
};

// Entry (row, col) of L_ii for a leaf whose coefficients are in LDS
// (row, col index interior points in tensor order).
template <int P>
__device__ __forceinline__ double leaf2d_lii(int row, int col, const double (*coef)[P * P],
                                             const double* d1, const double* d2, const int* active) {
  constexpr int NI = Leaf2DCfg<P>::NI, Q = P - 2;
  if (row >= NI || col >= NI) return 0.0;
  const int ixr = 1 + row % Q, iyr = 1 + row / Q;
  const int pr = ixr + P * iyr;
  const int ixc = 1 + col % Q, iyc = 1 + col / Q;
  double v = 0.0;
  if (iyr == iyc) v += coef[0][pr] * d2[ixr * P + ixc] + coef[3][pr] * d1[ixr * P + ixc];
  if (ixr == ixc) v += coef[2][pr] * d2[iyr * P + iyc] + coef[4][pr] * d1[iyr * P + iyc];
  if (active[1]) v += coef[1][pr] * d1[iyr * P + iyc] * d1[ixr * P + ixc];
  if (row == col) v += coef[5][pr];
  return v;
}

// Stage augmented columns [c0, c0 + nc) of L_ie P = sum_t diag(c_t) M_t into
// LDS (column-major, leading dimension NI).
template <int P>
__device__ __forceinline__ void leaf2d_stage_aug(double* s_aug, int c0, int nc, const double (*coef)[P * P],
                                                 const int* active, const double* __restrict__ Mt,
                                                 int tid, int nt) {
  constexpr int NI = Leaf2DCfg<P>::NI, NB = Leaf2DCfg<P>::NB, Q = P - 2;
  for (int e = tid; e < NI * nc; e += nt) {
    const int row = e % NI, j = c0 - NI + e / NI;
    const int pr = (1 + row % Q) + P * (1 + row / Q);
    double v = 0.0;
    if (j < NB) {
#pragma unroll
      for (int t = 0; t < 5; ++t)  // the zeroth-order term has no L_ie part
        if (active[t]) v += coef[t][pr] * Mt[(long long)t * NI * NB + row + (long long)j * NI];
    }
    s_aug[e] = v;
  }
}

template <int P>
__global__ __launch_bounds__(Leaf2DCfg<P>::NT) void leaf2d_factor_kernel(
    const double* __restrict__ coeffs,  // [nl][6][P*P]
    const double* __restrict__ D1g,     // [P*P] row-major, d/dx on the leaf
    const double* __restrict__ D2g,     // [P*P] row-major, d2/dx2 on the leaf
    const double* __restrict__ Mt,      // [6][NI x NB] column-major (ld NI)
    double* __restrict__ LU,            // [nl][NI x NI] per column: U part (pivot order), L part (row order)
    int* __restrict__ perm,             // [nl][NI]  row chosen at step k
    int* __restrict__ pos,              // [nl][NI]  step at which row was chosen
    double* __restrict__ Y,             // [nl][NI x NB] column-major
    int* __restrict__ flag) {
  typedef Leaf2DCfg<P> C;
  constexpr int NI = C::NI, NB = C::NB, NC = C::NC, TR = C::TR, TC = C::TC, NT = C::NT;
  constexpr int RI = C::RI, RJ = C::RJ, RJP = C::RJP, NBLK = C::NBLK;

  __shared__ double s_coef[6][P * P];
  __shared__ double s_d1[P * P], s_d2[P * P];
  __shared__ double s_lcol[2][RI * TR];
  __shared__ double s_urow[2][RJ * TC];
  __shared__ double s_xrow[2][NB];
  // block 0's L columns for the late block's replay; later the staged U
  // columns of the back substitution
  __shared__ double s_L0[TC][RI * TR];
  __shared__ double s_aug[C::SAUG > 0 ? NI * C::SAUG : 1];
  __shared__ double s_dinv[NI];
  __shared__ int s_perm[NI], s_pos[RI * TR];
  __shared__ int s_piv[2];
  __shared__ int s_active[6];

  const long long leaf = blockIdx.x;
  const int tid = threadIdx.x;
  const int tr = tid % TR, tc = tid / TR;
  const int lane = tid & 63;
  const int gbase = lane - tr;  // first lane of this thread's column group

  // ---- stage coefficients and 1D operators
  const double* cf = coeffs + leaf * 6 * C::NPTS;
  for (int i = tid; i < 6 * C::NPTS; i += NT) s_coef[i / C::NPTS][i % C::NPTS] = cf[i];
  for (int i = tid; i < P * P; i += NT) { s_d1[i] = D1g[i]; s_d2[i] = D2g[i]; }
  if (tid < 6) s_active[tid] = 0;
  for (int i = tid; i < RI * TR; i += NT) s_pos[i] = -1;
  __syncthreads();
  for (int i = tid; i < 6 * C::NPTS; i += NT)
    if (s_coef[i / C::NPTS][i % C::NPTS] != 0.0) s_active[i / C::NPTS] = 1;
  __syncthreads();

  // ---- registers: slot s holds global column block (r + s) after r rotations
  if (C::AUG_IN_SLOTS > 0)
    leaf2d_stage_aug<P>(s_aug, NI, C::AUG_IN_SLOTS, s_coef, s_active, Mt, tid, NT);
  __syncthreads();
  double a[RI][RJ];
#pragma unroll
  for (int s = 0; s < RJ; ++s)
#pragma unroll
    for (int ri = 0; ri < RI; ++ri) {
      const int row = tr + TR * ri, col = tc + TC * s;
      double v = 0.0;
      if (row < NI) {
        if (col < NI) v = leaf2d_lii<P>(row, col, s_coef, s_d1, s_d2, s_active);
        else if (col < NI + C::AUG_IN_SLOTS) v = s_aug[row + (col - NI) * NI];
      }
      a[ri][s] = v;
    }
  unsigned used = 0;  // bit ri: row tr + TR*ri has been a pivot (or is padding)
#pragma unroll
  for (int ri = 0; ri < RI; ++ri)
    if (tr + TR * ri >= NI) used |= 1u << ri;

  double* LUl = LU + leaf * (long long)NI * NI;

  // ---- forward elimination with implicit partial pivoting
  // the block loop is expanded at compile time (static_for) so that the
  // rotation count r = kb is a constant: slot rotation becomes register
  // renaming and the number of live slots is known in every step
  static_for<0, RJP>([&](auto kbc) {
    constexpr int kb = decltype(kbc)::value;
    constexpr int r = kb;  // rotations done
    for (int t = 0; t < TC; ++t) {
      const int k = kb * TC + t;
      if (k >= NI) break;
      const int buf = k & 1;
      if (tc == t) {
        // pivot search: the largest |x| over the group's unused rows, as one
        // unsigned max of packed keys (pivot_key32_c8: |x| to 12 mantissa bits
        // above the row's rank code 255 - row), ties to the lower row
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
        for (int ri = 0; ri < RI; ++ri) {
          const bool keep = ((used >> ri) & 1u) || (ri == bri && tr == btr);
          const double l = keep ? 0.0 : a[ri][0] * pinv;
          if (!keep) a[ri][0] = l;
          s_lcol[buf][tr + TR * ri] = l;
        }
        if (tr == 0) {
          s_piv[buf] = brow;
          s_perm[k] = brow;
          s_pos[brow] = k;
          s_dinv[k] = pinv;
          if (!(pv != 0.0) || !isfinite(pv) || !isfinite(pinv)) atomicOr(flag, 1);
        }
      }
      __syncthreads();
      const int pr = __builtin_amdgcn_readfirstlane(s_piv[buf]);  // uniform: scalar branches below
      if (tr == pr % TR) {
        const int rip = pr / TR;  // uniform: one scalar branch is taken
        used |= 1u << rip;
#pragma unroll
        for (int ri = 0; ri < RI; ++ri)
          if (ri == rip) {
#pragma unroll
            for (int s = 0; s < RJ; ++s)
              if (r + s < NBLK) s_urow[buf][tc + TC * s] = a[ri][s];
          }
      }
      // the pivot row's entries of column tc + TC*s are read only by the TR
      // lanes of this thread's column group, which share its wavefront: a
      // wavefront-level barrier orders the LDS write before their reads
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int s = 0; s < RJ; ++s) {
        if (r + s >= NBLK) break;
        const double u = (s > 0 || tc > t) ? s_urow[buf][tc + TC * s] : 0.0;
#pragma unroll
        for (int ri = 0; ri < RI; ++ri) a[ri][s] -= s_lcol[buf][tr + TR * ri] * u;
      }
    }
    // pivot block finished: its columns are final L / U entries.  Column col
    // is stored as [U entries in pivot order | L entries of the rows not yet
    // pivoted after step col, in row order]; an L row's slot is col + 1 plus
    // the number of L rows above it, counted by ballots over the column group
    {
      const int col = kb * TC + tc;
      const unsigned lanes_below = (1u << tr) - 1u;
      int above = 0;  // L rows in the earlier row slots of this column
#pragma unroll
      for (int ri = 0; ri < RI; ++ri) {
        const int row = tr + TR * ri;
        const int pk = row < NI ? s_pos[row] : 0;
        const bool lrow = row < NI && (pk < 0 || pk > col);
        const unsigned gm = (unsigned)(__ballot(lrow) >> gbase) & ((1u << TR) - 1u);
        if (col < NI && row < NI) {
          const int slot = lrow ? col + 1 + above + __popc(gm & lanes_below) : pk;
          LUl[(long long)col * NI + min(slot, NI - 1)] = a[ri][0];
        }
        above += __popc(gm);
      }
    }
    if constexpr (kb == RJP - 1) return;  // keep the last pivot block (it also holds augmented columns)
    if constexpr (C::EXTRA && kb == 0) {
#pragma unroll
      for (int ri = 0; ri < RI; ++ri) s_L0[tc][tr + TR * ri] = a[ri][0];
    }
    // rotate slots left
#pragma unroll
    for (int ri = 0; ri < RI; ++ri) {
#pragma unroll
      for (int s = 0; s + 1 < RJ; ++s) a[ri][s] = a[ri][s + 1];
      a[ri][RJ - 1] = 0.0;
    }
    if constexpr (C::EXTRA && kb == 0) {
      // the late column block enters slot RJ-1 and replays the TC steps of
      // block 0: x_row -= L(row, j) * x_perm[j] for rows pivoted after step j
      leaf2d_stage_aug<P>(s_aug, RJ * TC, C::AUG_LATE, s_coef, s_active, Mt, tid, NT);
      __syncthreads();
#pragma unroll
      for (int ri = 0; ri < RI; ++ri) {
        const int row = tr + TR * ri;
        a[ri][RJ - 1] = (row < NI && tc < C::AUG_LATE) ? s_aug[row + tc * NI] : 0.0;
      }
      for (int j = 0; j < TC; ++j) {
        const int pj = __builtin_amdgcn_readfirstlane(s_perm[j]);  // uniform: scalar branches below
        double mine = 0.0;
#pragma unroll
        for (int ri = 0; ri < RI; ++ri)
          if (tr + TR * ri == pj) mine = a[ri][RJ - 1];
        const double y = __shfl(mine, gbase + pj % TR);
#pragma unroll
        for (int ri = 0; ri < RI; ++ri) {
          const int row = tr + TR * ri;
          const int pk = s_pos[row];
          if (row < NI && (pk < 0 || pk > j)) a[ri][RJ - 1] -= s_L0[j][row] * y;
        }
      }
    }
  });
  __syncthreads();

  // ---- back substitution of the augmented columns:  U X = (forward-eliminated L_ie P)
  // After the forward pass slot s holds block RF + s (RF = RJP - 1 rotations);
  // only NLB slots are live.  Blocked by TC columns: the block's U columns
  // (entries of rows pivoted before the column, zero elsewhere) are staged in
  // LDS once; then each column group, whose TR lanes hold every row of its
  // columns, runs the block's steps on its own with x_k broadcast inside the
  // group, so a block costs two workgroup barriers instead of one per step.
  constexpr int RF = RJP - 1;
  constexpr int NLB = (NBLK - RF) < RJ ? (NBLK - RF) : RJ;
  constexpr int RT = RI * TR;
  for (int kb = RJP - 1; kb >= 0; --kb) {
    if (kb < RJP - 1) __syncthreads();  // the previous block's reads are done
    for (int e = tid; e < TC * RT; e += NT) {
      const int c = e / RT, row = e % RT, k = kb * TC + c;
      double u = 0.0;
      if (k < NI && row < NI) {
        const int pk = s_pos[row];
        if (pk < k) u = LUl[(long long)k * NI + pk];  // U part, pivot order
      }
      s_L0[c][row] = u;
    }
    __syncthreads();
    const int tlast = (NI - kb * TC) < TC ? (NI - kb * TC) : TC;  // steps in this block
    int pr_n = s_perm[kb * TC + tlast - 1];
    double dinv_n = s_dinv[kb * TC + tlast - 1];
    for (int t = tlast - 1; t >= 0; --t) {
      const int k = kb * TC + t;
      const int pr = __builtin_amdgcn_readfirstlane(pr_n);  // uniform
      const int rip = pr / TR, trp = pr % TR;
      const double dinv = dinv_n;
      if (t > 0) {  // the next step's pivot row and reciprocal, ahead of time
        pr_n = s_perm[k - 1];
        dinv_n = s_dinv[k - 1];
      }
      double x[NLB];
      // x_k of each live column: the pivot row's entry, scaled, from lane trp;
      // the uniform register index becomes a scalar branch
      static_for<0, RI>([&](auto ric) {
        constexpr int R = decltype(ric)::value;
        if (R == rip) {
#pragma unroll
          for (int s = 0; s < NLB; ++s) {
            x[s] = __shfl(a[R][s] * dinv, gbase + trp);
            if (tr == trp) a[R][s] = x[s];
          }
        }
      });
#pragma unroll
      for (int s = 0; s < NLB; ++s)
#pragma unroll
        for (int ri = 0; ri < RI; ++ri) a[ri][s] -= s_L0[t][tr + TR * ri] * x[s];
    }
  }

  // ---- outputs: X row k (unknown k) sits in augmented row perm[k]
  double* Yl = Y + leaf * (long long)NI * NB;
#pragma unroll
  for (int ri = 0; ri < RI; ++ri) {
    const int row = tr + TR * ri;
    if (row >= NI) continue;
    const int pk = s_pos[row];
#pragma unroll
    for (int s = 0; s < NLB; ++s) {
      const int col = (RF + s) * TC + tc;
      if (col < NI || col >= NC) continue;
      Yl[pk + (long long)(col - NI) * NI] = -a[ri][s];
    }
  }
  for (int i = tid; i < NI; i += NT) {
    perm[leaf * NI + i] = s_perm[i];
    pos[leaf * NI + i] = s_pos[i];
  }
}

template <int P>
static void launch_leaf2d(const double* coeffs, const double* D1, const double* D2, const double* Mt,
                          double* LU, int* perm, int* pos, double* Y, int* flag, long long nl,
                          hipStream_t st) {
  hipLaunchKernelGGL((leaf2d_factor_kernel<P>), dim3((unsigned)nl), dim3(Leaf2DCfg<P>::NT), 0, st,
                     coeffs, D1, D2, Mt, LU, perm, pos, Y, flag);
}

int leaf2d_launch(int p, const double* coeffs, const double* D1, const double* D2, const double* Mt,
                  double* LU, int* perm, int* pos, double* Y, int* flag, long long nl, hipStream_t st) {
  switch (p) {
    case 4: launch_leaf2d<4>(coeffs, D1, D2, Mt, LU, perm, pos, Y, flag, nl, st); break;
    case 5: launch_leaf2d<5>(coeffs, D1, D2, Mt, LU, perm, pos, Y, flag, nl, st); break;
    case 6: launch_leaf2d<6>(coeffs, D1, D2, Mt, LU, perm, pos, Y, flag, nl, st); break;
    case 7: launch_leaf2d<7>(coeffs, D1, D2, Mt, LU, perm, pos, Y, flag, nl, st); break;
    case 8: launch_leaf2d<8>(coeffs, D1, D2, Mt, LU, perm, pos, Y, flag, nl, st); break;
    case 9: launch_leaf2d<9>(coeffs, D1, D2, Mt, LU, perm, pos, Y, flag, nl, st); break;
    case 10: launch_leaf2d<10>(coeffs, D1, D2, Mt, LU, perm, pos, Y, flag, nl, st); break;
    case 11: launch_leaf2d<11>(coeffs, D1, D2, Mt, LU, perm, pos, Y, flag, nl, st); break;
    case 12: launch_leaf2d<12>(coeffs, D1, D2, Mt, LU, perm, pos, Y, flag, nl, st); break;
    case 13: launch_leaf2d<13>(coeffs, D1, D2, Mt, LU, perm, pos, Y, flag, nl, st); break;
    case 14: launch_leaf2d<14>(coeffs, D1, D2, Mt, LU, perm, pos, Y, flag, nl, st); break;
    case 15: launch_leaf2d<15>(coeffs, D1, D2, Mt, LU, perm, pos, Y, flag, nl, st); break;
    case 16: launch_leaf2d<16>(coeffs, D1, D2, Mt, LU, perm, pos, Y, flag, nl, st); break;
    default:
      set_error("2D leaf kernel supports 4 <= p <= 16");
      return HPS_EUNSUPPORTED;
  }
  HPS_HIP_TRY(hipGetLastError());
  return HPS_OK;
}

}  // namespace hps
