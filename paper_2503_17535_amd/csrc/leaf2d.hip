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

// Matrix-core helpers of the back substitution: 16 x 16 products on
// v_mfma_f64_16x16x4f64 (lane l, accumulator element e holds row (l >> 4) + 4e,
// column l & 15 of the product) and the inverse of a unit triangular block.
typedef double v4d_l __attribute__((ext_vector_type(4)));


__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ v4d_l mfma_f64(double a, double b, v4d_l c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Z = X Y for 16 x 16 row-major matrices in LDS, by one wavefront (Z may not
// alias X or Y).
__device__ __forceinline__ void mm16(const double (*X)[16], const double (*Yv)[16], double (*Z)[16], int g, int cl) {
  v4d_l z = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int c = 0; c < 4; ++c) z = mfma_f64(X[cl][4 * c + g], Yv[4 * c + g][cl], z);
#pragma unroll
  for (int e = 0; e < 4; ++e) Z[g + 4 * e][cl] = z[e];
  wave_sync();
}

// (I + N)^{-1} = (I - N)(I + N^2)(I + N^4)(I + N^8) for a strictly
// triangular 16 x 16 N (N^16 = 0), as six products on the matrix cores by one
// wavefront.  N is overwritten; work holds three 16 x 16 matrices; the
// result goes to out.
__device__ __forceinline__ void tri_inv16(double (*N)[16], double (*work)[16][16], double (*out)[16], int lane) {
  const int g = lane >> 4, cl = lane & 15;
  double (*A)[16] = work[0];
  double (*B)[16] = work[1];
  double (*Cm)[16] = work[2];
  // A = I - N, B = I + N^2 (N^2 in Cm)
  mm16(N, N, Cm, g, cl);
  for (int e = lane; e < 256; e += 64) {
    const int i = e >> 4, m = e & 15;
    const double d = (i == m) ? 1.0 : 0.0;
    A[i][m] = d - N[i][m];
    B[i][m] = d + Cm[i][m];
  }
  wave_sync();
  mm16(A, B, out, g, cl);          // out = (I - N)(I + N^2)
  mm16(Cm, Cm, N, g, cl);          // N  = N^4
  for (int e = lane; e < 256; e += 64) {
    const int i = e >> 4, m = e & 15;
    B[i][m] = ((i == m) ? 1.0 : 0.0) + N[i][m];
  }
  wave_sync();
  mm16(out, B, A, g, cl);          // A = ... (I + N^4)
  mm16(N, N, Cm, g, cl);           // Cm = N^8
  for (int e = lane; e < 256; e += 64) {
    const int i = e >> 4, m = e & 15;
    B[i][m] = ((i == m) ? 1.0 : 0.0) + Cm[i][m];
  }
  wave_sync();
  mm16(A, B, out, g, cl);          // out = ... (I + N^8)
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
  __shared__ double s_uinv[(NI + 15) / 16][16][16];  // inverses of the diagonal U blocks
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

  // ---- back substitution of the augmented columns:  U X = Yp, on the matrix cores.
  // Yp (the forward-eliminated L_ie P) leaves the registers in pivot order
  // (unknown k = pivot step of its row) into Y, which X then overwrites.
  // Blocked by 16 unknowns: for block J (last to first)
  //   X_J = U_JJ^{-1} (Yp_J - sum_{J2 > J} U_{J,J2} X_J2),
  // the U blocks read from the factor just written, the inverses of the
  // diagonal blocks formed first, one wavefront per 16 right-hand sides.
  constexpr int RF = RJP - 1;
  constexpr int NLB = (NBLK - RF) < RJ ? (NBLK - RF) : RJ;
  constexpr int NPB = (NI + 15) / 16;          // blocks of 16 unknowns
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
      Yl[pk + (long long)(col - NI) * NI] = a[ri][s];
    }
  }
  __syncthreads();
  {
    // inverses of the diagonal U blocks: U = D (I + N), N = D^{-1}(U - D)
    // strictly upper, U^{-1} = (I + N)^{-1} D^{-1}; workspaces in s_L0
    // (a dedicated workspace for small leaves, whose s_L0 is smaller than one)
    const int lane64 = tid & 63, wv = tid >> 6;
    constexpr int NWL0 = (TC * RI * TR) / (5 * 256);
    constexpr int NWI = NWL0 < 1 ? 1 : (NWL0 < NT / 64 ? NWL0 : NT / 64);
    __shared__ double s_triw[NWL0 < 1 ? 5 * 256 : 1];
    if (wv < NWI) {
      double* twb = NWL0 < 1 ? s_triw : &s_L0[0][0] + wv * 5 * 256;
      double (*tw)[16][16] = reinterpret_cast<double (*)[16][16]>(twb);
      for (int jb = wv; jb < NPB; jb += NWI) {
        const int k0 = 16 * jb, npiv = min(16, NI - k0);
        for (int e = lane64; e < 256; e += 64) {
          const int i = e >> 4, m = e & 15;
          double v = 0.0;
          if (i < m && m < npiv) v = LUl[(long long)(k0 + m) * NI + k0 + i] / LUl[(long long)(k0 + i) * NI + k0 + i];
          tw[0][i][m] = v;
        }
        wave_sync();
        tri_inv16(tw[0], &tw[1], tw[4], lane64);
        for (int e = lane64; e < 256; e += 64) {
          const int i = e >> 4, m = e & 15;
          const double dinv = m < npiv ? 1.0 / LUl[(long long)(k0 + m) * NI + k0 + m] : 1.0;
          s_uinv[jb][i][m] = tw[4][i][m] * dinv;
        }
        wave_sync();
      }
    }
    __syncthreads();
    constexpr int NBT = (NB + 15) / 16;
    static_assert(NBT <= NT / 64, "one wavefront per 16 right-hand sides");
    if (wv < NBT) {
      const int g = lane64 >> 4, cl = lane64 & 15;
      const int rhs = 16 * wv + cl;
      v4d_l X[NPB];
      static_for<0, NPB>([&](auto jc) {
        constexpr int J = NPB - 1 - decltype(jc)::value;
        v4d_l z;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int k = 16 * J + g + 4 * e;
          z[e] = (k < NI && rhs < NB) ? Yl[(long long)rhs * NI + k] : 0.0;
        }
        // this block row's U blocks, all loads issued before the products
        double ua[NPB > J + 1 ? NPB - J - 1 : 1][4];
        static_for<J + 1, NPB>([&](auto j2c) {
          constexpr int J2 = decltype(j2c)::value;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const int sc = 16 * J2 + 4 * c + g;
            ua[J2 - J - 1][c] = (sc < NI && 16 * J + cl < NI) ? -LUl[(long long)sc * NI + 16 * J + cl] : 0.0;
          }
        });
        static_for<J + 1, NPB>([&](auto j2c) {
          constexpr int J2 = decltype(j2c)::value;
#pragma unroll
          for (int c = 0; c < 4; ++c) z = mfma_f64(ua[J2 - J - 1][c], X[J2][c], z);
        });
        v4d_l x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < 4; ++c) x = mfma_f64(s_uinv[J][cl][4 * c + g], z[c], x);
        X[J] = x;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int k = 16 * J + g + 4 * e;
          if (k < NI && rhs < NB) Yl[(long long)rhs * NI + k] = -x[e];
        }
      });
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
