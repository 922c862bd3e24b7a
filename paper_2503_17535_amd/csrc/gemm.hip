// Grouped, strided-batched GEMM on CDNA4 matrix cores.
//
// fp64: v_mfma_f64_16x16x4f64 (one 16x16x4 product per wavefront).
// fp32: v_mfma_f32_16x16x4f32.
// Workgroup tile 64 x 64 (4 wavefronts, each 32 x 32 = 2 x 2 MFMA blocks),
// k-step 16 staged through LDS.  The MFMA is fed with (B-fragment, A-fragment)
// so that its accumulator layout puts consecutive lanes on consecutive rows
// of the column-major C: the epilogue stores 128-byte runs.  Accumulator
// layout (measured on gfx950): fp64 lane l, element v holds D(l/16 + 4v, l%16);
// fp32 lane l, element v holds D(4 (l/16) + v, l%16).
//
// Products with at most 16 columns and neither operand transposed (the solve's
// per-right-hand-side products) take gemm_skinny_kernel: the same blocks, but
// the wavefronts read their MFMA fragments straight from memory (no LDS).
//
// One launch covers a list of groups (GemmGroup); every (group, batch item,
// tile) triple is one workgroup.  Block indices are remapped so that the
// blocks the hardware dispatches to one XCD (block id mod 8) are consecutive
// tiles of one product, which keeps their shared A/B panels in that XCD's L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.hpp"
#include "../../include/hps.h"

namespace hps {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16, GEMM_THREADS = 256, NXCD = 8;

template <typename G>
__device__ __forceinline__ const G* find_group(const G* groups, int ngroups, long long lb) {
  int lo = 0, hi = ngroups - 1;
  while (lo < hi) {  // last group with first_block <= lb
    int mid = (lo + hi + 1) >> 1;
    if (groups[mid].first_block <= lb) lo = mid; else hi = mid - 1;
  }
  return groups + lo;
}

__device__ __forceinline__ long long xcd_remap(long long b, long long nblocks) {
  // hardware dispatch: block b -> XCD b % NXCD.  Give each XCD a contiguous
  // range of logical blocks.
  const long long q = nblocks / NXCD, r = nblocks % NXCD;
  const long long x = b % NXCD, local = b / NXCD;
  const long long start = x * q + (x < r ? x : r);
  return start + local;
}

// Pointers read from the group table in memory are generic (flat) to the
// compiler.  A flat load counts against both the vector-memory and the
// LDS/scalar wait counters, and the compiler then tends to wait for all
// outstanding loads at once; a cast to the global address space gives global
// loads, whose waits count vector-memory operations only, so that loads
// issued ahead stay in flight.
template <typename T> using gmem = __attribute__((address_space(1))) T;
template <typename T> __device__ __forceinline__ const gmem<T>* gptr(const T* p) { return (const gmem<T>*)p; }
template <typename T> __device__ __forceinline__ gmem<T>* gptr(T* p) { return (gmem<T>*)p; }

template <typename T> struct MfmaOp;
// col(lane, v): column of C (within the 16 x 16 block) that accumulator
// element v of `lane` holds; its row is lane % 16 (see the feeding order).
template <> struct MfmaOp<double> {
  typedef v4d acc_t;
  static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // fp64 accumulator: lane l, element v holds D(l/16 + 4v, l%16)
  static __device__ __forceinline__ int col(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <> struct MfmaOp<float> {
  typedef v4f acc_t;
  static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // fp32 accumulator: lane l, element v holds D(4 (l/16) + v, l%16)
  static __device__ __forceinline__ int col(int lane, int v) { return 4 * (lane >> 4) + v; }
};

template <typename T, typename G, bool TA, bool TB>
__global__ __launch_bounds__(GEMM_THREADS) void gemm_grouped_kernel(const G* __restrict__ groups,
                                                                    int ngroups, long long nblocks, int n_override) {
  typedef typename MfmaOp<T>::acc_t acc_t;
  __shared__ T As[BK][BM + 1];
  __shared__ T Bs[BK][BN + 1];

  const long long lb = xcd_remap(blockIdx.x, nblocks);
  const G* g = find_group(groups, ngroups, lb);
  const int ks_n = g->ksplit > 1 ? g->ksplit : 1;
  const long long rel0 = lb - g->first_block;
  const int ks = (int)(rel0 % ks_n);
  const long long rel = rel0 / ks_n;
  const int tiles = g->tiles_m * g->tiles_n;
  const long long bat = rel / tiles;
  const int tile = (int)(rel - bat * tiles);
  const int tm = tile % g->tiles_m, tn = tile / g->tiles_m;
  if (g->gate && g->gate[bat] == 0) return;  // whole workgroup, before any barrier
  const int M = g->M, K = g->K;
  const int N = (n_override > 0 && n_override < g->N) ? n_override : g->N;
  const int i0 = tm * BM, j0 = tn * BN;
  const int lda = g->lda, ldb = g->ldb;
  const T* Abase = g->A + bat * g->sA;
  const T* Bbase = g->B + bat * g->sB;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;

  acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

  // The next k-tile's global loads are issued into registers before the
  // current tile's MFMAs, so their latency overlaps the math.
  T ra[4], rb[4];
  auto load_tiles = [&](const T* A, const T* B, int k0, int kend) {
    if (!TA) {
      const int i = tid & 63, kk = tid >> 6;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = i0 + i, gk = k0 + kk + 4 * r;
        ra[r] = (gi < M && gk < kend) ? A[gi + (long long)gk * lda] : T(0);
      }
    } else {
      const int k = tid & 15, ii = tid >> 4;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = i0 + ii + 16 * r, gk = k0 + k;
        ra[r] = (gi < M && gk < kend) ? A[gk + (long long)gi * lda] : T(0);
      }
    }
    if (!TB) {
      const int k = tid & 15, jj = tid >> 4;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gj = j0 + jj + 16 * r, gk = k0 + k;
        rb[r] = (gj < N && gk < kend) ? B[gk + (long long)gj * ldb] : T(0);
      }
    } else {
      const int j = tid & 63, kk = tid >> 6;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gj = j0 + j, gk = k0 + kk + 4 * r;
        rb[r] = (gj < N && gk < kend) ? B[gj + (long long)gk * ldb] : T(0);
      }
    }
  };
  auto store_tiles = [&]() {
    if (!TA) {
      const int i = tid & 63, kk = tid >> 6;
#pragma unroll
      for (int r = 0; r < 4; ++r) As[kk + 4 * r][i] = ra[r];
    } else {
      const int k = tid & 15, ii = tid >> 4;
#pragma unroll
      for (int r = 0; r < 4; ++r) As[k][ii + 16 * r] = ra[r];
    }
    if (!TB) {
      const int k = tid & 15, jj = tid >> 4;
#pragma unroll
      for (int r = 0; r < 4; ++r) Bs[k][jj + 16 * r] = rb[r];
    } else {
      const int j = tid & 63, kk = tid >> 6;
#pragma unroll
      for (int r = 0; r < 4; ++r) Bs[kk + 4 * r][j] = rb[r];
    }
  };

  const int kbeg = ks_n > 1 ? ks * g->kchunk : 0;
  const int kend = ks_n > 1 ? min(K, kbeg + g->kchunk) : K;
  for (int s = 0; s < g->nseg; ++s) {
    const T* A = Abase + g->aseg[s];
    const T* B = Bbase + g->bseg[s];
    if (kbeg < kend) load_tiles(A, B, kbeg, kend);
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
      store_tiles();
      __syncthreads();
      if (k0 + BK < kend) load_tiles(A, B, k0 + BK, kend);
#pragma unroll
      for (int ks = 0; ks < BK / 4; ++ks) {
        const int k = 4 * ks + (lane >> 4);
        T af[2], bf[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) af[a] = As[k][wr * 32 + a * 16 + (lane & 15)];
#pragma unroll
        for (int b = 0; b < 2; ++b) bf[b] = Bs[k][wc * 32 + b * 16 + (lane & 15)];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) acc[a][b] = MfmaOp<T>::run(bf[b], af[a], acc[a][b]);
      }
      __syncthreads();
    }
  }
  // ---- epilogue: acc[a][b][v] = C(row = .. + lane%16, col = .. + MfmaOp<T>::col(lane, v))
  if (ks_n > 1) {  // split-K: store the raw partial product of this K range
    T* W = g->part + (bat * ks_n + ks) * (long long)M * g->N;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int row = i0 + wr * 32 + a * 16 + (lane & 15);
      if (row >= M) continue;
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int col = j0 + wc * 32 + b * 16 + MfmaOp<T>::col(lane, v);
          if (col < N) W[row + (long long)col * M] = acc[a][b][v];
        }
    }
    return;
  }
  T* C = g->C + bat * g->sC;
  const T* C0 = g->C0 ? g->C0 + bat * g->sC0 : nullptr;
  const T alpha = g->alpha, beta = g->beta;
  const int ldc = g->ldc, ldc0 = g->ldc0;
  // C0 may alias C: every C0 value of the tile is loaded (all loads in
  // flight together) before the first store
  T c0v[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int row = i0 + wr * 32 + a * 16 + (lane & 15);
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = j0 + wc * 32 + b * 16 + MfmaOp<T>::col(lane, v);
        c0v[a][b][v] = (beta != T(0) && row < M && col < N) ? C0[row + (long long)col * ldc0] : T(0);
      }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int row = i0 + wr * 32 + a * 16 + (lane & 15);
    if (row >= M) continue;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = j0 + wc * 32 + b * 16 + MfmaOp<T>::col(lane, v);
        if (col >= N) continue;
        T val = alpha * acc[a][b][v];
        if (beta != T(0)) val += beta * c0v[a][b][v];
        C[row + (long long)col * ldc] = val;
      }
    }
  }
}

// Skinny products (N <= 16, as in the solve: one column per right-hand side),
// A and B not transposed.  The same block / tile / split-K decomposition as
// gemm_grouped_kernel, but each wavefront owns 16 rows of the 64-row tile and
// reads its MFMA fragments straight from memory: no LDS staging, no barriers.
// Loads go out at clamped, valid addresses; out-of-range rows, columns and k
// are masked where used.
constexpr int SKK = 2;
template <typename T, typename G>
__global__ __launch_bounds__(GEMM_THREADS) void gemm_skinny_kernel(const G* __restrict__ groups, int ngroups,
                                                                   long long nblocks, int n_override) {
  typedef typename MfmaOp<T>::acc_t acc_t;
  const long long lb = xcd_remap(blockIdx.x, nblocks);
  const G* g = find_group(groups, ngroups, lb);
  const int ks_n = g->ksplit > 1 ? g->ksplit : 1;
  const long long rel0 = lb - g->first_block;
  const int ks = (int)(rel0 % ks_n);
  const long long rel = rel0 / ks_n;
  const int tiles = g->tiles_m * g->tiles_n;
  const long long bat = rel / tiles;
  const int tile = (int)(rel - bat * tiles);
  const int tm = tile % g->tiles_m, tn = tile / g->tiles_m;
  if (tn > 0) return;  // columns past 64: none when N <= 16
  if (g->gate && g->gate[bat] == 0) return;
  const int M = g->M, K = g->K;
  const int N = (n_override > 0 && n_override < g->N) ? n_override : g->N;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = tm * BM + 16 * wave;  // this wavefront's rows r0 .. r0 + 15
  if (r0 >= M) return;                 // wave-uniform
  const int lda = g->lda, ldb = g->ldb;
  const int arow = r0 + (lane & 15), bcol = lane & 15, kl = lane >> 4;
  const bool arow_ok = arow < M, bcol_ok = bcol < N;
  const int arow_c = arow_ok ? arow : M - 1, bcol_c = bcol_ok ? bcol : N - 1;
  const int kbeg = ks_n > 1 ? ks * g->kchunk : 0;
  const int kend = ks_n > 1 ? min(K, kbeg + g->kchunk) : K;
  acc_t acc = acc_t{0, 0, 0, 0};
  const int nseg = kbeg < kend ? g->nseg : 0;  // an empty K range reads nothing
  for (int s = 0; s < nseg; ++s) {
    const gmem<T>* A = gptr(g->A) + bat * g->sA + g->aseg[s];
    const gmem<T>* B = gptr(g->B) + bat * g->sB + g->bseg[s];
    // two register buffers of SKK k-steps each: the loads of one are in
    // flight while the MFMAs of the other run.  Loads past the end of the K
    // range re-read (clamped) the last k; their MFMAs add zeros.
    T af[SKK], bf[SKK], an[SKK], bn[SKK];
    auto load = [&](T* a_, T* b_, int k0) {
#pragma unroll
      for (int u = 0; u < SKK; ++u) {
        const int k = min(k0 + 4 * u + kl, kend - 1);
        a_[u] = A[arow_c + (long long)k * lda];
        b_[u] = B[k + (long long)bcol_c * ldb];
      }
    };
    auto mma = [&](const T* a_, const T* b_, int k0) {
#pragma unroll
      for (int u = 0; u < SKK; ++u) {
        const bool kok = k0 + 4 * u + kl < kend;
        acc = MfmaOp<T>::run((kok && bcol_ok) ? b_[u] : T(0), (kok && arow_ok) ? a_[u] : T(0), acc);
      }
    };
    load(af, bf, kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += 8 * SKK) {
      load(an, bn, k0 + 4 * SKK);
      mma(af, bf, k0);
      load(af, bf, k0 + 8 * SKK);
      mma(an, bn, k0 + 4 * SKK);
    }
  }
  // epilogue: acc[v] = C(row = arow, col = MfmaOp<T>::col(lane, v))
  if (ks_n > 1) {
    gmem<T>* W = gptr(g->part) + (bat * ks_n + ks) * (long long)M * g->N;
    if (arow_ok)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = MfmaOp<T>::col(lane, v);
        if (col < N) W[arow + (long long)col * M] = acc[v];
      }
    return;
  }
  gmem<T>* C = gptr(g->C) + bat * g->sC;
  const gmem<T>* C0 = g->C0 ? gptr(g->C0) + bat * g->sC0 : nullptr;
  const T alpha = g->alpha, beta = g->beta;
  T c0v[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int col = MfmaOp<T>::col(lane, v);
    c0v[v] = (beta != T(0) && arow_ok && col < N) ? C0[arow + (long long)col * g->ldc0] : T(0);
  }
  if (!arow_ok) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int col = MfmaOp<T>::col(lane, v);
    if (col >= N) continue;
    T val = alpha * acc[v];
    if (beta != T(0)) val += beta * c0v[v];
    C[arow + (long long)col * g->ldc] = val;
  }
}

// Second pass of a split-K product: C = alpha * sum_ks part_ks + beta * C0,
// the partials added in ks order (deterministic).  One thread per element.
constexpr int RED_THREADS = 256;
template <typename T, typename G>
__global__ __launch_bounds__(RED_THREADS) void gemm_splitk_reduce_kernel(const G* __restrict__ groups, int ngroups,
                                                                         int n_override) {
  const long long rb = blockIdx.x;
  int lo = 0, hi = ngroups - 1;
  while (lo < hi) {  // last group with first_rblock <= rb
    const int mid = (lo + hi + 1) >> 1;
    if (groups[mid].first_rblock <= rb) lo = mid;
    else hi = mid - 1;
  }
  const G* g = groups + lo;
  const int M = g->M, Nf = g->N, ks_n = g->ksplit;
  const int N = (n_override > 0 && n_override < Nf) ? n_override : Nf;
  const long long e = (rb - g->first_rblock) * RED_THREADS + threadIdx.x;
  const long long mn = (long long)M * Nf;
  const long long bat = e / mn;
  if (bat >= g->batch) return;
  if (g->gate && g->gate[bat] == 0) return;
  const int rem = (int)(e - bat * mn);
  const int col = rem / M, row = rem - col * M;
  if (col >= N) return;
  const gmem<T>* W = gptr(g->part) + bat * ks_n * mn + row + (long long)col * M;
  T sum = T(0);
  for (int k = 0; k < ks_n; ++k) sum += W[k * mn];
  T val = g->alpha * sum;
  if (g->beta != T(0)) val += g->beta * gptr(g->C0)[bat * g->sC0 + row + (long long)col * g->ldc0];
  gptr(g->C)[bat * g->sC + row + (long long)col * g->ldc] = val;
}

template <typename G>
static long long prepare_groups(std::vector<G>& groups) {
  long long total = 0, rtotal = 0;
  for (auto& g : groups) {
    g.tiles_m = (g.M + BM - 1) / BM;
    g.tiles_n = (g.N + BN - 1) / BN;
    const int ks = g.ksplit > 1 ? g.ksplit : 1;
    g.first_block = total;
    g.first_rblock = rtotal;
    if (g.M > 0 && g.N > 0) {
      total += (long long)g.tiles_m * g.tiles_n * g.batch * ks;
      if (ks > 1) rtotal += ((long long)g.batch * g.M * g.N + RED_THREADS - 1) / RED_THREADS;
    }
  }
  return total;
}

template <typename G>
static long long rblocks_of(const std::vector<G>& groups) {
  long long r = 0;
  for (const auto& g : groups)
    if (g.ksplit > 1 && g.M > 0 && g.N > 0) r += ((long long)g.batch * g.M * g.N + RED_THREADS - 1) / RED_THREADS;
  return r;
}

// Choose split-K factors for a launch that would otherwise fill few
// workgroups (skinny products: the solve's N <= 16 right-hand sides against
// large operators): aim at ~1024 workgroups, K ranges of >= 256.  Assigns
// each split group a workspace offset (consecutive from 0) and returns the
// workspace elements the launch needs.
template <typename G>
static long long plan_split(std::vector<G>& groups) {
  long long tiles = 0;
  for (auto& g : groups) {
    g.ksplit = 1;
    g.kchunk = 0;
    g.part_off = 0;
    tiles += (long long)((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN) * g.batch;
  }
  if (tiles == 0 || tiles >= 512) return 0;
  const long long want = (1024 + tiles - 1) / tiles;
  long long off = 0;
  for (auto& g : groups) {
    long long ks = std::min<long long>(want, g.K / 256);
    if (ks < 2) continue;
    int kchunk = (int)((g.K + ks - 1) / ks);
    kchunk = (kchunk + BK - 1) / BK * BK;
    ks = (g.K + kchunk - 1) / kchunk;
    if (ks < 2) continue;
    g.ksplit = (int)ks;
    g.kchunk = kchunk;
    g.part_off = off;
    off += (long long)g.batch * ks * g.M * g.N;
  }
  return off;
}

// Launch a grouped GEMM whose descriptors already live in device memory
// (dev_groups) and whose host copy (with first_block filled by
// gemm_prepare) is `groups`.
long long gemm_prepare(std::vector<GemmGroup>& groups) { return prepare_groups(groups); }
long long gemm_prepare_f32(std::vector<GemmGroupF32>& groups) { return prepare_groups(groups); }
long long gemm_rblocks(const std::vector<GemmGroup>& groups) { return rblocks_of(groups); }
long long gemm_rblocks_f32(const std::vector<GemmGroupF32>& groups) { return rblocks_of(groups); }
long long gemm_plan_split(std::vector<GemmGroup>& groups) { return plan_split(groups); }
long long gemm_plan_split_f32(std::vector<GemmGroupF32>& groups) { return plan_split(groups); }

int gemm_launch(const GemmGroup* dev_groups, int ngroups, long long nblocks, long long nrblocks, bool ta, bool tb,
                hipStream_t st, int n_override) {
  if (nblocks <= 0) return HPS_OK;
  dim3 grid((unsigned)nblocks), block(GEMM_THREADS);
  if (!ta && !tb && n_override > 0 && n_override <= 16)
    hipLaunchKernelGGL((gemm_skinny_kernel<double, GemmGroup>), grid, block, 0, st, dev_groups, ngroups, nblocks, n_override);
  else if (!ta && !tb)
    hipLaunchKernelGGL((gemm_grouped_kernel<double, GemmGroup, false, false>), grid, block, 0, st, dev_groups, ngroups, nblocks, n_override);
  else if (ta && !tb)
    hipLaunchKernelGGL((gemm_grouped_kernel<double, GemmGroup, true, false>), grid, block, 0, st, dev_groups, ngroups, nblocks, n_override);
  else if (!ta && tb)
    hipLaunchKernelGGL((gemm_grouped_kernel<double, GemmGroup, false, true>), grid, block, 0, st, dev_groups, ngroups, nblocks, n_override);
  else
    hipLaunchKernelGGL((gemm_grouped_kernel<double, GemmGroup, true, true>), grid, block, 0, st, dev_groups, ngroups, nblocks, n_override);
  HPS_HIP_TRY(hipGetLastError());
  if (nrblocks > 0) {
    hipLaunchKernelGGL((gemm_splitk_reduce_kernel<double, GemmGroup>), dim3((unsigned)nrblocks), dim3(RED_THREADS), 0,
                       st, dev_groups, ngroups, n_override);
    HPS_HIP_TRY(hipGetLastError());
  }
  return HPS_OK;
}

int gemm_launch_f32(const GemmGroupF32* dev_groups, int ngroups, long long nblocks, long long nrblocks, bool ta,
                    bool tb, hipStream_t st, int n_override) {
  if (nblocks <= 0) return HPS_OK;
  dim3 grid((unsigned)nblocks), block(GEMM_THREADS);
  if (!ta && !tb && n_override > 0 && n_override <= 16)
    hipLaunchKernelGGL((gemm_skinny_kernel<float, GemmGroupF32>), grid, block, 0, st, dev_groups, ngroups, nblocks, n_override);
  else if (!ta && !tb)
    hipLaunchKernelGGL((gemm_grouped_kernel<float, GemmGroupF32, false, false>), grid, block, 0, st, dev_groups, ngroups, nblocks, n_override);
  else if (ta && !tb)
    hipLaunchKernelGGL((gemm_grouped_kernel<float, GemmGroupF32, true, false>), grid, block, 0, st, dev_groups, ngroups, nblocks, n_override);
  else if (!ta && tb)
    hipLaunchKernelGGL((gemm_grouped_kernel<float, GemmGroupF32, false, true>), grid, block, 0, st, dev_groups, ngroups, nblocks, n_override);
  else
    hipLaunchKernelGGL((gemm_grouped_kernel<float, GemmGroupF32, true, true>), grid, block, 0, st, dev_groups, ngroups, nblocks, n_override);
  HPS_HIP_TRY(hipGetLastError());
  if (nrblocks > 0) {
    hipLaunchKernelGGL((gemm_splitk_reduce_kernel<float, GemmGroupF32>), dim3((unsigned)nrblocks), dim3(RED_THREADS),
                       0, st, dev_groups, ngroups, n_override);
    HPS_HIP_TRY(hipGetLastError());
  }
  return HPS_OK;
}

}  // namespace hps
