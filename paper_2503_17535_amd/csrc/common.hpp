// Shared definitions of the HPS HIP library (host + device).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace hps {

// ---------------------------------------------------------------------------
// Grouped, strided-batched fp64 GEMM descriptor.
//   C[b] = alpha * sum_{s < nseg} op(A)[b, s] op(B)[b, s] + beta * C0[b]
// op(A)[b,s] is M x K starting at A + b*sA + aseg[s] (leading dim lda),
// op(B)[b,s] is K x N starting at B + b*sB + bseg[s] (leading dim ldb),
// all column-major.  beta == 0 never reads C0.
// ---------------------------------------------------------------------------
constexpr int kMaxSeg = 3;
struct GemmGroup {
  const double* A;
  const double* B;
  double* C;
  const double* C0;
  long long sA, sB, sC, sC0;
  long long aseg[kMaxSeg], bseg[kMaxSeg];
  int lda, ldb, ldc, ldc0;
  int M, N, K, nseg;
  double alpha, beta;
  int batch;
  // split-K: ksplit workgroups per tile each sum a K range of kchunk; their
  // partial products go to part (+ batch item * ksplit * M * N) and a second
  // pass adds them in a fixed order (ksplit <= 1: no split)
  int ksplit, kchunk;
  long long part_off;
  double* part;
  // gate[b] == 0 skips batch item b (NULL: every item runs); read on the
  // device, so a kernel earlier on the stream can switch items on and off
  const int* gate;
  // filled by the launcher
  int tiles_m, tiles_n;
  long long first_block, first_rblock;
};

// Same for fp32 operands with fp32 accumulation (mixed-precision solve).
struct GemmGroupF32 {
  const float* A;
  const float* B;
  float* C;
  const float* C0;
  long long sA, sB, sC, sC0;
  long long aseg[kMaxSeg], bseg[kMaxSeg];
  int lda, ldb, ldc, ldc0;
  int M, N, K, nseg;
  float alpha, beta;
  int batch;
  int ksplit, kchunk;
  long long part_off;
  float* part;
  const int* gate;
  int tiles_m, tiles_n;
  long long first_block, first_rblock;
};

// ---------------------------------------------------------------------------
// Block copy/add: dst block (rows x cols, column-major, ld dst_ld) =
//   sum of up to two source blocks (or zero).  Sources come from one of two
//   base buffers (src_buf 0 / 1).  Offsets are relative to the batch item's
//   base (base + b * stride).
// ---------------------------------------------------------------------------
struct BlockOp {
  long long dst_off;
  long long src_off[2];
  int dst_ld;
  int src_ld[2];
  int src_buf[2];
  int nsrc;
  int rows, cols;
};

// Work decomposition of a table of BlockOps: an item is a column range of one
// op (c1 < 0: all runtime columns); a task (one workgroup per batch item) is a
// run of consecutive items, sized so that every workgroup moves a similar
// number of elements.  Items of a task with per_wave = 0 are copied one after
// the other by the whole workgroup; with per_wave = 1 (small items) each
// wavefront copies every fourth item of the task on its own.
struct CopyItem {
  int op, r0, r1, c0, c1;  // rows [r0, r1), columns [c0, c1) (c1 < 0: the run-time column count)
};
struct CopyTask {
  int begin, end, per_wave;
};

// ---------------------------------------------------------------------------
// Batched solve over several operators: one launch per pass stage covers the
// work of every operator in the batch.  A job is one operator's share of a
// launch; `first_block` is the prefix sum of the blocks of earlier jobs.
// ---------------------------------------------------------------------------
constexpr int kBatchMaxRhs = 16;

struct LeafJob {
  const double *LU, *Y, *P, *g;
  const int *perm, *pos, *Ii, *Ie;
  double *v, *g0;
  int NI, NE, NB, npts, nrhs, NRcap, nb0;
  long long nl, first_block;
  const double* bdry[kBatchMaxRhs];
  const double* src[kBatchMaxRhs];  // NULL entries mean f = 0
  double* u[kBatchMaxRhs];
};

struct CopyJob {
  const BlockOp* ops;
  const CopyItem* items;
  const CopyTask* tasks;  // the call's first task
  int ntasks, ncols_rt;
  long long batch, first_block;
  double* dst;
  long long dst_stride;
  const double* src0;
  long long s0_stride;
  const double* src1;
  long long s1_stride;
};

// error reporting (implemented in api.cpp)
void set_error(const std::string& msg);

}  // namespace hps

#define HPS_HIP_TRY(expr)                                                          \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess) {                                                        \
      ::hps::set_error(std::string(#expr " failed: ") + hipGetErrorString(_e));    \
      return HPS_EDEVICE;                                                          \
    }                                                                              \
  } while (0)
