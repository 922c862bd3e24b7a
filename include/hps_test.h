/* Test hooks of the HPS library: inspection of a built operator's internal
 * buffers, the library's GEMM kernels on a single product, and the host
 * precompute.  They are exported by libhps.so for the test suite and are not
 * part of the solver's interface (include/hps.h). */
#ifndef HPS_TEST_H_
#define HPS_TEST_H_

#include "hps.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Operator inspection, for tests: copies an internal device buffer of a
 * built operator to host memory (synchronizes the op's stream).  which:
 *   0 leaf LU factors   [n_leaves][n_i*n_i]  (2D: column s = U(0..s, s) in pivot order,
 *                                              then the L entries of the rows not yet
 *                                              pivoted after step s, in row order;
 *                                              3D: L_ii^{-1}, column-major)
 *   1 leaf pivot order  [n_leaves][n_i]      (as doubles)
 *   2 leaf Y_int        [n_leaves][n_i*n_b]  (column-major)
 *   3 leaf T            [n_leaves][n_b*n_b]
 *   4 merge D^{-1} of tree level `level`   [merges][m*m]
 *   5 merge S of tree level `level`        [merges][m*n_parent]
 *   6 merge parent T of tree level `level` [merges][n_parent^2]
 * For an ItI operator (real representation of complex data, 2p^2 reals per
 * leaf): 0 is (S B)^{-1} [n_leaves][(2p^2)^2], S the row equilibration of
 * B, and 2 is Y [n_leaves][2p^2 * n_b],
 * both column-major; T below the root is build workspace (levels reuse it).
 * Returns the number of doubles written, or a negative error code. */
long long hps_debug_download(const hps_op_t* op, int which, int level, double* out, long long cap);

/* Kernel check, for tests: the library's grouped MFMA GEMM on one product,
 *   C = alpha op(A) op(B) + beta C   (column-major, dev pointers, fp64),
 * op(X) = X or X^T per trans_a / trans_b.  With n <= 16 and neither operand
 * transposed it runs the skinny kernel the solve uses.  Asynchronous on
 * `stream`. */
int hps_debug_gemm(int m, int n, int k, double alpha, const double* a, int lda, int trans_a,
                   const double* b, int ldb, int trans_b, double beta, double* c, int ldc,
                   void* stream);

/* The same GEMM kernel with fp32 operands and fp32 accumulation (the
 * mixed-precision solve's products), for tests. */
int hps_debug_gemm_f32(int m, int n, int k, float alpha, const float* a, int lda, int trans_a,
                       const float* b, int ldb, int trans_b, float beta, float* c, int ldc,
                       void* stream);

/* Host precompute inspection, for tests (no device work).  which:
 *   0 Chebyshev nodes (p), 1 Gauss nodes (q), 2 Gauss weights (q),
 *   3 D (p x p), 4 P (n_e x n_b), 5 Q on [-1,1]^dim (n_b x p^dim),
 *   6 interior index list I_i (n_i), 7 exterior index list I_e (n_e)
 * Writes row-major into out (capacity cap doubles) and the shape into
 * rows/cols. */
int hps_precompute_matrix(int dim, int p, int which, double* out, long long cap,
                          int* rows, int* cols);

#ifdef __cplusplus
}
#endif
#endif /* HPS_TEST_H_ */
