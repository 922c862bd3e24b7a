// C ABI of the HPS solver: host orchestration of the build and solve stages.
//
// Build (Algorithm "Local solve stage" + Algorithm "Merge stage"):
//   leaves   fused factor kernel -> LU(L_ii), Y_int;  T = Q_e P + Q_i Y_int (GEMM)
//   level l  (l = L-1 .. 0, parents on tree level l)
//            D   = sum of child DtN blocks on shared interfaces (gather)
//            Z   = D^{-1}                      (register GJ or blocked GJ)
//            S   = -Z C                        (grouped GEMM, C's zero blocks skipped)
//            Bnz = nonzero blocks of B         (gather; kept for the solve)
//            T   = A + B S                     (gather of A + grouped GEMM; not at the root)
// Solve (source split of Section 3 + Algorithm "Downward pass"):
//   up       v = L_ii^{-1} f, h = Q_i v; per level gt = -Z h_int, h = h_ext + B gt
//   down     per level g_int = S g + gt, children g cut from [g; g_int]
//   leaves   u = [P g; Y_int g + v]
#include <hip/hip_runtime.h>

#include <algorithm>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/hps.h"
#include "../../include/hps_test.h"
#include "common.hpp"
#include "op.hpp"
#include "precompute.hpp"

namespace hps {

// launchers (kernels in the .hip files)
int leaf2d_launch(int p, const double* coeffs, const double* D1, const double* D2, const double* Mt, double* LU,
                  int* perm, int* pos, double* Y, int* flag, long long nl, hipStream_t st);
int gj_small_max();
int gj_small_launch(const double* D, double* Z, int m, int* flag, long long batch, hipStream_t st);
int gj_panel_width(int m);
int gj_panel_max_nb();
int gj_update_launch(double* A, const double* W, const int* piv, int m, int j0, int w, long long batch,
                     hipStream_t st, int cb, int cw);
int gj_block_prep_launch(const double* A, const int* piv, int m, int b0, int w, int ob, double* Wk, double* Pk,
                         long long batch, hipStream_t st);
int gj_panel_launch(double* A, int m, int j0, int nbw, int* pos, int* piv, double* W, int* flag,
                    long long batch, hipStream_t st);
int gj_step_launch(double* A, int m, int j0, int nbw, int* pos, int* piv, double* W, const double* Wp, int wp,
                   int* flag, long long batch, hipStream_t st, int cb, int cw);
int gj_init_launch(int* pos, long long n, hipStream_t st);
int gj_unscramble_launch(const double* R, double* Z, int m, const int* pos, const int* piv, long long batch,
                         hipStream_t st);
int leaf3d_assemble_launch(const double* coeffs, const double* D1, const double* D2, const double* Mt, int p,
                           double* Lii, double* R, long long nl, hipStream_t st);
int leaf_gather_int_launch(const double* src, const int* Ii, int ni, int npts, long long nl, int nrhs, int NRcap,
                           double* fint, hipStream_t st);
int leaf_gather_pts_launch(const double* w, const int* idx, int n, int npts, long long nl, int nrhs, int NRcap,
                           double* out, hipStream_t st,
                           long long rstride = 0);
int leaf_scatter_int_launch(const double* fint, const int* pos_i, int ni, int npts, long long nl, int nrhs, int NRcap,
                            double* lam, hipStream_t st,
                            long long rstride = 0);
int leaf_src_t_launch(const double* LU, const int* perm, const double* b, int NI, long long nl, int nrhs, int NRcap,
                      double* x, hipStream_t st);
int block_copy_launch_f32(const BlockOp* dev_ops, const CopyItem* dev_items, const CopyTask* dev_tasks, int ntasks,
                          int ncols_rt, float* dst, long long dst_stride, const float* src0, long long s0_stride,
                          const float* src1, long long s1_stride, long long batch, hipStream_t st);
int leaf_src_f32_launch(const float* LU, const int* perm, const int* pos, const double* r, int NI, long long nl,
                        int nrhs, int NRcap, float* v, hipStream_t st);
int to_f32_launch(const double* src, float* dst, long long n, hipStream_t st);
int refine_init_launch(const double* bdry, const long long* bidx, int q, int nb0, long long nl, int nrhs, int NRcap,
                       double* gam, hipStream_t st);
int refine_residual_launch(const double* coef, const double* src, const double* gam, const double* D1,
                           const double* D2, const double* P, const double* C2G, const int* Ii, const int* Ie, int p,
                           long long nl, int nrhs, int NRcap, double* u, double* r1, double* Qu, hipStream_t st);
int refine_flux_launch(const double* Qu, const int* nbr, int q, long long nl, int nrhs, int NRcap, float* hx,
                       hipStream_t st);
int refine_update_launch(const float* dg, const float* Y32, const float* v32, const int* Ii, int ni, int nb, int npts,
                         long long nl, int nrhs, int NRcap, double* gam, double* u, hipStream_t st);
int coeff_grad_launch(int d, int p, const double* u, const double* lam, const double* D1, const double* D2,
                      long long nl, int nrhs, double* grad, hipStream_t st);
int block_copy_launch(const BlockOp* dev_ops, const CopyItem* dev_items, const CopyTask* dev_tasks, int ntasks,
                      int ncols_rt, double* dst, long long dst_stride, const double* src0, long long s0_stride,
                      const double* src1, long long s1_stride, long long batch, hipStream_t st);
int leaf_src_launch(const double* LU, const int* perm, const int* pos, const double* src, const int* Ii, int NI,
                    int npts, long long nl, int nrhs, double* v, int NRcap, hipStream_t st, long long rstride = 0,
                    int max_wg_per_cu = 0);
int leaf_out_launch(const double* Y, const double* P, const double* g, const double* v, const int* Ii, const int* Ie,
                    int NI, int NE, int NB, int npts, long long nl, int nrhs, int NRcap, double* u, hipStream_t st,
                    long long rstride = 0);
int probe_reduce_launch(const double* r, long long stride, int m, double inv_xmax, double tau, double* rho,
                        int* gate, long long nodes, hipStream_t st);
int gated_copy_launch(double* dst, const double* src, long long n, const int* gate, long long nodes,
                      hipStream_t st);
int static_ws_ptr(void** out);
int iti_leaf_assemble_launch(const double* coeffs, const double* D1, const double* D2, const double* Gr,
                             const int* Ii, int p, long long nl, double* scale, double* B, hipStream_t st);
int iti_gather_src_launch(const double* src, const int* Iir, const double* scale, int ni2, int m, long long nl,
                          int nrhs, int NRcap, double* fint, hipStream_t st);
int zero_fill_launch(double* x, long long n, hipStream_t st);

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }


// ---------------------------------------------------------------------------
// device memory: a size-keyed cache of freed blocks, so repeated builds of the
// same shape reuse their allocations instead of calling hipMalloc again.  The
// cache holds at most kCacheBytes, in blocks of at most kCacheBlock; larger
// blocks, and blocks beyond that total, go back to the device at once, so
// that memory freed by the library is available to other allocators (a build
// of a deep tree hands back hundreds of gigabytes).
// ---------------------------------------------------------------------------
namespace {
std::mutex g_pool_mu;
std::multimap<size_t, void*> g_pool_free;
size_t g_cached = 0;
constexpr size_t kCacheBytes = 16ull << 30;
constexpr size_t kCacheBlock = 2ull << 30;

// bytes handed out by dalloc and not returned, and their high-water mark
size_t g_in_use = 0, g_peak = 0;

size_t round_size(size_t b) { return (b + 4095) & ~(size_t)4095; }

void count_out(size_t bytes) {
  g_in_use += bytes;
  if (g_in_use > g_peak) g_peak = g_in_use;
}

// allocator callback (hps_set_allocator): operator blocks come from it when set
hps_alloc_fn g_cb_alloc = nullptr;
hps_free_fn g_cb_free = nullptr;
void* g_cb_ctx = nullptr;

void* dalloc(size_t bytes) {
  bytes = round_size(bytes ? bytes : 1);
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    auto it = g_pool_free.find(bytes);
    if (it != g_pool_free.end()) {
      void* p = it->second;
      g_pool_free.erase(it);
      g_cached -= bytes;
      count_out(bytes);
      return p;
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    // release cached blocks and retry once
    std::lock_guard<std::mutex> lk(g_pool_mu);
    (void)hipDeviceSynchronize();
    for (auto& kv : g_pool_free) (void)hipFree(kv.second);
    g_pool_free.clear();
    g_cached = 0;
    (void)hipGetLastError();
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  std::lock_guard<std::mutex> lk(g_pool_mu);
  count_out(bytes);
  return p;
}

void dfree(void* p, size_t bytes) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  const size_t b = round_size(bytes ? bytes : 1);
  g_in_use -= b;
  if (b > kCacheBlock || g_cached + b > kCacheBytes) {
    (void)hipFree(p);  // callers (hps_free) have waited for the device
    return;
  }
  g_pool_free.emplace(b, p);
  g_cached += b;
}

// An operator's block: from the allocator callback when one is set (its
// free function and context are recorded in *rec), else from the pool.
void* op_dalloc(size_t bytes, Alloc* rec) {
  hps_alloc_fn a = nullptr;
  hps_free_fn f = nullptr;
  void* ctx = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    a = g_cb_alloc;
    f = g_cb_free;
    ctx = g_cb_ctx;
  }
  rec->cb_free = nullptr;
  rec->cb_ctx = nullptr;
  if (!a) return dalloc(bytes);
  const size_t b = round_size(bytes ? bytes : 1);
  void* p = a(b, ctx);  // the callback runs outside the pool lock
  if (!p) return nullptr;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  count_out(b);
  rec->cb_free = f;
  rec->cb_ctx = ctx;
  return p;
}

void op_dfree(const Alloc& al) {
  if (!al.cb_free) {
    dfree(al.p, al.bytes);
    return;
  }
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    g_in_use -= round_size(al.bytes ? al.bytes : 1);
  }
  al.cb_free(al.p, round_size(al.bytes ? al.bytes : 1), al.cb_ctx);
}

// device copies of the precomputed leaf operators, per (d, p, leaf half-width)
std::mutex g_cst_mu;
std::map<std::tuple<int, int, double>, DevConsts> g_cst;

template <typename T>
int upload(T** dst, const std::vector<T>& host) {
  *dst = (T*)dalloc(host.size() * sizeof(T));
  if (!*dst) { set_error("device allocation failed (constants)"); return HPS_ENOMEM; }
  HPS_HIP_TRY(hipMemcpy(*dst, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice));
  return HPS_OK;
}

int get_consts(int d, int p, double r, DevConsts** out) {
  std::lock_guard<std::mutex> lk(g_cst_mu);
  auto key = std::make_tuple(d, p, r);
  auto it = g_cst.find(key);
  if (it != g_cst.end()) { *out = &it->second; return HPS_OK; }
  const LeafOps& o = leaf_ops(d, p);
  DevConsts c;
  const int n_i = o.n_i, n_e = o.n_e, n_b = o.n_b, np = o.npts;
  // 1D derivative matrices on the leaf (row-major)
  std::vector<double> D1((size_t)p * p), D2((size_t)p * p, 0.0);
  for (int i = 0; i < p * p; ++i) D1[i] = o.D[i] / r;
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j) {
      double s = 0.0;
      for (int k = 0; k < p; ++k) s += D1[(size_t)i * p + k] * D1[(size_t)k * p + j];
      D2[(size_t)i * p + j] = s;
    }
  // Q on the leaf, split into interior / exterior columns (column-major)
  std::vector<double> Qi((size_t)n_b * n_i), Qe((size_t)n_b * n_e);
  for (int b = 0; b < n_b; ++b) {
    for (int k = 0; k < n_i; ++k) Qi[b + (size_t)k * n_b] = o.Qref[(size_t)b * np + o.Ii[k]] / r;
    for (int k = 0; k < n_e; ++k) Qe[b + (size_t)k * n_b] = o.Qref[(size_t)b * np + o.Ie[k]] / r;
  }
  std::vector<double> QeP((size_t)n_b * n_b, 0.0), Pc((size_t)n_e * n_b);
  for (int e = 0; e < n_e; ++e)
    for (int b = 0; b < n_b; ++b) Pc[e + (size_t)b * n_e] = o.P[(size_t)e * n_b + b];
  for (int e = 0; e < n_e; ++e)
    for (int a = 0; a < n_b; ++a) {
      const double qa = Qe[a + (size_t)e * n_b];
      if (qa == 0.0) continue;
      for (int b = 0; b < n_b; ++b) QeP[a + (size_t)b * n_b] += qa * Pc[e + (size_t)b * n_e];
    }
  // M_t = D_t(I_i, I_e) P for every term, column-major n_i x n_b
  const int nt = n_terms(d);
  std::vector<double> Mt((size_t)nt * n_i * n_b, 0.0), blk;
  for (int t = 0; t < nt; ++t) {
    term_block(o, t, r, o.Ii, o.Ie, blk);  // n_i x n_e row-major, mostly zero (stencil)
    for (int i = 0; i < n_i; ++i)
      for (int e = 0; e < n_e; ++e) {
        const double l = blk[(size_t)i * n_e + e];
        if (l == 0.0) continue;
        for (int b = 0; b < n_b; ++b) Mt[(size_t)t * n_i * n_b + i + (size_t)b * n_i] += l * Pc[e + (size_t)b * n_e];
      }
  }
  HPS_TRY(upload(&c.D1, D1));
  HPS_TRY(upload(&c.D2, D2));
  HPS_TRY(upload(&c.Mt, Mt));
  HPS_TRY(upload(&c.QeP, QeP));
  HPS_TRY(upload(&c.Qi, Qi));
  HPS_TRY(upload(&c.P, Pc));
  HPS_TRY(upload(&c.Ii, o.Ii));
  HPS_TRY(upload(&c.Ie, o.Ie));
  HPS_TRY(upload(&c.PosI, o.pos_i));
  auto res = g_cst.emplace(key, c);
  *out = &res.first->second;
  return HPS_OK;
}

// ItI leaf constants (Appendix B.1) for leaves of half-width r, impedance
// parameter eta, in the real representation (see iti.hip).  The Robin rows
// of a corner belong to the side that starts at it on a counterclockwise walk
// (S and E keep their first p - 1 points, N and W their last p - 1).
std::map<std::tuple<int, double, double>, ItiConsts> g_iti_cst;

int get_iti_consts(int p, double r, double eta, ItiConsts** out) {
  std::lock_guard<std::mutex> lk(g_cst_mu);
  auto key = std::make_tuple(p, r, eta);
  auto it = g_iti_cst.find(key);
  if (it != g_iti_cst.end()) { *out = &it->second; return HPS_OK; }
  using cd = std::complex<double>;
  const LeafOps& o = leaf_ops(2, p);
  const MergeGeom& geo = merge_geom(2);
  const int q = p - 2, np = p * p, nr = 4 * p - 4, nbq = 4 * q;
  std::vector<double> D1((size_t)p * p);
  for (int i = 0; i < p * p; ++i) D1[i] = o.D[i] / r;
  // outward normal derivative at point pt of side f, as a row over the points
  auto normal = [&](int pt, int f, std::vector<cd>& row) {
    std::fill(row.begin(), row.end(), cd(0.0));
    const FaceDesc& fd = geo.faces[f];
    const double sign = fd.side ? 1.0 : -1.0;
    const int xy[2] = {pt % p, pt / p};
    const int ca = xy[fd.axis];
    for (int m = 0; m < p; ++m) {
      int c2[2] = {xy[0], xy[1]};
      c2[fd.axis] = m;
      row[c2[0] + p * c2[1]] += sign * D1[(size_t)ca * p + m];
    }
  };
  std::vector<cd> G((size_t)nr * np), H((size_t)4 * p * np), row(np);
  std::vector<double> P((size_t)nr * nbq, 0.0);
  int k = 0;
  for (int f = 0; f < 4; ++f) {
    const int t0 = (f == 0 || f == 1) ? 0 : 1;
    for (int t = t0; t < t0 + p - 1; ++t, ++k) {
      const int pt = o.face_cheb[f][t];
      normal(pt, f, row);
      row[pt] += cd(0.0, eta);                                   // G = N~ + i eta I
      for (int j = 0; j < np; ++j) G[(size_t)k * np + j] = row[j];
      for (int s = 0; s < q; ++s) P[(size_t)k * nbq + f * q + s] = o.G2C[(size_t)t * q + s];
    }
    for (int t = 0; t < p; ++t) {
      const int pt = o.face_cheb[f][t];
      normal(pt, f, row);
      row[pt] -= cd(0.0, eta);                                   // H = N - i eta I
      for (int j = 0; j < np; ++j) H[((size_t)f * p + t) * np + j] = row[j];
    }
  }
  // Q H: Chebyshev -> Gauss per side
  std::vector<cd> QH((size_t)nbq * np, cd(0.0));
  for (int f = 0; f < 4; ++f)
    for (int s = 0; s < q; ++s)
      for (int t = 0; t < p; ++t) {
        const double w = o.C2G[(size_t)s * p + t];
        for (int j = 0; j < np; ++j) QH[((size_t)f * q + s) * np + j] += w * H[((size_t)f * p + t) * np + j];
      }
  // real representations, column-major
  auto real_rep = [](const std::vector<cd>& M, int rows, int cols) {
    std::vector<double> R((size_t)4 * rows * cols);
    const size_t ld = 2 * (size_t)rows;
    for (int i = 0; i < rows; ++i)
      for (int j = 0; j < cols; ++j) {
        const cd z = M[(size_t)i * cols + j];
        R[(2 * j) * ld + 2 * i] = z.real();
        R[(2 * j) * ld + 2 * i + 1] = z.imag();
        R[(2 * j + 1) * ld + 2 * i] = -z.imag();
        R[(2 * j + 1) * ld + 2 * i + 1] = z.real();
      }
    return R;
  };
  // equilibrate the Robin rows (1 / max |G_kj|), in G and in P: the solve
  // applies B^{-1}(:, Robin rows) P = (D B)^{-1}(:, Robin rows) (D P)
  std::vector<cd> Pc(P.begin(), P.end());
  for (int kk = 0; kk < nr; ++kk) {
    double mx = 0.0;
    for (int j = 0; j < np; ++j) mx = std::max(mx, std::abs(G[(size_t)kk * np + j]));
    const double s = 1.0 / mx;
    for (int j = 0; j < np; ++j) G[(size_t)kk * np + j] *= s;
    for (int j = 0; j < nbq; ++j) Pc[(size_t)kk * nbq + j] *= s;
  }
  ItiConsts c;
  HPS_TRY(upload(&c.Gr, real_rep(G, nr, np)));
  HPS_TRY(upload(&c.Pr, real_rep(Pc, nr, nbq)));
  HPS_TRY(upload(&c.QHr, real_rep(QH, nbq, np)));
  std::vector<int> Iir(2 * o.Ii.size()), ident(2 * np);
  for (size_t a2 = 0; a2 < o.Ii.size(); ++a2) {
    Iir[2 * a2] = 2 * o.Ii[a2];
    Iir[2 * a2 + 1] = 2 * o.Ii[a2] + 1;
  }
  for (int i = 0; i < 2 * np; ++i) ident[i] = i;
  HPS_TRY(upload(&c.Ii, o.Ii));
  HPS_TRY(upload(&c.Iir, Iir));
  HPS_TRY(upload(&c.ident, ident));
  auto res = g_iti_cst.emplace(key, c);
  *out = &res.first->second;
  return HPS_OK;
}

}  // namespace
}  // namespace hps


namespace hps {
namespace {

void* op_alloc(hps_op* op, size_t bytes, bool resident = true) {
  Alloc rec{nullptr, bytes, nullptr, nullptr};
  void* p = op_dalloc(bytes, &rec);
  if (p) {
    rec.p = p;
    op->allocs.push_back(rec);
    if (resident) op->resident += round_size(bytes);
  }
  return p;
}

int add_gemm(hps_op* op, std::vector<GemmGroup> groups, GemmCall* call, bool ta = false, bool tb = false) {
  static const bool dump = std::getenv("HPS_PLAN_DUMP") != nullptr;  // diagnostic: the planned GEMM table
  if (dump) {
    std::fprintf(stderr, "gemm call %zu: %zu groups ta=%d tb=%d\n", op->hgroups.size(), groups.size(), (int)ta, (int)tb);
    for (const GemmGroup& g : groups)
      std::fprintf(stderr, "  M=%d N=%d K=%d batch=%d nseg=%d beta=%g\n", g.M, g.N, g.K, g.batch, g.nseg, g.beta);
  }
  call->first = (int)op->hgroups.size();
  call->count = (int)groups.size();
  op->split_elems = std::max(op->split_elems, gemm_plan_split(groups));
  call->nblocks = gemm_prepare(groups);
  call->nrblocks = gemm_rblocks(groups);
  call->ta = ta;
  call->tb = tb;
  op->hgroups.insert(op->hgroups.end(), groups.begin(), groups.end());
  return HPS_OK;
}

// Split a table of block ops into workgroup tasks of about kTaskElems elements
// (runtime-column ops count as 16 columns); long ops are cut by rows and
// columns, so no workgroup copies more than about kTaskElems elements.  Pieces
// of at most kWaveElems elements are collected in tasks of their own in which
// each wavefront takes every fourth piece: a whole workgroup walking a small
// block leaves most of its lanes idle.
// batch: the number of nodes the copy runs over (0: unknown).  Tasks hold up to
// 16K elements; a copy over few nodes gets smaller ones (down to 1K), so that
// a launch has about 1,024 workgroups where the work allows it
void add_copy(hps_op* op, const std::vector<BlockOp>& ops, CopyCall* call, long long batch = 0) {
  constexpr long long kWaveElems = 1024;
  constexpr int kRtCols = 16;
  long long kTaskElems = 16384;
  if (batch > 0) {
    long long total = 0;
    for (const BlockOp& o : ops) total += (long long)std::max(1, o.rows) * (o.cols <= 0 ? kRtCols : o.cols);
    kTaskElems = std::min<long long>(16384, std::max<long long>(kWaveElems, total * batch / 1024));
  }
  const int op0 = (int)op->hops.size();
  op->hops.insert(op->hops.end(), ops.begin(), ops.end());
  call->first_task = (int)op->htasks.size();
  struct Piece {
    CopyItem item;
    long long e;
  };
  std::vector<Piece> big, small;
  auto piece = [&](int opi, int r0, int r1, int c0, int c1, long long e) {
    (e <= kWaveElems ? small : big).push_back({{opi, r0, r1, c0, c1}, e});
  };
  for (size_t i = 0; i < ops.size(); ++i) {
    const BlockOp& o = ops[i];
    const int opi = op0 + (int)i;
    if (o.cols <= 0) {
      const int rchunk = (int)std::max<long long>(1, kTaskElems / kRtCols);
      for (int r0 = 0; r0 < o.rows; r0 += rchunk) {
        const int r1 = std::min(o.rows, r0 + rchunk);
        piece(opi, r0, r1, 0, -1, (long long)(r1 - r0) * kRtCols);
      }
      continue;
    }
    const int rchunk = (int)std::min<long long>(std::max(1, o.rows), kTaskElems);
    const int cchunk = (int)std::max<long long>(1, kTaskElems / rchunk);
    for (int r0 = 0; r0 < o.rows; r0 += rchunk) {
      const int r1 = std::min(o.rows, r0 + rchunk);
      for (int c0 = 0; c0 < o.cols; c0 += cchunk) {
        const int c1 = std::min(o.cols, c0 + cchunk);
        piece(opi, r0, r1, c0, c1, (long long)(r1 - r0) * (c1 - c0));
      }
    }
  }
  // runs of about kTaskElems elements: of big pieces for the whole workgroup,
  // of small pieces for the wavefronts in turn
  for (int per_wave = 0; per_wave < 2; ++per_wave) {
    const std::vector<Piece>& list = per_wave ? small : big;
    CopyTask cur{(int)op->hitems.size(), (int)op->hitems.size(), per_wave};
    long long load = 0;
    for (const Piece& pc : list) {
      if (load + pc.e > kTaskElems && cur.end > cur.begin) {
        op->htasks.push_back(cur);
        cur.begin = cur.end;
        load = 0;
      }
      op->hitems.push_back(pc.item);
      cur.end = (int)op->hitems.size();
      load += pc.e;
    }
    if (cur.end > cur.begin) op->htasks.push_back(cur);
  }
  call->ntasks = (int)op->htasks.size() - call->first_task;
}

GemmGroup make_group(const double* A, long long sA, int lda, const double* B, long long sB, int ldb, double* C,
                     long long sC, int ldc, int M, int N, int K, double alpha, double beta, long long batch,
                     const double* C0 = nullptr, long long sC0 = 0, int ldc0 = 0) {
  GemmGroup g;
  std::memset(&g, 0, sizeof(g));
  g.A = A; g.B = B; g.C = C; g.C0 = C0;
  g.sA = sA; g.sB = sB; g.sC = sC; g.sC0 = sC0;
  g.lda = lda; g.ldb = ldb; g.ldc = ldc; g.ldc0 = ldc0 ? ldc0 : ldc;
  g.M = M; g.N = N; g.K = K; g.nseg = 1;
  g.alpha = alpha; g.beta = beta;
  g.batch = (int)batch;
  return g;
}

BlockOp make_op(long long dst_off, int dst_ld, int rows, int cols) {
  BlockOp o;
  std::memset(&o, 0, sizeof(o));
  o.dst_off = dst_off;
  o.dst_ld = dst_ld;
  o.rows = rows;
  o.cols = cols;
  return o;
}

void op_src(BlockOp& o, int buf, long long off, int ld) {
  o.src_buf[o.nsrc] = buf;
  o.src_off[o.nsrc] = off;
  o.src_ld[o.nsrc] = ld;
  o.nsrc++;
}

int run_gemm(hps_op* op, const GemmCall& c, hipStream_t st, int n_override = 0) {
  return gemm_launch(op->dgroups + c.first, c.count, c.nblocks, c.nrblocks, c.ta, c.tb, st, n_override);
}

int run_copy(hps_op* op, const CopyCall& c, int ncols_rt, double* dst, long long dst_stride, const double* s0,
             long long s0_stride, const double* s1, long long s1_stride, long long batch, hipStream_t st) {
  return block_copy_launch(op->dops, op->ditems, op->dtasks + c.first_task, c.ntasks, ncols_rt, dst, dst_stride, s0,
                           s0_stride, s1, s1_stride, batch, st);
}

void stage_begin(hps_op* op, const char* name, hipStream_t st) {
  if (!(op->flags & HPS_FLAG_TIMING)) return;
  // timing is diagnostic: a stage whose events cannot be created is skipped
  TimedStage t;
  t.name = name;
  if (hipEventCreate(&t.a) != hipSuccess) return;
  if (hipEventCreate(&t.b) != hipSuccess) {
    (void)hipEventDestroy(t.a);
    return;
  }
  (void)hipEventRecord(t.a, st);
  op->stages.push_back(t);
}
void stage_end(hps_op* op, hipStream_t st) {
  if (!(op->flags & HPS_FLAG_TIMING) || op->stages.empty()) return;
  (void)hipEventRecord(op->stages.back().b, st);
}
void clear_stages(hps_op* op) {
  for (auto& s : op->stages) {
    (void)hipEventDestroy(s.a);
    (void)hipEventDestroy(s.b);
  }
  op->stages.clear();
}

// ---------------------------------------------------------------------------
// batched Gauss-Jordan inversion: register form for m <= 112 (and up to 224
// for batches that fill the GPU), blocked above
// ---------------------------------------------------------------------------
constexpr int kGjSmallAlways = 112;

long long al256(long long bytes) { return (bytes + 255) / 256 * 256; }

// the next piece of the merge-level build workspace (reset per level)
void* lvl_take(hps_op* op, long long bytes) {
  const long long b = al256(bytes);
  if (!op->lvl_ws || op->lvl_cur + b > op->lvl_ws_bytes) {
    set_error("merge-level build workspace exhausted (internal sizing error)");
    return nullptr;
  }
  void* p = op->lvl_ws + op->lvl_cur;
  op->lvl_cur += b;
  return p;
}

bool gj_is_small(int m, long long batch) { return m <= kGjSmallAlways || (m <= gj_small_max() && batch >= 256); }

// The two-level form (column blocks of kGjBlockCols) where the one-level
// form's per-panel update of every column is bound by HBM traffic: large
// matrices, and batches whose matrices together exceed ~1.2 GB (the leaves of
// 3D p = 12 and ItI p = 16 operators)
constexpr int kGjBlockCols = 256;
bool gj_two_level(int m, long long batch) {
  return m >= 2049 || (m >= 2 * kGjBlockCols && (double)batch * m * m >= 1.5e8);
}

// bytes plan_gj takes from the level workspace for a blocked inverse
long long gj_ws_bytes(int m, long long batch) {
  if (gj_is_small(m, batch)) return 0;
  long long b = 2 * al256((long long)sizeof(int) * batch * m) +
                al256((long long)sizeof(double) * 2 * batch * m * gj_panel_max_nb());
  if (gj_two_level(m, batch)) b += 2 * al256((long long)sizeof(double) * batch * m * kGjBlockCols);
  return b;
}

// level_ws: workspace from the shared merge-level region (else owned by op)
int plan_gj(hps_op* op, GJPlan* g, double* A, double* Z, int m, long long batch, bool level_ws = false) {
  g->m = m;
  g->batch = batch;
  g->A = A;
  g->Z = Z;
  g->flag = op->flag;
  // the single-workgroup kernel (one CU per matrix) up to kGjSmallAlways, and
  // up to its limit when the batch alone fills the GPU; otherwise the blocked
  // form, whose column updates run on many CUs beside the panel
  g->small = gj_is_small(m, batch);
  if (g->small) return HPS_OK;
  g->nb = gj_panel_width(m);
  if (g->nb == 0) {
    set_error("matrix of size " + std::to_string(m) + " exceeds the blocked Gauss-Jordan limit (16384)");
    return HPS_EUNSUPPORTED;
  }
  const int mnb = gj_panel_max_nb();
  auto take = [&](long long bytes) { return level_ws ? lvl_take(op, bytes) : op_alloc(op, (size_t)bytes, false); };
  g->pos = (int*)take((long long)sizeof(int) * batch * m);
  g->piv = (int*)take((long long)sizeof(int) * batch * m);
  g->W = (double*)take((long long)sizeof(double) * 2 * batch * m * mnb);  // two buffers, by panel parity
  if (!g->pos || !g->piv || !g->W) {
    set_error("device allocation failed (Gauss-Jordan workspace)");
    return HPS_ENOMEM;
  }
  if (gj_two_level(m, batch)) {
    // per column block [b0, b0 + w): A(:, j) += Wk Pk(:, j) for the columns
    // left and right of the block (in place: C0 = C)
    const int ob = kGjBlockCols;
    g->ob = ob;
    g->Wk = (double*)take((long long)sizeof(double) * batch * m * ob);
    g->Pk = (double*)take((long long)sizeof(double) * batch * m * ob);
    if (!g->Wk || !g->Pk) {
      set_error("device allocation failed (Gauss-Jordan block workspace)");
      return HPS_ENOMEM;
    }
    const long long mm = (long long)m * m, mo = (long long)m * ob;
    for (int b0 = 0; b0 < m; b0 += ob) {
      const int w = std::min(ob, m - b0), r0 = b0 + w;
      std::vector<GemmGroup> gs;
      if (b0 > 0)
        gs.push_back(make_group(g->Wk, mo, m, g->Pk, mo, ob, A, mm, m, m, b0, w, 1.0, 1.0, batch, A, mm, m));
      if (r0 < m)
        gs.push_back(make_group(g->Wk, mo, m, g->Pk + (long long)r0 * ob, mo, ob, A + (long long)r0 * m, mm, m, m,
                                m - r0, w, 1.0, 1.0, batch, A + (long long)r0 * m, mm, m));
      GemmCall call;
      add_gemm(op, gs, &call);
      g->blk.push_back(call);
    }
  }
  return HPS_OK;
}

int run_gj(hps_op* op, const GJPlan& g, hipStream_t st) {
  if (g.small) return gj_small_launch(g.A, g.Z, g.m, g.flag, g.batch, st);
  HPS_TRY(gj_init_launch(g.pos, g.batch * g.m, st));
  if (g.ob > 0) {
    // two-level form: inside each column block the panels update only the
    // block (the pivot search still runs over every unused row); then the
    // block's combined elimination operator updates the other columns on the
    // matrix cores
    const long long wbuf = g.batch * g.m * gj_panel_max_nb();
    int K = 0;
    for (int b0 = 0; b0 < g.m; b0 += g.ob, ++K) {
      const int w = std::min(g.ob, g.m - b0);
      const int np = (w + g.nb - 1) / g.nb;
      HPS_TRY(gj_panel_launch(g.A, g.m, b0, std::min(g.nb, w), g.pos, g.piv, g.W, g.flag, g.batch, st));
      for (int k = 1; k < np; ++k) {
        const int j0 = b0 + k * g.nb, wk = std::min(g.nb, b0 + w - j0);
        HPS_TRY(gj_step_launch(g.A, g.m, j0, wk, g.pos, g.piv, g.W + (k % 2) * wbuf, g.W + ((k - 1) % 2) * wbuf,
                               g.nb, g.flag, g.batch, st, b0, w));
      }
      const int jl = b0 + (np - 1) * g.nb;
      HPS_TRY(gj_update_launch(g.A, g.W + ((np - 1) % 2) * wbuf, g.piv, g.m, jl, b0 + w - jl, g.batch, st, b0, w));
      HPS_TRY(gj_block_prep_launch(g.A, g.piv, g.m, b0, w, g.ob, g.Wk, g.Pk, g.batch, st));
      HPS_TRY(run_gemm(op, g.blk[K], st));
    }
    return gj_unscramble_launch(g.A, g.Z, g.m, g.pos, g.piv, g.batch, st);
  }
  // panel k writes W buffer k % 2; launch k (k >= 1) factors panel k beside
  // the update by panel k - 1 of the columns outside both panels
  const long long wbuf = g.batch * g.m * gj_panel_max_nb();
  const int np = (g.m + g.nb - 1) / g.nb;
  HPS_TRY(gj_panel_launch(g.A, g.m, 0, std::min(g.nb, g.m), g.pos, g.piv, g.W, g.flag, g.batch, st));
  for (int k = 1; k < np; ++k) {
    const int j0 = k * g.nb, w = std::min(g.nb, g.m - j0);
    HPS_TRY(gj_step_launch(g.A, g.m, j0, w, g.pos, g.piv, g.W + (k % 2) * wbuf, g.W + ((k - 1) % 2) * wbuf, g.nb,
                           g.flag, g.batch, st, 0, 0));
  }
  const int jl = (np - 1) * g.nb;
  HPS_TRY(gj_update_launch(g.A, g.W + ((np - 1) % 2) * wbuf, g.piv, g.m, jl, g.m - jl, g.batch, st, 0, 0));
  return gj_unscramble_launch(g.A, g.Z, g.m, g.pos, g.piv, g.batch, st);
}

// Block inversion of the merge matrix D (m = 2s + r) with interfaces ordered
// [P1 | P2 | R], D(P1, P2) = D(P2, P1) = 0:
//   A_b^{-1} = D(P_b, P_b)^{-1}                    (batched Gauss-Jordan, 2 per node)
//   X_b = A_b^{-1} D(P_b, R),  Y_b = D(R, P_b) A_b^{-1}
//   Sc  = D(R, R) - sum_b D(R, P_b) X_b,  Sc^{-1}  (Gauss-Jordan)
//   Z(R, R) = Sc^{-1},  Z(P_b, R) = -X_b Sc^{-1},  Z(R, P_b) = -Sc^{-1} Y_b,
//   Z(P_b, P_b') = delta_bb' A_b^{-1} - Z(P_b, R) Y_b'
// It is exact block elimination of D in an order that skips D's zero
// blocks; pivoting happens inside A_b and Sc.
int plan_schur(hps_op* op, LevelPlan& P, int schur_p) {
  const int n = P.n, m = P.m;
  const long long nm = P.nm, mm = (long long)m * m;
  const int s = schur_p * n, r = m - 2 * s;
  P.schur = true;
  P.sP = s;
  P.sR = r;
  P.Ablk = (double*)lvl_take(op, sizeof(double) * nm * 2 * s * s);
  P.Ainv = (double*)lvl_take(op, sizeof(double) * nm * 2 * s * s);
  P.Xs = (double*)lvl_take(op, sizeof(double) * nm * 2 * s * r);
  P.Ys = (double*)lvl_take(op, sizeof(double) * nm * 2 * r * s);
  P.Sc = (double*)lvl_take(op, sizeof(double) * nm * r * r);
  P.Scinv = (double*)lvl_take(op, sizeof(double) * nm * r * r);
  if (!P.Ablk || !P.Ainv || !P.Xs || !P.Ys || !P.Sc || !P.Scinv) return HPS_ENOMEM;
  HPS_TRY(plan_gj(op, &P.gjA, P.Ablk, P.Ainv, s, 2 * nm, true));
  HPS_TRY(plan_gj(op, &P.gjS, P.Sc, P.Scinv, r, nm, true));
  // a zero pivot inside a block is not a singular D: it goes to its own flag
  // slot, and the checked build then falls back to pivoting over all of D
  P.gjA.flag = P.gjS.flag = op->flag + 1;
  const long long s2 = 2LL * s * s, sr2 = 2LL * s * r, r2 = (long long)r * r;
  {  // A_b = D(P_b, P_b)
    std::vector<BlockOp> ops;
    for (int b = 0; b < 2; ++b) {
      BlockOp o = make_op((long long)b * s * s, s, s, s);
      op_src(o, 0, (long long)b * s + (long long)b * s * m, m);
      ops.push_back(o);
    }
    add_copy(op, ops, &P.copyA, P.nm);
  }
  {  // X_b = A_b^{-1} D(P_b, R);  Y_b = D(R, P_b) A_b^{-1}
    std::vector<GemmGroup> gs;
    for (int b = 0; b < 2; ++b) {
      gs.push_back(make_group(P.Ainv + (long long)b * s * s, s2, s, P.Dbuf + (long long)b * s + 2LL * s * m, mm, m,
                              P.Xs + (long long)b * s * r, sr2, s, s, r, s, 1.0, 0.0, nm));
      gs.push_back(make_group(P.Dbuf + 2LL * s + (long long)b * s * m, mm, m, P.Ainv + (long long)b * s * s, s2, s,
                              P.Ys + (long long)b * r * s, sr2, r, r, s, s, 1.0, 0.0, nm));
    }
    add_gemm(op, gs, &P.gemmXY);
  }
  {  // Sc = D(R, R) - sum_b D(R, P_b) X_b
    GemmGroup g = make_group(P.Dbuf + 2LL * s, mm, m, P.Xs, sr2, s, P.Sc, r2, r, r, r, s, -1.0, 1.0, nm,
                             P.Dbuf + 2LL * s + 2LL * s * m, mm, m);
    g.nseg = 2;
    for (int b = 0; b < 2; ++b) {
      g.aseg[b] = (long long)b * s * m;
      g.bseg[b] = (long long)b * s * r;
    }
    add_gemm(op, {g}, &P.gemmSc);
  }
  {  // Z(P_b, R) = -X_b Sc^{-1};  Z(R, P_b) = -Sc^{-1} Y_b
    std::vector<GemmGroup> gs;
    for (int b = 0; b < 2; ++b) {
      gs.push_back(make_group(P.Xs + (long long)b * s * r, sr2, s, P.Scinv, r2, r,
                              P.Z + (long long)b * s + 2LL * s * m, mm, m, s, r, r, -1.0, 0.0, nm));
      gs.push_back(make_group(P.Scinv, r2, r, P.Ys + (long long)b * r * s, sr2, r,
                              P.Z + 2LL * s + (long long)b * s * m, mm, m, r, s, r, -1.0, 0.0, nm));
    }
    add_gemm(op, gs, &P.gemmZ1);
  }
  {  // Z(R, R) = Sc^{-1}
    BlockOp o = make_op(2LL * s + 2LL * s * m, m, r, r);
    op_src(o, 0, 0, r);
    add_copy(op, {o}, &P.copyScZ, P.nm);
  }
  {  // Z(P_b, P_b') = delta_bb' A_b^{-1} - Z(P_b, R) Y_b'
    std::vector<GemmGroup> gs;
    for (int b = 0; b < 2; ++b)
      for (int c = 0; c < 2; ++c) {
        GemmGroup g = make_group(P.Z + (long long)b * s + 2LL * s * m, mm, m, P.Ys + (long long)c * r * s, sr2, r,
                                 P.Z + (long long)b * s + (long long)c * s * m, mm, m, s, s, r, -1.0,
                                 b == c ? 1.0 : 0.0, nm, b == c ? P.Ainv + (long long)b * s * s : nullptr,
                                 b == c ? s2 : 0, b == c ? s : 0);
        gs.push_back(g);
      }
    add_gemm(op, gs, &P.gemmZPP);
  }
  return HPS_OK;
}

int run_schur(hps_op* op, LevelPlan& P, hipStream_t st) {
  const long long mm = (long long)P.m * P.m, s2 = 2LL * P.sP * P.sP, r2 = (long long)P.sR * P.sR;
  HPS_TRY(run_copy(op, P.copyA, 0, P.Ablk, s2, P.Dbuf, mm, nullptr, 0, P.nm, st));
  HPS_TRY(run_gj(op, P.gjA, st));
  HPS_TRY(run_gemm(op, P.gemmXY, st));
  HPS_TRY(run_gemm(op, P.gemmSc, st));
  HPS_TRY(run_gj(op, P.gjS, st));
  HPS_TRY(run_gemm(op, P.gemmZ1, st));
  HPS_TRY(run_copy(op, P.copyScZ, 0, P.Z, mm, P.Scinv, r2, nullptr, 0, P.nm, st));
  HPS_TRY(run_gemm(op, P.gemmZPP, st));
  return HPS_OK;
}

// ---------------------------------------------------------------------------
// accuracy guard of the merge inverses: probe residual per node, gated
// Newton-Schulz steps on the block-eliminated levels
// ---------------------------------------------------------------------------
constexpr int kProbes = 4;           // probe vectors per merge inverse
constexpr int kNsSteps = 2;          // Newton-Schulz steps at most
constexpr double kNsRefine = 1e-12;  // refine a node whose probe residual is above this
constexpr double kNsAccept = 1e-10;  // above this after refinement: pivot over all of D instead

int plan_guard(hps_op* op, LevelPlan& P) {
  const int m = P.m;
  const long long nm = P.nm, mm = (long long)m * m;
  const long long mp = (long long)m * kProbes;
  const int ldx = op->probe_ld;
  P.py = (double*)lvl_take(op, sizeof(double) * nm * mp);
  P.pr = (double*)lvl_take(op, sizeof(double) * nm * mp);
  if (op->rho_used + (kNsSteps + 1) * nm > op->rho_n) {
    set_error("internal: probe residual block too small");
    return HPS_EINVAL;
  }
  P.rho = op->rho_all + op->rho_used;
  op->rho_used += (kNsSteps + 1) * nm;
  P.gate = (int*)op_alloc(op, sizeof(int) * nm, false);
  if (!P.py || !P.pr || !P.rho || !P.gate) {
    set_error("device allocation failed (merge inverse probe)");
    return HPS_ENOMEM;
  }
  // block-eliminated: y = Z x, r = D y - x;  whole-D: y = D x (before the
  // inversion), r = Z y - x
  const double* first = P.schur ? P.Z : P.Dbuf;
  const double* second = P.schur ? P.Dbuf : P.Z;
  add_gemm(op, {make_group(first, mm, m, op->probe_x, 0, ldx, P.py, mp, m, m, kProbes, m, 1.0, 0.0, nm)},
           &P.probe1);
  add_gemm(op, {make_group(second, mm, m, P.py, mp, m, P.pr, mp, m, m, kProbes, m, 1.0, -1.0, nm, op->probe_x, 0,
                           ldx)},
           &P.probe2);
  if (!P.schur) return HPS_OK;
  P.Wns = (double*)lvl_take(op, sizeof(double) * nm * mm);
  P.Zns = (double*)lvl_take(op, sizeof(double) * nm * mm);
  if (!P.Wns || !P.Zns) {
    set_error("device allocation failed (Newton-Schulz workspace)");
    return HPS_ENOMEM;
  }
  // W = D Z;  Zns = 2 Z - Z W   (I - D Zns = (I - D Z)^2)
  GemmGroup w = make_group(P.Dbuf, mm, m, P.Z, mm, m, P.Wns, mm, m, m, m, m, 1.0, 0.0, nm);
  w.gate = P.gate;
  add_gemm(op, {w}, &P.nsW);
  GemmGroup z = make_group(P.Z, mm, m, P.Wns, mm, m, P.Zns, mm, m, m, m, m, -1.0, 2.0, nm, P.Z, mm, m);
  z.gate = P.gate;
  add_gemm(op, {z}, &P.nsZ);
  return HPS_OK;
}

// bytes one merge level takes from the level workspace (the pieces of
// plan_op, plan_schur, plan_gj and plan_guard above, in any order)
long long level_ws_bytes(int m, int n, long long nm, bool schur, int schur_p) {
  const long long mm = (long long)m * m, d8 = sizeof(double);
  long long b = al256(d8 * nm * mm) + 2 * al256(d8 * nm * m * kProbes);  // D, probe products
  if (schur) {
    const long long s = (long long)schur_p * n, r = m - 2 * s;
    b += 2 * al256(d8 * nm * 2 * s * s) + 2 * al256(d8 * nm * 2 * s * r) + 2 * al256(d8 * nm * r * r);
    b += gj_ws_bytes((int)s, 2 * nm) + gj_ws_bytes((int)r, nm);
    b += 2 * al256(d8 * nm * mm);  // Newton-Schulz
  } else {
    b += gj_ws_bytes(m, nm);
  }
  return b;
}

// the probe after the inversion (k = 0) or after Newton-Schulz step k
int run_probe(hps_op* op, LevelPlan& P, int k, hipStream_t st) {
  if (P.schur) HPS_TRY(run_gemm(op, P.probe1, st, kProbes));
  HPS_TRY(run_gemm(op, P.probe2, st, kProbes));
  return probe_reduce_launch(P.pr, (long long)P.m * kProbes, P.m * kProbes, op->probe_inv_xmax, kNsRefine,
                             P.rho + k * P.nm, P.gate, P.nm, st);
}

int run_refine(hps_op* op, LevelPlan& P, hipStream_t st) {
  for (int k = 1; k <= kNsSteps; ++k) {
    HPS_TRY(run_gemm(op, P.nsW, st));
    HPS_TRY(run_gemm(op, P.nsZ, st));
    HPS_TRY(gated_copy_launch(P.Z, P.Zns, (long long)P.m * P.m, P.gate, P.nm, st));
    HPS_TRY(run_probe(op, P, k, st));
  }
  return HPS_OK;
}

// ---------------------------------------------------------------------------
// the allocation-free solve: the solve's GEMM descriptors with every pointer
// into the solve workspace moved to the same offset in the device's static
// workspace, and split-K partial products placed after it.  Copies take
// their buffers at launch time and need no second table.
// ---------------------------------------------------------------------------
std::vector<const GemmCall*> solve_gemm_calls(hps_op* op) {
  std::vector<const GemmCall*> calls;
  if (op->d == 3) calls.push_back(&op->gemmVleaf);
  calls.push_back(&op->gemmHleaf);
  for (auto& P : op->levels) {
    calls.push_back(&P.gemmGt);
    calls.push_back(&P.gemmHp);
    calls.push_back(&P.gemmDown);
  }
  return calls;
}

int plan_static_solve(hps_op* op) {
  op->static_ok = false;
  if (op->ext_side > 0 || op->root_h || op->iti || op->ad) return HPS_OK;  // subtree parts, ItI, adaptive: not offered
  void* base = nullptr;
  HPS_TRY(static_ws_ptr(&base));
  op->static_base = (char*)base;
  // split-K parts of the solve's calls, packed after the workspace copy
  long long part_elems = 0;
  for (const GemmCall* c : solve_gemm_calls(op))
    for (int i = 0; i < c->count; ++i) {
      const GemmGroup& g = op->hgroups[c->first + i];
      if (g.ksplit > 1)
        part_elems = std::max(part_elems, g.part_off + (long long)g.batch * g.ksplit * g.M * g.N);
    }
  op->static_need = op->ws_bytes + part_elems * (long long)sizeof(double);
  if (op->static_need > (long long)HPS_STATIC_WS_BYTES) return HPS_OK;  // too large: the entry point says so
  op->hgroups_static = op->hgroups;
  auto mv = [op](const double* p) -> double* {
    const char* c = (const char*)p;
    if (c >= op->ws_base && c < op->ws_base + op->ws_bytes) return (double*)(op->static_base + (c - op->ws_base));
    return (double*)p;
  };
  double* part0 = (double*)(op->static_base + op->ws_bytes);
  for (const GemmCall* c : solve_gemm_calls(op))
    for (int i = 0; i < c->count; ++i) {
      GemmGroup& g = op->hgroups_static[c->first + i];
      g.A = mv(g.A);
      g.B = mv(g.B);
      g.C = mv(g.C);
      if (g.C0) g.C0 = mv(g.C0);
      g.part = g.ksplit > 1 ? part0 + g.part_off : nullptr;
    }
  op->static_ok = true;
  return HPS_OK;
}

// Buffers and descriptor table one solve runs on: the operator's own
// workspace, or (allocation-free solve) the static workspace.
struct SolveCtx {
  const hps_op* op;
  const GemmGroup* groups;
  const char* base;  // where the solve workspace starts
  double* at(double* p) const {
    return base == op->ws_base ? p : (double*)(base + ((const char*)p - op->ws_base));
  }
};

SolveCtx own_ctx(hps_op* op) { return {op, op->dgroups, op->ws_base}; }

int run_gemm_ctx(const SolveCtx& c, const GemmCall& call, hipStream_t st, int n_override) {
  return gemm_launch(c.groups + call.first, call.count, call.nblocks, call.nrblocks, call.ta, call.tb, st, n_override);
}

// ---------------------------------------------------------------------------
// plan: allocations + every descriptor table
// ---------------------------------------------------------------------------
int finish_plan(hps_op* op);

int plan_op(hps_op* op) {
  const int d = op->d, L = op->tree.depth, nd = op->nd;
  const MergeGeom& G = merge_geom(d);
  const int ni = op->ni, nb = op->nb, NR = op->NR;
  const long long nl = op->nl;
  const bool ext = op->ext_side > 0;  // leaves are subtree roots (their T arrive from outside)
  // leaf storage
  if (!ext) {
    op->LU = (double*)op_alloc(op, sizeof(double) * nl * ni * ni);
    op->Y = (double*)op_alloc(op, sizeof(double) * nl * ni * nb);
    op->perm = (int*)op_alloc(op, sizeof(int) * nl * ni);
    op->pos = (int*)op_alloc(op, sizeof(int) * nl * ni);
  }
  if (d == 3) {
    op->Lbuf = (double*)op_alloc(op, sizeof(double) * nl * ni * ni, false);
    op->Rbuf = (double*)op_alloc(op, sizeof(double) * nl * ni * nb, false);
    if (!op->Lbuf || !op->Rbuf) { set_error("device allocation failed (3D leaf workspace)"); return HPS_ENOMEM; }
    HPS_TRY(plan_gj(op, &op->leaf_gj, op->Lbuf, op->LU, ni, nl));
    // Y_int = -L_ii^{-1} (L_ie P);  v = L_ii^{-1} f_int
    add_gemm(op, {make_group(op->LU, (long long)ni * ni, ni, op->Rbuf, (long long)ni * nb, ni, op->Y,
                             (long long)ni * nb, ni, ni, nb, ni, -1.0, 0.0, nl)},
             &op->gemmYleaf);
  }
  // T of the leaves (Tbuf[0]) and of the levels below the root: level lev
  // writes Tbuf[(L - lev) % 2] while its children's T sit in the other one
  {
    const long long side0 = ext ? op->ext_side : (d == 2 ? op->p - 2 : (long long)(op->p - 2) * (op->p - 2));
    long long tb[2] = {nl * nb * nb, 0};
    for (int lev = 1; lev < L; ++lev) {
      const long long nbp = 2LL * d * (side0 << ((d - 1) * (L - lev)));
      tb[(L - lev) % 2] = std::max(tb[(L - lev) % 2], (1LL << (d * lev)) * nbp * nbp);
    }
    for (int k = 0; k < 2; ++k)
      if (tb[k] > 0) {
        op->Tbuf[k] = (double*)op_alloc(op, sizeof(double) * tb[k], false);
        if (!op->Tbuf[k]) { set_error("device allocation failed (T workspace)"); return HPS_ENOMEM; }
      }
  }
  op->Tleaf = op->Tbuf[0];
  // status block: flags (padded to 8 doubles), then the probe residuals of
  // every merge level (kNsSteps + 1 per node)
  op->rho_n = 0;
  op->rho_used = 0;
  for (int lev = 0; lev < L; ++lev) op->rho_n += (kNsSteps + 1) * (1LL << (d * lev));
  op->flag = (int*)op_alloc(op, sizeof(double) * (8 + op->rho_n), false);
  op->rho_all = op->flag ? (double*)op->flag + 8 : nullptr;
  if ((!ext && (!op->LU || !op->Y || !op->perm || !op->pos)) || !op->Tleaf || !op->flag) {
    set_error("device allocation failed (leaf operators)");
    return HPS_ENOMEM;
  }
  // solve workspace, one contiguous block (so that the allocation-free solve
  // can run the same plans on a copy of it at another address): per tree
  // level g, h [nodes][NR][nbl]; leaf v [nl][NR][ni]; per merge level
  // hint, gt, gint [nm][NR][m]
  op->g.assign(L + 1, nullptr);
  op->h.assign(L + 1, nullptr);
  op->nbl.assign(L + 1, 0);
  for (int l = 0; l <= L; ++l) {
    const long long base = ext ? op->ext_side : (d == 2 ? op->p - 2 : (long long)(op->p - 2) * (op->p - 2));
    const long long side = base << ((d - 1) * (L - l));
    op->nbl[l] = (int)(2 * d * side);
  }
  {
    auto al = [](long long elems) { return (elems * (long long)sizeof(double) + 255) / 256 * 256; };
    long long bytes = 0;
    for (int l = 0; l <= L; ++l) bytes += 2 * al((1LL << (d * l)) * NR * op->nbl[l]);
    bytes += (d == 3 ? 2 : 1) * al(nl * NR * ni);  // v (and the gathered interior sources in 3D)
    for (int lev = 0; lev < L; ++lev) {
      const long long nm = 1LL << (d * lev), m = (long long)G.nint * (op->nbl[lev + 1] / (2 * d));
      bytes += 3 * al(nm * NR * m);
    }
    op->ws_base = (char*)op_alloc(op, (size_t)bytes, false);
    if (!op->ws_base) { set_error("device allocation failed (solve workspace)"); return HPS_ENOMEM; }
    op->ws_bytes = bytes;
    long long cur = 0;
    op->ws_take = [op, cur, al](long long elems) mutable {
      double* p = (double*)(op->ws_base + cur);
      cur += al(elems);
      return p;
    };
  }
  for (int l = 0; l <= L; ++l) {
    const long long nodes = 1LL << (d * l);
    op->g[l] = op->ws_take(nodes * NR * op->nbl[l]);
    op->h[l] = op->ws_take(nodes * NR * op->nbl[l]);
  }
  op->v = op->ws_take(nl * NR * ni);
  if (d == 3) op->fint = op->ws_take(nl * NR * ni);
  if (d == 3)
    add_gemm(op, {make_group(op->LU, (long long)ni * ni, ni, op->fint, (long long)NR * ni, ni, op->v, (long long)NR * ni,
                             ni, ni, NR, ni, 1.0, 0.0, nl)},
             &op->gemmVleaf);
  // adjoint leaf products
  if (!ext) {
    const int ne = op->ne;
    if (d == 2) {
      op->fint = (double*)op_alloc(op, sizeof(double) * nl * NR * ni, false);
      if (!op->fint) { set_error("device allocation failed (adjoint workspace)"); return HPS_ENOMEM; }
    }
    op->wext = (double*)op_alloc(op, sizeof(double) * nl * NR * ne, false);
    if (!op->wext) { set_error("device allocation failed (adjoint workspace)"); return HPS_ENOMEM; }
    // g_leaf = Y^T w_int,  += P^T w_ext
    add_gemm(op, {make_group(op->Y, (long long)ni * nb, ni, op->v, (long long)NR * ni, ni, op->g[L], (long long)NR * nb,
                             nb, nb, NR, ni, 1.0, 0.0, nl)},
             &op->adjYt, true, false);
    add_gemm(op, {make_group(op->cst->P, 0, ne, op->wext, (long long)NR * ne, ne, op->g[L], (long long)NR * nb, nb, nb,
                             NR, ne, 1.0, 1.0, nl, op->g[L], (long long)NR * nb, nb)},
             &op->adjPt, true, false);
    // v += Q_i^T h_leaf
    add_gemm(op, {make_group(op->cst->Qi, 0, nb, op->h[L], (long long)NR * nb, nb, op->v, (long long)NR * ni, ni, ni, NR,
                             nb, 1.0, 1.0, nl, op->v, (long long)NR * ni, ni)},
             &op->adjQt, true, false);
    if (d == 3)  // f = L_ii^{-T} v
      add_gemm(op, {make_group(op->LU, (long long)ni * ni, ni, op->v, (long long)NR * ni, ni, op->fint,
                               (long long)NR * ni, ni, ni, NR, ni, 1.0, 0.0, nl)},
               &op->adjLinvT, true, false);
  }

  if (!ext) {
    // leaf T = Q_e P + Q_i Y_int
    add_gemm(op, {make_group(op->cst->Qi, 0, nb, op->Y, (long long)ni * nb, ni, op->Tleaf, (long long)nb * nb, nb, nb,
                             nb, ni, 1.0, 1.0, nl, op->cst->QeP, 0, nb)},
             &op->gemmTleaf);
    // h = Q_i v (solve)
    add_gemm(op, {make_group(op->cst->Qi, 0, nb, op->v, (long long)NR * ni, ni, op->h[L], (long long)NR * nb, nb, nb,
                             NR, ni, 1.0, 0.0, nl)},
             &op->gemmHleaf);
  }
  // root data: bdry -> g[0]
  {
    BlockOp o = make_op(0, op->nbl[0], op->nbl[0], 0);
    op_src(o, 0, 0, op->nbl[0]);
    add_copy(op, {o}, &op->copyRoot);
  }

  // probe vectors of the merge-inverse guard: fixed pseudo-random values in
  // [-1, 1) (splitmix64 of the element index)
  {
    long long mmax = 1;
    const long long n0 = op->nbl[L] / (2 * d);  // Gauss points per leaf face
    for (int lev = L - 1; lev >= 0; --lev) mmax = std::max<long long>(mmax, G.nint * (n0 << ((d - 1) * (L - 1 - lev))));
    op->probe_ld = (int)mmax;
    std::vector<double> x((size_t)mmax * kProbes);
    double xmax = 0.0;
    for (size_t i = 0; i < x.size(); ++i) {
      uint64_t z = (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ULL;
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
      z ^= z >> 31;
      x[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
      xmax = std::max(xmax, std::fabs(x[i]));
    }
    op->probe_x = (double*)op_alloc(op, sizeof(double) * x.size(), false);
    if (!op->probe_x) { set_error("device allocation failed (probe vector)"); return HPS_ENOMEM; }
    HPS_HIP_TRY(hipMemcpy(op->probe_x, x.data(), sizeof(double) * x.size(), hipMemcpyHostToDevice));
    op->probe_inv_xmax = 1.0 / xmax;
  }
  // the merge-level build workspace, sized for the largest level
  {
    long long need = 0;
    for (int lev = 0; lev < L; ++lev) {
      const int n = op->nbl[lev + 1] / (2 * d), m = G.nint * n;
      const bool schur = m > kGjSmallAlways && !(op->flags & HPS_FLAG_FULL_PIVOT);
      need = std::max(need, level_ws_bytes(m, n, 1LL << (d * lev), schur, G.schur_p));
    }
    op->lvl_ws = (char*)op_alloc(op, (size_t)need, false);
    if (!op->lvl_ws) { set_error("device allocation failed (merge-level build workspace)"); return HPS_ENOMEM; }
    op->lvl_ws_bytes = need;
  }
  op->levels.assign(L, LevelPlan());
  for (int lev = L - 1; lev >= 0; --lev) {
    LevelPlan& P = op->levels[lev];
    op->lvl_cur = 0;
    P.lev = lev;
    P.nm = 1LL << (d * lev);
    P.nbc = op->nbl[lev + 1];
    P.nbp = op->nbl[lev];
    P.n = P.nbc / (2 * d);
    P.m = G.nint * P.n;
    P.dn = d * P.n;
    const int n = P.n, m = P.m, nbc = P.nbc, nbp = P.nbp, dn = P.dn;
    const long long nm = P.nm;
    const long long childT = (long long)nbc * nbc;  // per child
    const double* Tchild = lev == L - 1 ? op->Tleaf : op->levels[lev + 1].Tp;
    P.Z = (double*)op_alloc(op, sizeof(double) * nm * m * m);
    P.S = (double*)op_alloc(op, sizeof(double) * nm * m * nbp);
    P.Bnz = (double*)op_alloc(op, sizeof(double) * nm * nd * dn * dn);
    P.Dbuf = (double*)lvl_take(op, sizeof(double) * nm * m * m);
    const bool formT = lev > 0 || (op->flags & HPS_FLAG_ROOT_T);
    if (formT) P.Tp = lev == 0 ? (double*)op_alloc(op, sizeof(double) * nm * nbp * nbp) : op->Tbuf[(L - lev) % 2];
    P.hint = op->ws_take(nm * NR * m);
    P.gt = op->ws_take(nm * NR * m);
    P.gint = op->ws_take(nm * NR * m);
    if (!P.Z || !P.S || !P.Bnz || !P.Dbuf || (formT && !P.Tp)) {
      set_error("device allocation failed (merge level)");
      return HPS_ENOMEM;
    }
    if (m > kGjSmallAlways && !(op->flags & HPS_FLAG_FULL_PIVOT)) {
      // block elimination over the interface pieces (measured faster from here on)
      HPS_TRY(plan_schur(op, P, G.schur_p));
    } else {
      HPS_TRY(plan_gj(op, &P.gj, P.Dbuf, P.Z, m, nm, true));
    }
    HPS_TRY(plan_guard(op, P));
    // --- D = sum over children touching interfaces i and j of T_c(face_i, face_j)
    {
      std::vector<BlockOp> ops;
      for (int i = 0; i < G.nint; ++i)
        for (int j = 0; j < G.nint; ++j) {
          BlockOp o = make_op((long long)i * n + (long long)j * n * m, m, n, n);
          for (int c = 0; c < nd; ++c) {
            const int fi = G.face_on_iface[c][i], fj = G.face_on_iface[c][j];
            if (fi < 0 || fj < 0) continue;
            op_src(o, 0, c * childT + (long long)fi * n + (long long)fj * n * nbc, nbc);
          }
          ops.push_back(o);
        }
      add_copy(op, ops, &P.copyD, P.nm);
    }
    // --- S = -Z C, one group per parent boundary group (child c, face F)
    {
      std::vector<GemmGroup> gs;
      const int ngrp = 2 * d * G.sub_per_face;
      for (int gi = 0; gi < ngrp; ++gi) {
        const int c = G.group_child[gi], F = G.group_face[gi];
        GemmGroup g = make_group(P.Z, (long long)m * m, m, Tchild, nd * childT, nbc, P.S + (long long)gi * n * m,
                                 (long long)m * nbp, m, m, n, n, -1.0, 0.0, nm);
        g.nseg = d;
        for (int k = 0; k < d; ++k) {
          const int i = G.int_list[c][k];
          g.aseg[k] = (long long)i * n * m;
          g.bseg[k] = c * childT + (long long)G.face_on_iface[c][i] * n + (long long)F * n * nbc;
        }
        gs.push_back(g);
      }
      add_gemm(op, gs, &P.gemmS);
    }
    // --- Bnz[c] = T_c(exterior faces, interface faces)
    {
      std::vector<BlockOp> ops;
      for (int c = 0; c < nd; ++c)
        for (int e = 0; e < d; ++e)
          for (int k = 0; k < d; ++k) {
            BlockOp o = make_op((long long)c * dn * dn + (long long)e * n + (long long)k * n * dn, dn, n, n);
            const int Fe = G.ext_face[c][e], Fk = G.face_on_iface[c][G.int_list[c][k]];
            op_src(o, 0, c * childT + (long long)Fe * n + (long long)Fk * n * nbc, nbc);
            ops.push_back(o);
          }
      add_copy(op, ops, &P.copyB, P.nm);
    }
    // --- parent T = A + B S: the product B S first, then A added in place on
    // its nonzero blocks (a child's exterior faces against its own), so T is
    // written once and only A's blocks are read back
    if (formT) {
      const int ngrp = 2 * d * G.sub_per_face;
      std::vector<BlockOp> ops;
      for (int gr = 0; gr < ngrp; ++gr)
        for (int gc = 0; gc < ngrp; ++gc) {
          const int c = G.group_child[gr];
          if (G.group_child[gc] != c) continue;
          const long long off = (long long)gr * n + (long long)gc * n * nbp;
          BlockOp o = make_op(off, nbp, n, n);
          op_src(o, 0, c * childT + (long long)G.group_face[gr] * n + (long long)G.group_face[gc] * n * nbc, nbc);
          op_src(o, 1, off, nbp);
          ops.push_back(o);
        }
      add_copy(op, ops, &P.fillT, P.nm);
      std::vector<GemmGroup> gs;
      for (int gr = 0; gr < ngrp; ++gr) {
        const int c = G.group_child[gr], F = G.group_face[gr];
        GemmGroup g = make_group(Tchild, nd * childT, nbc, P.S, (long long)m * nbp, m, P.Tp + (long long)gr * n,
                                 (long long)nbp * nbp, nbp, n, nbp, n, 1.0, 0.0, nm);
        g.nseg = d;
        for (int k = 0; k < d; ++k) {
          const int i = G.int_list[c][k];
          g.aseg[k] = c * childT + (long long)F * n + (long long)G.face_on_iface[c][i] * n * nbc;
          g.bseg[k] = (long long)i * n;
        }
        gs.push_back(g);
      }
      add_gemm(op, gs, &P.gemmT);
    }
    // --- solve: h_int(i) = h_c1(face) + h_c2(face)
    const double* hchild = op->h[lev + 1];
    const long long hstride_c = (long long)NR * nbc;
    {
      std::vector<BlockOp> ops;
      for (int i = 0; i < G.nint; ++i) {
        BlockOp o = make_op((long long)i * n, m, n, 0);
        op_src(o, 0, G.iface[i][0] * hstride_c + (long long)G.iface[i][1] * n, nbc);
        op_src(o, 0, G.iface[i][2] * hstride_c + (long long)G.iface[i][3] * n, nbc);
        ops.push_back(o);
      }
      add_copy(op, ops, &P.copyHint, P.nm);
    }
    // gt = -Z h_int
    add_gemm(op, {make_group(P.Z, (long long)m * m, m, P.hint, (long long)NR * m, m, P.gt, (long long)NR * m, m, m,
                             NR, m, -1.0, 0.0, nm)},
             &P.gemmGt);
    // h_parent(c, F) = h_c(F) + Bnz_c(F, :) gt(interfaces of c)
    if (lev > 0 || op->root_h) {
      std::vector<GemmGroup> gs;
      const int ngrp = 2 * d * G.sub_per_face;
      for (int gi = 0; gi < ngrp; ++gi) {
        const int c = G.group_child[gi], F = G.group_face[gi];
        int e = 0;
        while (G.ext_face[c][e] != F) ++e;
        GemmGroup g = make_group(P.Bnz, (long long)nd * dn * dn, dn, P.gt, (long long)NR * m, m,
                                 op->h[lev] + (long long)gi * n, (long long)NR * nbp, nbp, n, NR, n, 1.0, 1.0, nm,
                                 hchild + c * hstride_c + (long long)F * n, nd * hstride_c, nbc);
        g.nseg = d;
        for (int k = 0; k < d; ++k) {
          g.aseg[k] = (long long)c * dn * dn + (long long)e * n + (long long)k * n * dn;
          g.bseg[k] = (long long)G.int_list[c][k] * n;
        }
        gs.push_back(g);
      }
      add_gemm(op, gs, &P.gemmHp);
    }
    // down: g_int = S g + gt
    add_gemm(op, {make_group(P.S, (long long)m * nbp, m, op->g[lev], (long long)NR * nbp, nbp, P.gint,
                             (long long)NR * m, m, m, NR, nbp, 1.0, 1.0, nm, P.gt, (long long)NR * m, m)},
             &P.gemmDown);
    // children g: exterior faces from the parent's g, interface faces from g_int
    {
      std::vector<BlockOp> ops;
      for (int c = 0; c < nd; ++c)
        for (int f = 0; f < 2 * d; ++f) {
          BlockOp o = make_op(c * hstride_c + (long long)f * n, nbc, n, 0);
          if (G.group_of[c][f] >= 0) {
            op_src(o, 0, (long long)G.group_of[c][f] * n, nbp);
          } else {
            int i = 0;
            while (G.face_on_iface[c][i] != f) ++i;
            op_src(o, 1, (long long)i * n, m);
          }
          ops.push_back(o);
        }
      add_copy(op, ops, &P.copyGchild, P.nm);
    }
    // --- adjoint: parent groups <- children's exterior faces
    {
      std::vector<BlockOp> ops;
      const int ngrp = 2 * d * G.sub_per_face;
      for (int gi = 0; gi < ngrp; ++gi) {
        BlockOp o = make_op((long long)gi * n, nbp, n, 0);
        op_src(o, 0, G.group_child[gi] * hstride_c + (long long)G.group_face[gi] * n, nbc);
        ops.push_back(o);
      }
      add_copy(op, ops, &P.copyPext, P.nm);
    }
    // g_parent += S^T g_int
    add_gemm(op, {make_group(P.S, (long long)m * nbp, m, P.gint, (long long)NR * m, m, op->g[lev], (long long)NR * nbp,
                             nbp, nbp, NR, m, 1.0, 1.0, nm, op->g[lev], (long long)NR * nbp, nbp)},
             &P.gemmSt, true, false);
    // gt_total(i) = g_int(i) + sum over both children of Bnz_c(., i)^T h_parent(c, .)
    // (at the root only when the root's h comes from outside: a subtree root)
    if (lev > 0 || op->root_h) {
      for (int pass = 0; pass < 2; ++pass) {
        std::vector<GemmGroup> gs;
        for (int c = 0; c < nd; ++c)
          for (int k = 0; k < d; ++k) {
            const int i = G.int_list[c][k];
            if ((G.iface[i][pass == 0 ? 0 : 2]) != c) continue;
            const double* C0 = pass == 0 ? P.gint + (long long)i * n : P.gt + (long long)i * n;
            GemmGroup g = make_group(P.Bnz, (long long)nd * dn * dn, dn, op->h[lev], (long long)NR * nbp, nbp,
                                     P.gt + (long long)i * n, (long long)NR * m, m, n, NR, n, 1.0, 1.0, nm, C0,
                                     (long long)NR * m, m);
            g.nseg = d;
            for (int e = 0; e < d; ++e) {
              g.aseg[e] = (long long)c * dn * dn + (long long)e * n + (long long)k * n * dn;
              g.bseg[e] = (long long)G.group_of[c][G.ext_face[c][e]] * n;
            }
            gs.push_back(g);
          }
        add_gemm(op, gs, pass == 0 ? &P.gemmBt1 : &P.gemmBt2, true, false);
      }
    }
    // h_int = -Z^T gt_total
    add_gemm(op, {make_group(P.Z, (long long)m * m, m, (lev > 0 || op->root_h) ? P.gt : P.gint, (long long)NR * m, m,
                             P.hint,
                             (long long)NR * m, m, m, NR, m, -1.0, 0.0, nm)},
             &P.gemmZt, true, false);
  }
  return finish_plan(op);
}

// split-K workspace, allocation-free descriptor copy, descriptor upload
int finish_plan(hps_op* op) {
  // split-K workspace, shared by all calls (they run one after another)
  if (op->split_elems > 0) {
    op->splitws = (double*)op_alloc(op, sizeof(double) * op->split_elems, false);
    if (!op->splitws) { set_error("device allocation failed (split-K workspace)"); return HPS_ENOMEM; }
  }
  for (auto& g : op->hgroups) g.part = g.ksplit > 1 ? op->splitws + g.part_off : nullptr;
  HPS_TRY(plan_static_solve(op));
  // upload the descriptor tables: one allocation, one copy
  struct Table {
    const void* src;
    size_t bytes;
    void** dst;
  };
  const size_t ns = op->static_ok ? op->hgroups_static.size() : 0;
  const Table tabs[5] = {
      {op->hgroups.data(), sizeof(GemmGroup) * op->hgroups.size(), (void**)&op->dgroups},
      {op->hops.data(), sizeof(BlockOp) * op->hops.size(), (void**)&op->dops},
      {op->hitems.data(), sizeof(CopyItem) * op->hitems.size(), (void**)&op->ditems},
      {op->htasks.data(), sizeof(CopyTask) * op->htasks.size(), (void**)&op->dtasks},
      {op->hgroups_static.data(), sizeof(GemmGroup) * ns, (void**)&op->dgroups_static}};
  size_t off[5], total = 0;
  for (int t = 0; t < 5; ++t) {
    off[t] = total;
    total += (size_t)al256((long long)std::max<size_t>(tabs[t].bytes, 1));
  }
  char* dev = (char*)op_alloc(op, total, false);
  if (!dev) {
    set_error("device allocation failed (descriptors)");
    return HPS_ENOMEM;
  }
  std::vector<char> host(total, 0);
  for (int t = 0; t < 5; ++t) {
    if (tabs[t].bytes) std::memcpy(host.data() + off[t], tabs[t].src, tabs[t].bytes);
    *tabs[t].dst = dev + off[t];
  }
  if (!op->static_ok) op->dgroups_static = nullptr;
  HPS_HIP_TRY(hipMemcpy(dev, host.data(), total, hipMemcpyHostToDevice));
  return HPS_OK;
}

// the build's status block on the host: flags, then every level's residuals
// (synchronizes the op's stream)
int download_status(hps_op* op, std::vector<double>* out) {
  out->assign(8 + op->rho_n, 0.0);
  hipError_t e = hipMemcpyAsync(out->data(), op->flag, sizeof(double) * out->size(), hipMemcpyDeviceToHost,
                                op->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(op->stream);
  if (e != hipSuccess) {
    set_error(std::string("build failed on the device: ") + hipGetErrorString(e));
    return HPS_EDEVICE;
  }
  return HPS_OK;
}

// Per-level probe results; status is the downloaded status block (nullptr:
// download it here).  Node residuals are read from the last probe each node
// went through.
int collect_info(hps_op* op, const std::vector<double>* status = nullptr) {
  if (op->info_ready) return HPS_OK;
  std::vector<double> own;
  if (!status) {
    HPS_TRY(download_status(op, &own));
    status = &own;
  }
  const int L = op->tree.depth;
  op->info.assign(L, hps_level_info_t());
  for (int lev = 0; lev < L; ++lev) {
    const LevelPlan& P = op->levels[lev];
    const int nk = (P.schur && !(op->flags & HPS_FLAG_TEST_NO_REFINE)) ? kNsSteps + 1 : 1;
    const double* rho = status->data() + 8 + (P.rho - op->rho_all);
    hps_level_info_t& I = op->info[lev];
    I.level = lev;
    I.m = P.m;
    I.nodes = P.nm;
    I.block_inverse = P.schur ? 1 : 0;
    I.ns_steps = 0;
    I.residual0 = 0.0;
    I.residual = 0.0;
    I.worst_node = 0;
    for (long long b = 0; b < P.nm; ++b) {
      const double r0 = rho[b];
      // a node is refined at step k + 1 when the probe after step k is above
      // the threshold (the gate); its final residual is that of the last probe
      int steps = 0;
      double rf = r0;
      for (int k = 0; k + 1 < nk; ++k) {
        if (!(rho[(size_t)k * P.nm + b] <= kNsRefine)) {
          steps = k + 1;
          rf = rho[(size_t)(k + 1) * P.nm + b];
        } else {
          break;
        }
      }
      if (!(r0 <= I.residual0)) I.residual0 = r0;
      if (!(rf <= I.residual)) {
        I.residual = rf;
        I.worst_node = b;
        I.ns_steps = steps;
      }
    }
  }
  op->info_ready = true;
  return HPS_OK;
}

int run_build(hps_op* op, const double* coeffs, hipStream_t st, bool reset_flags = true,
              const std::function<int(int)>* after = nullptr) {
  const int L = op->tree.depth, nd = op->nd;
  if (reset_flags) HPS_HIP_TRY(hipMemsetAsync(op->flag, 0, sizeof(int) * 4, st));
  if (op->ext_side > 0) {
    // top levels of a subtree-recomputing operator: Tleaf holds the subtree roots' T
  } else {
  stage_begin(op, "leaf_factor", st);
  if (op->d == 2) {
    HPS_TRY(leaf2d_launch(op->p, coeffs, op->cst->D1, op->cst->D2, op->cst->Mt, op->LU, op->perm, op->pos, op->Y,
                          op->flag, op->nl, st));
  } else {
    HPS_TRY(leaf3d_assemble_launch(coeffs, op->cst->D1, op->cst->D2, op->cst->Mt, op->p, op->Lbuf, op->Rbuf, op->nl,
                                   st));
    HPS_TRY(run_gj(op, op->leaf_gj, st));
    HPS_TRY(run_gemm(op, op->gemmYleaf, st));
  }
  stage_end(op, st);
  stage_begin(op, "leaf_T", st);
  HPS_TRY(run_gemm(op, op->gemmTleaf, st));
  stage_end(op, st);
  }
  if (after) HPS_TRY((*after)(L));
  static const char* names[] = {"merge_l0", "merge_l1", "merge_l2", "merge_l3", "merge_l4", "merge_l5",
                                "merge_l6", "merge_l7", "merge_l8", "merge_l9", "merge_l10", "merge_l11"};
  for (int lev = L - 1; lev >= 0; --lev) {
    LevelPlan& P = op->levels[lev];
    const double* Tchild = lev == L - 1 ? op->Tleaf : op->levels[lev + 1].Tp;
    const long long childstride = (long long)nd * P.nbc * P.nbc;
    stage_begin(op, names[lev < 12 ? lev : 11], st);
    HPS_TRY(run_copy(op, P.copyD, 0, P.Dbuf, (long long)P.m * P.m, Tchild, childstride, nullptr, 0, P.nm, st));
    if (!P.schur) HPS_TRY(run_gemm(op, P.probe1, st, kProbes));  // D x, before the inversion overwrites D
    if (P.schur) {
      HPS_TRY(run_schur(op, P, st));
      HPS_TRY(run_probe(op, P, 0, st));
      if (!(op->flags & HPS_FLAG_TEST_NO_REFINE)) HPS_TRY(run_refine(op, P, st));
    } else {
      HPS_TRY(run_gj(op, P.gj, st));
      HPS_TRY(run_probe(op, P, 0, st));
    }
    HPS_TRY(run_gemm(op, P.gemmS, st));
    HPS_TRY(run_copy(op, P.copyB, 0, P.Bnz, (long long)nd * P.dn * P.dn, Tchild, childstride, nullptr, 0, P.nm, st));
    if (P.Tp) {
      HPS_TRY(run_gemm(op, P.gemmT, st));
      HPS_TRY(run_copy(op, P.fillT, 0, P.Tp, (long long)P.nbp * P.nbp, Tchild, childstride, P.Tp,
                       (long long)P.nbp * P.nbp, P.nm, st));
    }
    stage_end(op, st);
    if (after) HPS_TRY((*after)(lev));
  }
  return HPS_OK;
}

// Upward part of a solve: root data (when bdry is given), the sources' leaf
// solutions and the upward pass of their fluxes; without sources the
// interface data of every merge start at zero.  Operators whose leaves are
// subtree roots take the leaf-level fluxes h[L] as already filled.
// Source part of a solve at the leaves: v = L_ii^{-1} f_int and h = Q_i v.
int run_solve_leaf_src(hps_op* op, const SolveCtx& c, const double* src, int nrhs, hipStream_t st,
                       int max_wg_per_cu = 0) {
  const int NR = op->NR;
  if (op->d == 2) {
    HPS_TRY(leaf_src_launch(op->LU, op->perm, op->pos, src, op->cst->Ii, op->ni, op->npts, op->nl, nrhs, c.at(op->v),
                            NR, st, op->rstride, max_wg_per_cu));
  } else {
    HPS_TRY(leaf_gather_int_launch(src, op->cst->Ii, op->ni, op->npts, op->nl, nrhs, NR, c.at(op->fint), st));
    HPS_TRY(run_gemm_ctx(c, op->gemmVleaf, st, nrhs));
  }
  return run_gemm_ctx(c, op->gemmHleaf, st, nrhs);
}

// Upward pass of the sources' fluxes over merge levels lev_hi down to lev_lo:
// h_int gathered from the children, g~ = -Z h_int, h = h_ext + B g~.
int run_solve_levels_up(hps_op* op, const SolveCtx& c, int lev_hi, int lev_lo, int nrhs, hipStream_t st) {
  const int nd = op->nd, NR = op->NR;
  for (int lev = lev_hi; lev >= lev_lo; --lev) {
    LevelPlan& P = op->levels[lev];
    HPS_TRY(run_copy(op, P.copyHint, nrhs, c.at(P.hint), (long long)NR * P.m, c.at(op->h[lev + 1]),
                     (long long)nd * NR * P.nbc, nullptr, 0, P.nm, st));
    HPS_TRY(run_gemm_ctx(c, P.gemmGt, st, nrhs));
    if (lev > 0 || op->root_h) HPS_TRY(run_gemm_ctx(c, P.gemmHp, st, nrhs));
  }
  return HPS_OK;
}

int run_solve_up(hps_op* op, const SolveCtx& c, const double* bdry, const double* src, bool has_src, int nrhs,
                 bool graph_safe, hipStream_t st) {
  const int L = op->tree.depth, NR = op->NR;
  if (bdry) HPS_TRY(run_copy(op, op->copyRoot, nrhs, c.at(op->g[0]), 0, bdry, 0, nullptr, 0, 1, st));
  if (has_src) {
    if (op->ext_side == 0) HPS_TRY(run_solve_leaf_src(op, c, src, nrhs, st));
    HPS_TRY(run_solve_levels_up(op, c, L - 1, 0, nrhs, st));
  } else {
    for (int lev = 0; lev < L; ++lev) {
      LevelPlan& P = op->levels[lev];
      if (graph_safe)
        HPS_TRY(zero_fill_launch(c.at(P.gt), P.nm * NR * P.m, st));
      else
        HPS_HIP_TRY(hipMemsetAsync(P.gt, 0, sizeof(double) * P.nm * NR * P.m, st));
    }
  }
  return HPS_OK;
}

// Downward pass and (ordinary leaves) the leaf solutions u = [P g; Y g + v].
int run_solve_down(hps_op* op, const SolveCtx& c, bool has_src, double* u, int nrhs, hipStream_t st) {
  const int L = op->tree.depth, nd = op->nd, NR = op->NR;
  for (int lev = 0; lev < L; ++lev) {
    LevelPlan& P = op->levels[lev];
    HPS_TRY(run_gemm_ctx(c, P.gemmDown, st, nrhs));
    HPS_TRY(run_copy(op, P.copyGchild, nrhs, c.at(op->g[lev + 1]), (long long)nd * NR * P.nbc, c.at(op->g[lev]),
                     (long long)NR * P.nbp, c.at(P.gint), (long long)NR * P.m, P.nm, st));
  }
  if (op->ext_side == 0)
    HPS_TRY(leaf_out_launch(op->Y, op->cst->P, c.at(op->g[L]), has_src ? c.at(op->v) : nullptr, op->cst->Ii,
                            op->cst->Ie, op->ni, op->ne, op->nb, op->npts, op->nl, nrhs, NR, u, st, op->rstride));
  return HPS_OK;
}

int run_solve_chunk(hps_op* op, const SolveCtx& c, const double* bdry, const double* src, double* u, int nrhs,
                    bool graph_safe, hipStream_t st) {
  if (!graph_safe) stage_begin(op, "solve", st);
  HPS_TRY(run_solve_up(op, c, bdry, src, src != nullptr, nrhs, graph_safe, st));
  HPS_TRY(run_solve_down(op, c, src != nullptr, u, nrhs, st));
  if (!graph_safe) stage_end(op, st);
  return HPS_OK;
}

// Solve of a subtree-recomputing operator (Algorithm "Subtree recomputation
// strategy", Section 4.1): with sources, every subtree is rebuilt from its
// coefficients and its sources' outgoing flux taken at its root; the top
// levels run their upward and downward passes; then every subtree is rebuilt
// once more and solved from the boundary data the top levels handed down.
int run_solve_subtrees(hps_op* top, const double* bdry, const double* src, double* u, int nrhs, hipStream_t st) {
  hps_op* sub = top->sub;
  const int Lt = top->tree.depth, NR = top->NR;
  const long long nsub = top->nl, nb = top->nbl[Lt];
  const long long coef_stride = sub->nl * (sub->d == 2 ? 6 : 10) * sub->npts;
  const long long pts_stride = sub->nl * sub->npts;
  const SolveCtx ct = own_ctx(top), cs = own_ctx(sub);
  if (src) {
    for (long long j = 0; j < nsub; ++j) {
      HPS_TRY(run_build(sub, top->sub_coef + j * coef_stride, st));
      HPS_TRY(run_solve_up(sub, cs, nullptr, src + j * pts_stride, true, nrhs, false, st));
      HPS_HIP_TRY(hipMemcpyAsync(top->h[Lt] + j * NR * nb, sub->h[0], sizeof(double) * nrhs * nb,
                                 hipMemcpyDeviceToDevice, st));
    }
  }
  HPS_TRY(run_solve_up(top, ct, bdry, nullptr, src != nullptr, nrhs, false, st));
  HPS_TRY(run_solve_down(top, ct, src != nullptr, nullptr, nrhs, st));
  for (long long j = 0; j < nsub; ++j) {
    HPS_TRY(run_build(sub, top->sub_coef + j * coef_stride, st));
    HPS_TRY(run_solve_up(sub, cs, top->g[Lt] + j * NR * nb, src ? src + j * pts_stride : nullptr, src != nullptr,
                         nrhs, false, st));
    HPS_TRY(run_solve_down(sub, cs, src != nullptr, u + j * pts_stride, nrhs, st));
  }
  return HPS_OK;
}

// Adjoint of the downward pass, leaves to root: (ordinary leaves) g_leaf =
// Y^T w_int + P^T w_ext and v = w_int, then per level the interface sums
// g_int, the parent's exterior faces and g_parent += S^T g_int.  Operators
// whose leaves are subtree roots take g[L] as already filled.
int run_adjoint_up(hps_op* op, const double* w, int nrhs, hipStream_t st) {
  const int L = op->tree.depth, nd = op->nd, NR = op->NR;
  if (op->ext_side == 0) {
    HPS_TRY(leaf_gather_pts_launch(w, op->cst->Ii, op->ni, op->npts, op->nl, nrhs, NR, op->v, st, op->rstride));
    HPS_TRY(leaf_gather_pts_launch(w, op->cst->Ie, op->ne, op->npts, op->nl, nrhs, NR, op->wext, st, op->rstride));
    HPS_TRY(run_gemm(op, op->adjYt, st, nrhs));
    HPS_TRY(run_gemm(op, op->adjPt, st, nrhs));
  }
  for (int lev = L - 1; lev >= 0; --lev) {
    LevelPlan& P = op->levels[lev];
    const long long cstride = (long long)nd * NR * P.nbc;
    HPS_TRY(run_copy(op, P.copyHint, nrhs, P.gint, (long long)NR * P.m, op->g[lev + 1], cstride, nullptr, 0, P.nm, st));
    HPS_TRY(run_copy(op, P.copyPext, nrhs, op->g[lev], (long long)NR * P.nbp, op->g[lev + 1], cstride, nullptr, 0, P.nm,
                     st));
    HPS_TRY(run_gemm(op, P.gemmSt, st, nrhs));
  }
  return HPS_OK;
}

// Adjoint of the source's upward pass, root to leaves, from h[0] (zero at the
// domain root, handed down at a subtree root), then (ordinary leaves)
// v += Q_i^T h_leaf, f_int = L_ii^{-T} v scattered into lam_src.
int run_adjoint_down(hps_op* op, double* lam_src, int nrhs, hipStream_t st) {
  const int L = op->tree.depth, nd = op->nd, NR = op->NR;
  if (!op->root_h) HPS_HIP_TRY(hipMemsetAsync(op->h[0], 0, sizeof(double) * NR * op->nbl[0], st));
  for (int lev = 0; lev < L; ++lev) {
    LevelPlan& P = op->levels[lev];
    if (lev > 0 || op->root_h) {
      HPS_TRY(run_gemm(op, P.gemmBt1, st, nrhs));
      HPS_TRY(run_gemm(op, P.gemmBt2, st, nrhs));
    }
    HPS_TRY(run_gemm(op, P.gemmZt, st, nrhs));
    HPS_TRY(run_copy(op, P.copyGchild, nrhs, op->h[lev + 1], (long long)nd * NR * P.nbc, op->h[lev],
                     (long long)NR * P.nbp, P.hint, (long long)NR * P.m, P.nm, st));
  }
  if (op->ext_side > 0) return HPS_OK;
  HPS_TRY(run_gemm(op, op->adjQt, st, nrhs));
  if (op->d == 2) {
    HPS_TRY(leaf_src_t_launch(op->LU, op->perm, op->v, op->ni, op->nl, nrhs, NR, op->fint, st));
  } else {
    HPS_TRY(run_gemm(op, op->adjLinvT, st, nrhs));
  }
  return leaf_scatter_int_launch(op->fint, op->cst->PosI, op->ni, op->npts, op->nl, nrhs, NR, lam_src, st,
                                 op->rstride);
}

int run_adjoint_chunk(hps_op* op, const double* w, double* lam_src, double* lam_bdry, int nrhs, hipStream_t st) {
  stage_begin(op, "adjoint", st);
  HPS_TRY(run_adjoint_up(op, w, nrhs, st));
  if (lam_bdry) HPS_TRY(run_copy(op, op->copyRoot, nrhs, lam_bdry, 0, op->g[0], 0, nullptr, 0, 1, st));
  HPS_TRY(run_adjoint_down(op, lam_src, nrhs, st));
  stage_end(op, st);
  return HPS_OK;
}

// Adjoint solve of a subtree-recomputing operator: the transposed passes in
// reverse order, with every subtree rebuilt twice (its leaves-to-root part
// gives the g of its root; after the top levels, the same part again, to
// restore its interface sums, and then its root-to-leaves part from the h
// the top levels hand down).
int run_adjoint_subtrees(hps_op* top, const double* w, double* lam_src, double* lam_bdry, int nrhs, hipStream_t st) {
  hps_op* sub = top->sub;
  const int Lt = top->tree.depth, NR = top->NR;
  const long long nsub = top->nl, nb = top->nbl[Lt];
  const long long coef_stride = sub->nl * 6 * sub->npts, pts_stride = sub->nl * sub->npts;
  for (long long j = 0; j < nsub; ++j) {
    HPS_TRY(run_build(sub, top->sub_coef + j * coef_stride, st));
    HPS_TRY(run_adjoint_up(sub, w + j * pts_stride, nrhs, st));
    HPS_HIP_TRY(hipMemcpyAsync(top->g[Lt] + j * NR * nb, sub->g[0], sizeof(double) * nrhs * nb,
                               hipMemcpyDeviceToDevice, st));
  }
  HPS_TRY(run_adjoint_up(top, nullptr, nrhs, st));
  if (lam_bdry) HPS_TRY(run_copy(top, top->copyRoot, nrhs, lam_bdry, 0, top->g[0], 0, nullptr, 0, 1, st));
  HPS_TRY(run_adjoint_down(top, nullptr, nrhs, st));
  for (long long j = 0; j < nsub; ++j) {
    HPS_TRY(run_build(sub, top->sub_coef + j * coef_stride, st));
    HPS_TRY(run_adjoint_up(sub, w + j * pts_stride, nrhs, st));
    HPS_HIP_TRY(hipMemcpyAsync(sub->h[0], top->h[Lt] + j * NR * nb, sizeof(double) * nrhs * nb,
                               hipMemcpyDeviceToDevice, st));
    HPS_TRY(run_adjoint_down(sub, lam_src + j * pts_stride, nrhs, st));
  }
  return HPS_OK;
}

// ---------------------------------------------------------------------------
// ItI variant (Appendix B), in the real representation of complex data (see
// iti.hip): at a merge whose children have n reals per side, the unknowns
// g_int are the incoming data of the children on the interfaces, in the
// order [g5a, g8a, g6c, g7c, g5b, g6b, g7d, g8d] of eq. (2D_ItI_merge_2).
// Unknown k belongs to child kItiUnk[k][0] on its face kItiUnk[k][1]; its
// constraint row reads the outgoing data of the neighbour kItiUnk[k][2] on
// face kItiUnk[k][3]:  g_k + T^y(f_y, .) g^y + h^y(f_y) = 0.  D, C, B and A
// are formed densely (their zero blocks included) by block copies from the
// children's T.
// ---------------------------------------------------------------------------
constexpr int kItiUnk[8][4] = {{0, 1, 1, 3}, {0, 2, 3, 0}, {2, 0, 1, 2}, {2, 3, 3, 1},
                               {1, 3, 0, 1}, {1, 2, 2, 0}, {3, 1, 2, 3}, {3, 0, 0, 2}};

// bytes of one ItI merge level's transient buffers (D12, D21, W, W^{-1}, C
// and the Gauss-Jordan panels of W)
long long iti_level_ws_bytes(int n, long long nm) {
  const long long w = 4LL * n, mi = 8LL * n, d8 = sizeof(double);
  return 4 * al256(d8 * nm * w * w) + al256(d8 * nm * mi * mi) + gj_ws_bytes((int)w, nm);
}

int plan_iti(hps_op* op) {
  const int L = op->tree.depth, NR = op->NR, p = op->p;
  const long long nl = op->nl;
  const int m = op->npts, nb = op->nb, nr2 = 2 * (4 * p - 4), ni2 = op->ni;
  const MergeGeom& G = merge_geom(2);
  const ItiConsts* ic = op->ic;
  // leaves: B (transient), B^{-1}, Y
  op->Lbuf = (double*)op_alloc(op, sizeof(double) * nl * m * m, false);
  op->Rbuf = (double*)op_alloc(op, sizeof(double) * nl * ni2);  // interior row scales
  op->LU = (double*)op_alloc(op, sizeof(double) * nl * m * m);
  op->Y = (double*)op_alloc(op, sizeof(double) * nl * m * nb);
  op->flag = (int*)op_alloc(op, sizeof(int) * 4, false);
  op->nbl.assign(L + 1, 0);
  for (int l = 0; l <= L; ++l) op->nbl[l] = nb << (L - l);
  // T of the leaves and of the levels below the root (two alternating buffers)
  for (int k = 0; k < (L >= 2 ? 2 : 1); ++k) {
    op->Tbuf[k] = (double*)op_alloc(op, sizeof(double) * nl * nb * nb, false);
    if (!op->Tbuf[k]) { set_error("device allocation failed (T workspace)"); return HPS_ENOMEM; }
  }
  op->Tleaf = op->Tbuf[0];
  if (!op->Lbuf || !op->Rbuf || !op->LU || !op->Y || !op->flag) {
    set_error("device allocation failed (ItI leaf operators)");
    return HPS_ENOMEM;
  }
  HPS_TRY(plan_gj(op, &op->leaf_gj, op->Lbuf, op->LU, m, nl));
  // solve workspace
  op->g.assign(L + 1, nullptr);
  op->h.assign(L + 1, nullptr);
  for (int l = 0; l <= L; ++l) {
    const long long nodes = 1LL << (2 * l);
    op->g[l] = (double*)op_alloc(op, sizeof(double) * nodes * NR * op->nbl[l], false);
    op->h[l] = (double*)op_alloc(op, sizeof(double) * nodes * NR * op->nbl[l], false);
    if (!op->g[l] || !op->h[l]) { set_error("device allocation failed (solve workspace)"); return HPS_ENOMEM; }
  }
  op->v = (double*)op_alloc(op, sizeof(double) * nl * NR * m, false);
  op->uws = (double*)op_alloc(op, sizeof(double) * nl * NR * m, false);
  op->fint = (double*)op_alloc(op, sizeof(double) * nl * NR * ni2, false);
  if (!op->v || !op->uws || !op->fint) { set_error("device allocation failed (solve workspace)"); return HPS_ENOMEM; }
  // leaf products: Y = B^{-1}(:, Robin rows) P, T = Q H Y; solve: v =
  // B^{-1}(:, interior rows) f_int, h = Q H v, u = Y g (+ v)
  add_gemm(op, {make_group(op->LU, (long long)m * m, m, ic->Pr, 0, nr2, op->Y, (long long)m * nb, m, m, nb, nr2, 1.0,
                           0.0, nl)},
           &op->gemmYleaf);
  add_gemm(op, {make_group(ic->QHr, 0, nb, op->Y, (long long)m * nb, m, op->Tleaf, (long long)nb * nb, nb, nb, nb, m,
                           1.0, 0.0, nl)},
           &op->gemmTleaf);
  add_gemm(op, {make_group(op->LU + (long long)nr2 * m, (long long)m * m, m, op->fint, (long long)NR * ni2, ni2, op->v,
                           (long long)NR * m, m, m, NR, ni2, 1.0, 0.0, nl)},
           &op->gemmVleaf);
  add_gemm(op, {make_group(ic->QHr, 0, nb, op->v, (long long)NR * m, m, op->h[L], (long long)NR * nb, nb, nb, NR, m,
                           1.0, 0.0, nl)},
           &op->gemmHleaf);
  add_gemm(op, {make_group(op->Y, (long long)m * nb, m, op->g[L], (long long)NR * nb, nb, op->uws, (long long)NR * m, m,
                           m, NR, nb, 1.0, 1.0, nl, op->v, (long long)NR * m, m)},
           &op->gemmUleaf);
  add_gemm(op, {make_group(op->Y, (long long)m * nb, m, op->g[L], (long long)NR * nb, nb, op->uws, (long long)NR * m, m,
                           m, NR, nb, 1.0, 0.0, nl)},
           &op->gemmUleaf0);
  {
    BlockOp o = make_op(0, op->nbl[0], op->nbl[0], 0);
    op_src(o, 0, 0, op->nbl[0]);
    add_copy(op, {o}, &op->copyRoot);
  }
  // merge-level build workspace and the identity for W = I - D12 D21
  {
    long long need = 0;
    int wmax = 1;
    for (int lev = 0; lev < L; ++lev) {
      const int n = op->nbl[lev + 1] / 4;
      need = std::max(need, iti_level_ws_bytes(n, 1LL << (2 * lev)));
      wmax = std::max(wmax, 4 * n);
    }
    op->lvl_ws = (char*)op_alloc(op, (size_t)need, false);
    op->ident = (double*)op_alloc(op, sizeof(double) * (size_t)wmax * wmax, false);
    if (!op->lvl_ws || !op->ident) { set_error("device allocation failed (ItI merge workspace)"); return HPS_ENOMEM; }
    op->lvl_ws_bytes = need;
    op->ident_ld = wmax;
    std::vector<double> I((size_t)wmax * wmax, 0.0);
    for (int i = 0; i < wmax; ++i) I[(size_t)i * wmax + i] = 1.0;
    HPS_HIP_TRY(hipMemcpy(op->ident, I.data(), sizeof(double) * I.size(), hipMemcpyHostToDevice));
  }
  op->levels.assign(L, LevelPlan());
  for (int lev = L - 1; lev >= 0; --lev) {
    LevelPlan& P = op->levels[lev];
    op->lvl_cur = 0;
    P.lev = lev;
    P.nm = 1LL << (2 * lev);
    P.nbc = op->nbl[lev + 1];
    P.nbp = op->nbl[lev];
    P.n = P.nbc / 4;
    const int n = P.n, w = 4 * n, mi = 8 * n, nbc = P.nbc, nbp = P.nbp;
    P.m = mi;
    const long long nm = P.nm, childT = (long long)nbc * nbc;
    P.Z = (double*)op_alloc(op, sizeof(double) * nm * mi * mi);
    P.S = (double*)op_alloc(op, sizeof(double) * nm * mi * nbp);
    P.Bnz = (double*)op_alloc(op, sizeof(double) * nm * nbp * mi);
    if (lev > 0) P.Tp = op->Tbuf[(L - lev) % 2];
    P.D12 = (double*)lvl_take(op, sizeof(double) * nm * w * w);
    P.D21 = (double*)lvl_take(op, sizeof(double) * nm * w * w);
    P.Dbuf = (double*)lvl_take(op, sizeof(double) * nm * w * w);
    P.Winv = (double*)lvl_take(op, sizeof(double) * nm * w * w);
    P.Cm = (double*)lvl_take(op, sizeof(double) * nm * mi * nbp);
    P.hint = (double*)op_alloc(op, sizeof(double) * nm * NR * mi, false);
    P.gt = (double*)op_alloc(op, sizeof(double) * nm * NR * mi, false);
    P.gint = (double*)op_alloc(op, sizeof(double) * nm * NR * mi, false);
    if (!P.Z || !P.S || !P.Bnz || !P.D12 || !P.D21 || !P.Dbuf || !P.Winv || !P.Cm || !P.hint || !P.gt || !P.gint) {
      set_error("device allocation failed (ItI merge level)");
      return HPS_ENOMEM;
    }
    HPS_TRY(plan_gj(op, &P.gj, P.Dbuf, P.Winv, w, nm, true));
    // D12 (rows: unknowns 0-3, columns: unknowns 4-7) and D21 (the reverse)
    for (int half = 0; half < 2; ++half) {
      std::vector<BlockOp> ops;
      for (int r = 0; r < 4; ++r)
        for (int s = 0; s < 4; ++s) {
          const int k = half * 4 + r, k2 = (1 - half) * 4 + s;
          BlockOp o = make_op((long long)r * n + (long long)s * n * w, w, n, n);
          const int y = kItiUnk[k][2];
          if (kItiUnk[k2][0] == y)
            op_src(o, 0, y * childT + (long long)kItiUnk[k][3] * n + (long long)kItiUnk[k2][1] * n * nbc, nbc);
          ops.push_back(o);
        }
      add_copy(op, ops, half == 0 ? &P.copyD : &P.copyD21, P.nm);
    }
    // W = I - D12 D21
    add_gemm(op, {make_group(P.D12, (long long)w * w, w, P.D21, (long long)w * w, w, P.Dbuf, (long long)w * w, w, w, w,
                             w, -1.0, 1.0, nm, op->ident, 0, op->ident_ld)},
             &P.gemmW);
    // Z = D^{-1} (eq. ItI_D_inv): Z11 = W^{-1}, Z12 = -W^{-1} D12,
    // Z21 = -D21 W^{-1}, Z22 = I - D21 Z12
    {
      BlockOp o = make_op(0, mi, w, w);
      op_src(o, 0, 0, w);
      add_copy(op, {o}, &P.copyZ11, P.nm);
    }
    add_gemm(op, {make_group(P.Winv, (long long)w * w, w, P.D12, (long long)w * w, w, P.Z + (long long)w * mi,
                             (long long)mi * mi, mi, w, w, w, -1.0, 0.0, nm),
                  make_group(P.D21, (long long)w * w, w, P.Winv, (long long)w * w, w, P.Z + w, (long long)mi * mi, mi,
                             w, w, w, -1.0, 0.0, nm)},
             &P.gemmZ1);
    add_gemm(op, {make_group(P.D21, (long long)w * w, w, P.Z + (long long)w * mi, (long long)mi * mi, mi,
                             P.Z + w + (long long)w * mi, (long long)mi * mi, mi, w, w, w, -1.0, 1.0, nm, op->ident, 0,
                             op->ident_ld)},
             &P.gemmZPP);
    // C (rows: unknowns, columns: parent groups); S = -Z C
    {
      std::vector<BlockOp> ops;
      for (int k = 0; k < 8; ++k)
        for (int gj = 0; gj < 8; ++gj) {
          BlockOp o = make_op((long long)k * n + (long long)gj * n * mi, mi, n, n);
          const int y = kItiUnk[k][2];
          if (G.group_child[gj] == y)
            op_src(o, 0, y * childT + (long long)kItiUnk[k][3] * n + (long long)G.group_face[gj] * n * nbc, nbc);
          ops.push_back(o);
        }
      add_copy(op, ops, &P.copyC, P.nm);
    }
    add_gemm(op, {make_group(P.Z, (long long)mi * mi, mi, P.Cm, (long long)mi * nbp, mi, P.S, (long long)mi * nbp, mi,
                             mi, nbp, mi, -1.0, 0.0, nm)},
             &P.gemmS);
    // B (rows: parent groups, columns: unknowns) and A (parent groups)
    {
      std::vector<BlockOp> ops;
      for (int gi = 0; gi < 8; ++gi)
        for (int k = 0; k < 8; ++k) {
          BlockOp o = make_op((long long)gi * n + (long long)k * n * nbp, nbp, n, n);
          const int c = G.group_child[gi];
          if (kItiUnk[k][0] == c)
            op_src(o, 0, c * childT + (long long)G.group_face[gi] * n + (long long)kItiUnk[k][1] * n * nbc, nbc);
          ops.push_back(o);
        }
      add_copy(op, ops, &P.copyB, P.nm);
    }
    if (P.Tp) {
      std::vector<BlockOp> ops;
      for (int gi = 0; gi < 8; ++gi)
        for (int gj = 0; gj < 8; ++gj) {
          BlockOp o = make_op((long long)gi * n + (long long)gj * n * nbp, nbp, n, n);
          const int c = G.group_child[gi];
          if (G.group_child[gj] == c)
            op_src(o, 0, c * childT + (long long)G.group_face[gi] * n + (long long)G.group_face[gj] * n * nbc, nbc);
          ops.push_back(o);
        }
      add_copy(op, ops, &P.fillT, P.nm);
      add_gemm(op, {make_group(P.Bnz, (long long)nbp * mi, nbp, P.S, (long long)mi * nbp, mi, P.Tp, (long long)nbp * nbp,
                               nbp, nbp, nbp, mi, 1.0, 1.0, nm, P.Tp, (long long)nbp * nbp, nbp)},
               &P.gemmT);
    }
    // solve: h_int, g~ = -Z h_int, h = h_ext + B g~, g_int = S g + g~
    const long long hstride_c = (long long)NR * nbc;
    {
      std::vector<BlockOp> ops;
      for (int k = 0; k < 8; ++k) {
        BlockOp o = make_op((long long)k * n, mi, n, 0);
        op_src(o, 0, kItiUnk[k][2] * hstride_c + (long long)kItiUnk[k][3] * n, nbc);
        ops.push_back(o);
      }
      add_copy(op, ops, &P.copyHint, P.nm);
    }
    add_gemm(op, {make_group(P.Z, (long long)mi * mi, mi, P.hint, (long long)NR * mi, mi, P.gt, (long long)NR * mi, mi,
                             mi, NR, mi, -1.0, 0.0, nm)},
             &P.gemmGt);
    if (lev > 0) {
      std::vector<BlockOp> ops;
      for (int gi = 0; gi < 8; ++gi) {
        BlockOp o = make_op((long long)gi * n, nbp, n, 0);
        op_src(o, 0, G.group_child[gi] * hstride_c + (long long)G.group_face[gi] * n, nbc);
        ops.push_back(o);
      }
      add_copy(op, ops, &P.copyHext, P.nm);
      add_gemm(op, {make_group(P.Bnz, (long long)nbp * mi, nbp, P.gt, (long long)NR * mi, mi, op->h[lev],
                               (long long)NR * nbp, nbp, nbp, NR, mi, 1.0, 1.0, nm, op->h[lev], (long long)NR * nbp,
                               nbp)},
               &P.gemmHp);
    }
    add_gemm(op, {make_group(P.S, (long long)mi * nbp, mi, op->g[lev], (long long)NR * nbp, nbp, P.gint,
                             (long long)NR * mi, mi, mi, NR, nbp, 1.0, 1.0, nm, P.gt, (long long)NR * mi, mi)},
             &P.gemmDown);
    {
      std::vector<BlockOp> ops;
      for (int c = 0; c < 4; ++c)
        for (int f = 0; f < 4; ++f) {
          BlockOp o = make_op(c * hstride_c + (long long)f * n, nbc, n, 0);
          if (G.group_of[c][f] >= 0) {
            op_src(o, 0, (long long)G.group_of[c][f] * n, nbp);
          } else {
            int k = 0;
            while (!(kItiUnk[k][0] == c && kItiUnk[k][1] == f)) ++k;
            op_src(o, 1, (long long)k * n, mi);
          }
          ops.push_back(o);
        }
      add_copy(op, ops, &P.copyGchild, P.nm);
    }
  }
  return finish_plan(op);
}

int run_build_iti(hps_op* op, const double* coeffs, hipStream_t st) {
  const int L = op->tree.depth;
  HPS_HIP_TRY(hipMemsetAsync(op->flag, 0, sizeof(int) * 4, st));
  stage_begin(op, "leaf_factor", st);
  HPS_TRY(iti_leaf_assemble_launch(coeffs, op->cst->D1, op->cst->D2, op->ic->Gr, op->ic->Ii, op->p, op->nl,
                                   op->Rbuf, op->Lbuf, st));
  HPS_TRY(run_gj(op, op->leaf_gj, st));
  stage_end(op, st);
  stage_begin(op, "leaf_T", st);
  HPS_TRY(run_gemm(op, op->gemmYleaf, st));
  HPS_TRY(run_gemm(op, op->gemmTleaf, st));
  stage_end(op, st);
  static const char* names[] = {"merge_l0", "merge_l1", "merge_l2", "merge_l3", "merge_l4", "merge_l5",
                                "merge_l6", "merge_l7", "merge_l8", "merge_l9", "merge_l10", "merge_l11"};
  for (int lev = L - 1; lev >= 0; --lev) {
    LevelPlan& P = op->levels[lev];
    const double* Tchild = lev == L - 1 ? op->Tleaf : op->levels[lev + 1].Tp;
    const long long cs = 4LL * P.nbc * P.nbc, w = 4LL * P.n, mi = P.m;
    stage_begin(op, names[lev < 12 ? lev : 11], st);
    HPS_TRY(run_copy(op, P.copyD, 0, P.D12, w * w, Tchild, cs, nullptr, 0, P.nm, st));
    HPS_TRY(run_copy(op, P.copyD21, 0, P.D21, w * w, Tchild, cs, nullptr, 0, P.nm, st));
    HPS_TRY(run_gemm(op, P.gemmW, st));
    HPS_TRY(run_gj(op, P.gj, st));
    HPS_TRY(run_copy(op, P.copyZ11, 0, P.Z, mi * mi, P.Winv, w * w, nullptr, 0, P.nm, st));
    HPS_TRY(run_gemm(op, P.gemmZ1, st));
    HPS_TRY(run_gemm(op, P.gemmZPP, st));
    HPS_TRY(run_copy(op, P.copyC, 0, P.Cm, mi * P.nbp, Tchild, cs, nullptr, 0, P.nm, st));
    HPS_TRY(run_gemm(op, P.gemmS, st));
    HPS_TRY(run_copy(op, P.copyB, 0, P.Bnz, (long long)P.nbp * mi, Tchild, cs, nullptr, 0, P.nm, st));
    if (P.Tp) {
      HPS_TRY(run_copy(op, P.fillT, 0, P.Tp, (long long)P.nbp * P.nbp, Tchild, cs, nullptr, 0, P.nm, st));
      HPS_TRY(run_gemm(op, P.gemmT, st));
    }
    stage_end(op, st);
  }
  return HPS_OK;
}

int run_solve_iti_chunk(hps_op* op, const double* bdry, const double* src, double* u, int nrhs, hipStream_t st) {
  const int L = op->tree.depth, NR = op->NR;
  stage_begin(op, "solve", st);
  HPS_TRY(run_copy(op, op->copyRoot, nrhs, op->g[0], 0, bdry, 0, nullptr, 0, 1, st));
  if (src) {
    HPS_TRY(iti_gather_src_launch(src, op->ic->Iir, op->Rbuf, op->ni, op->npts, op->nl, nrhs, NR, op->fint, st));
    HPS_TRY(run_gemm(op, op->gemmVleaf, st, nrhs));
    HPS_TRY(run_gemm(op, op->gemmHleaf, st, nrhs));
    for (int lev = L - 1; lev >= 0; --lev) {
      LevelPlan& P = op->levels[lev];
      HPS_TRY(run_copy(op, P.copyHint, nrhs, P.hint, (long long)NR * P.m, op->h[lev + 1], 4LL * NR * P.nbc, nullptr, 0,
                       P.nm, st));
      HPS_TRY(run_gemm(op, P.gemmGt, st, nrhs));
      if (lev > 0) {
        HPS_TRY(run_copy(op, P.copyHext, nrhs, op->h[lev], (long long)NR * P.nbp, op->h[lev + 1], 4LL * NR * P.nbc,
                         nullptr, 0, P.nm, st));
        HPS_TRY(run_gemm(op, P.gemmHp, st, nrhs));
      }
    }
  } else {
    for (int lev = 0; lev < L; ++lev) {
      LevelPlan& P = op->levels[lev];
      HPS_HIP_TRY(hipMemsetAsync(P.gt, 0, sizeof(double) * P.nm * NR * P.m, st));
    }
  }
  for (int lev = 0; lev < L; ++lev) {
    LevelPlan& P = op->levels[lev];
    HPS_TRY(run_gemm(op, P.gemmDown, st, nrhs));
    HPS_TRY(run_copy(op, P.copyGchild, nrhs, op->g[lev + 1], 4LL * NR * P.nbc, op->g[lev], (long long)NR * P.nbp,
                     P.gint, (long long)NR * P.m, P.nm, st));
  }
  HPS_TRY(run_gemm(op, src ? op->gemmUleaf : op->gemmUleaf0, st, nrhs));
  HPS_TRY(leaf_scatter_int_launch(op->uws, op->ic->ident, op->npts, op->npts, op->nl, nrhs, NR, u, st));
  stage_end(op, st);
  return HPS_OK;
}

// ---------------------------------------------------------------------------
// mixed-precision solve: fp32 operator copies + fp64 residual refinement
// ---------------------------------------------------------------------------
struct Map32 {
  struct E {
    const double* base;
    long long n;
    float* f;
  };
  std::vector<E> e;
  void add(const double* base, long long n, float* f) { e.push_back({base, n, f}); }
  const float* operator()(const double* p) const {
    if (!p) return nullptr;
    for (const E& x : e)
      if (p >= x.base && p < x.base + x.n) return x.f + (p - x.base);
    return nullptr;
  }
};

int to_group32(const GemmGroup& g, const Map32& m, GemmGroupF32* out) {
  GemmGroupF32 f;
  std::memset(&f, 0, sizeof(f));
  f.A = m(g.A);
  f.B = m(g.B);
  f.C = const_cast<float*>(m(g.C));
  f.C0 = g.C0 ? m(g.C0) : nullptr;
  if (!f.A || !f.B || !f.C || (g.C0 && !f.C0)) {
    set_error("internal: operand without an fp32 copy");
    return HPS_EINVAL;
  }
  f.sA = g.sA; f.sB = g.sB; f.sC = g.sC; f.sC0 = g.sC0;
  for (int k = 0; k < kMaxSeg; ++k) { f.aseg[k] = g.aseg[k]; f.bseg[k] = g.bseg[k]; }
  f.lda = g.lda; f.ldb = g.ldb; f.ldc = g.ldc; f.ldc0 = g.ldc0;
  f.M = g.M; f.N = g.N; f.K = g.K; f.nseg = g.nseg;
  f.alpha = (float)g.alpha; f.beta = (float)g.beta;
  f.batch = g.batch;
  f.ksplit = g.ksplit;
  f.kchunk = g.kchunk;
  f.part_off = g.part_off;
  f.part = nullptr;
  *out = f;
  return HPS_OK;
}

int add_gemm32(hps_op* op, const GemmCall& c, const Map32& m, GemmCall* out) {
  std::vector<GemmGroupF32> gs(c.count);
  for (int i = 0; i < c.count; ++i) HPS_TRY(to_group32(op->hgroups[c.first + i], m, &gs[i]));
  out->first = (int)op->hgroups32.size();
  out->count = c.count;
  out->nblocks = gemm_prepare_f32(gs);
  out->nrblocks = gemm_rblocks_f32(gs);
  out->ta = c.ta;
  out->tb = c.tb;
  op->hgroups32.insert(op->hgroups32.end(), gs.begin(), gs.end());
  return HPS_OK;
}

// fp32 copies of operators count as resident; solve workspaces do not (as for
// the fp64 solve's)
float* alloc32(hps_op* op, long long n, bool resident = true) {
  return (float*)op_alloc(op, sizeof(float) * std::max(1LL, n), resident);
}

// fp32 copies of the solve operators, fp32 / fp64 workspaces of the refined
// solve, the coefficient copy for the fp64 residual, leaf adjacency tables.
int setup_fp32(hps_op* op, const double* coeffs, hipStream_t st) {
  if (op->d != 2) { set_error("the mixed-precision solve supports 2D operators"); return HPS_EUNSUPPORTED; }
  const long long nl = op->nl;
  const int ni = op->ni, nb = op->nb, NR = op->NR, L = op->tree.depth, p = op->p, q = p - 2;
  const int nt = n_terms(op->d);
  op->coef = (double*)op_alloc(op, sizeof(double) * nl * nt * op->npts);
  op->LU32 = alloc32(op, nl * ni * ni);
  op->Y32 = alloc32(op, nl * ni * nb);
  op->Qi32 = alloc32(op, (long long)nb * ni);
  op->v32 = alloc32(op, nl * NR * ni, false);
  op->hx32 = alloc32(op, nl * NR * nb, false);
  op->gam = (double*)op_alloc(op, sizeof(double) * nl * NR * nb, false);
  op->r1 = (double*)op_alloc(op, sizeof(double) * nl * NR * ni, false);
  op->Qu = (double*)op_alloc(op, sizeof(double) * nl * NR * nb, false);
  op->C2G = (double*)op_alloc(op, sizeof(double) * q * p);
  op->nbr = (int*)op_alloc(op, sizeof(int) * nl * 4);
  op->bidx = (long long*)op_alloc(op, sizeof(long long) * nl * 4);
  if (!op->coef || !op->LU32 || !op->Y32 || !op->Qi32 || !op->v32 || !op->hx32 || !op->gam || !op->r1 || !op->Qu ||
      !op->C2G || !op->nbr || !op->bidx) {
    set_error("device allocation failed (mixed-precision copies)");
    return HPS_ENOMEM;
  }
  HPS_HIP_TRY(hipMemcpyAsync(op->coef, coeffs, sizeof(double) * nl * nt * op->npts, hipMemcpyDeviceToDevice, st));
  HPS_TRY(to_f32_launch(op->LU, op->LU32, nl * ni * ni, st));
  HPS_TRY(to_f32_launch(op->Y, op->Y32, nl * ni * nb, st));
  HPS_TRY(to_f32_launch(op->cst->Qi, op->Qi32, (long long)nb * ni, st));
  Map32 m;
  m.add(op->cst->Qi, (long long)nb * ni, op->Qi32);
  m.add(op->v, nl * NR * ni, op->v32);
  op->g32.assign(L + 1, nullptr);
  op->h32.assign(L + 1, nullptr);
  for (int l = 0; l <= L; ++l) {
    const long long n = (1LL << (2 * l)) * NR * op->nbl[l];
    op->g32[l] = alloc32(op, n, false);
    op->h32[l] = alloc32(op, n, false);
    if (!op->g32[l] || !op->h32[l]) { set_error("device allocation failed (fp32 workspace)"); return HPS_ENOMEM; }
    m.add(op->g[l], n, op->g32[l]);
    m.add(op->h[l], n, op->h32[l]);
  }
  for (auto& P : op->levels) {
    const long long nZ = P.nm * P.m * P.m, nS = P.nm * P.m * P.nbp, nB = P.nm * op->nd * P.dn * P.dn;
    const long long nw = P.nm * NR * P.m;
    P.Z32 = alloc32(op, nZ);
    P.S32 = alloc32(op, nS);
    P.Bnz32 = alloc32(op, nB);
    P.hint32 = alloc32(op, nw, false);
    P.gt32 = alloc32(op, nw, false);
    P.gint32 = alloc32(op, nw, false);
    if (!P.Z32 || !P.S32 || !P.Bnz32 || !P.hint32 || !P.gt32 || !P.gint32) {
      set_error("device allocation failed (fp32 merge copies)");
      return HPS_ENOMEM;
    }
    HPS_TRY(to_f32_launch(P.Z, P.Z32, nZ, st));
    HPS_TRY(to_f32_launch(P.S, P.S32, nS, st));
    HPS_TRY(to_f32_launch(P.Bnz, P.Bnz32, nB, st));
    m.add(P.Z, nZ, P.Z32);
    m.add(P.S, nS, P.S32);
    m.add(P.Bnz, nB, P.Bnz32);
    m.add(P.hint, nw, P.hint32);
    m.add(P.gt, nw, P.gt32);
    m.add(P.gint, nw, P.gint32);
  }
  // fp32 descriptor tables: the fp64 solve's groups with every operand mapped
  HPS_TRY(add_gemm32(op, op->gemmHleaf, m, &op->gemmHleaf32));
  {  // h = Q_i v + (flux imbalance handed to this leaf)
    GemmGroupF32& g = op->hgroups32[op->gemmHleaf32.first];
    g.beta = 1.0f;
    g.C0 = op->hx32;
    g.sC0 = (long long)NR * nb;
    g.ldc0 = nb;
  }
  for (auto& P : op->levels) {
    HPS_TRY(add_gemm32(op, P.gemmGt, m, &P.gemmGt32));
    if (P.lev > 0) HPS_TRY(add_gemm32(op, P.gemmHp, m, &P.gemmHp32));
    HPS_TRY(add_gemm32(op, P.gemmDown, m, &P.gemmDown32));
  }
  if (op->split_elems > 0) {
    op->splitws32 = alloc32(op, op->split_elems, false);
    if (!op->splitws32) { set_error("device allocation failed (split-K workspace)"); return HPS_ENOMEM; }
  }
  for (auto& g : op->hgroups32) g.part = g.ksplit > 1 ? op->splitws32 + g.part_off : nullptr;
  op->dgroups32 = (GemmGroupF32*)op_alloc(op, sizeof(GemmGroupF32) * std::max<size_t>(1, op->hgroups32.size()), false);
  if (!op->dgroups32) { set_error("device allocation failed (descriptors)"); return HPS_ENOMEM; }
  HPS_HIP_TRY(hipMemcpy(op->dgroups32, op->hgroups32.data(), sizeof(GemmGroupF32) * op->hgroups32.size(),
                        hipMemcpyHostToDevice));
  // host constants: Chebyshev -> Gauss interpolation, leaf adjacency
  const LeafOps& o = leaf_ops(op->d, p);
  HPS_HIP_TRY(hipMemcpy(op->C2G, o.C2G.data(), sizeof(double) * q * p, hipMemcpyHostToDevice));
  std::vector<int> nbr;
  std::vector<long long> bidx;
  leaf_face_tables(L, p, nbr, bidx);
  HPS_HIP_TRY(hipMemcpy(op->nbr, nbr.data(), sizeof(int) * nbr.size(), hipMemcpyHostToDevice));
  HPS_HIP_TRY(hipMemcpy(op->bidx, bidx.data(), sizeof(long long) * bidx.size(), hipMemcpyHostToDevice));
  op->fp32 = true;
  return HPS_OK;
}

// HPS_FLAG_FP32_ONLY: free the fp64 solve operators (leaf LU and Y, per
// level Z, S and B's blocks) after their fp32 copies were made; the refined
// solve reads only the copies, the pivot order and the coefficients.
int drop_fp64(hps_op* op) {
  HPS_HIP_TRY(hipStreamSynchronize(op->stream));
  std::vector<void*> drop = {op->LU, op->Y};
  for (auto& P : op->levels) {
    drop.push_back(P.Z);
    drop.push_back(P.S);
    drop.push_back(P.Bnz);
    P.Z = P.S = P.Bnz = nullptr;
  }
  op->LU = op->Y = nullptr;
  std::vector<Alloc> keep;
  for (const Alloc& al : op->allocs) {
    if (std::find(drop.begin(), drop.end(), al.p) != drop.end()) {
      op->resident -= round_size(al.bytes);
      op_dfree(al);
    } else {
      keep.push_back(al);
    }
  }
  op->allocs.swap(keep);
  op->static_ok = false;
  op->fp64_dropped = true;
  return HPS_OK;
}

int run_gemm32(hps_op* op, const GemmCall& c, hipStream_t st, int n_override) {
  return gemm_launch_f32(op->dgroups32 + c.first, c.count, c.nblocks, c.nrblocks, c.ta, c.tb, st, n_override);
}

int run_copy32(hps_op* op, const CopyCall& c, int ncols_rt, float* dst, long long dst_stride, const float* s0,
               long long s0_stride, const float* s1, long long s1_stride, long long batch, hipStream_t st) {
  return block_copy_launch_f32(op->dops, op->ditems, op->dtasks + c.first_task, c.ntasks, ncols_rt, dst, dst_stride,
                               s0, s0_stride, s1, s1_stride, batch, st);
}

// Iterative refinement on the composite collocation system: the iterate
// (gamma, u_int) is fp64, each correction is an fp32 HPS solve of the fp64
// residual (collocation rows as a source, flux-balance rows as an extra
// outgoing flux of the panel's lower-index leaf).
int run_solve_refined_chunk(hps_op* op, const double* bdry, const double* src, double* u, int nrhs, hipStream_t st) {
  const int L = op->tree.depth, nd = op->nd, NR = op->NR, p = op->p, q = p - 2;
  const long long nl = op->nl;
  stage_begin(op, "solve_refined", st);
  HPS_HIP_TRY(hipMemsetAsync(u, 0, sizeof(double) * nrhs * nl * op->npts, st));
  HPS_TRY(refine_init_launch(bdry, op->bidx, q, op->nbl[0], nl, nrhs, NR, op->gam, st));
  for (int sweep = 0; sweep <= op->refine_sweeps; ++sweep) {
    HPS_TRY(refine_residual_launch(op->coef, src, op->gam, op->cst->D1, op->cst->D2, op->cst->P, op->C2G, op->cst->Ii,
                                   op->cst->Ie, p, nl, nrhs, NR, u, op->r1, op->Qu, st));
    if (sweep == op->refine_sweeps) break;  // the last pass only completes u(I_e) = P gamma
    HPS_TRY(refine_flux_launch(op->Qu, op->nbr, q, nl, nrhs, NR, op->hx32, st));
    // fp32 correction solve with zero Dirichlet data
    HPS_TRY(leaf_src_f32_launch(op->LU32, op->perm, op->pos, op->r1, op->ni, nl, nrhs, NR, op->v32, st));
    HPS_TRY(run_gemm32(op, op->gemmHleaf32, st, nrhs));
    for (int lev = L - 1; lev >= 0; --lev) {
      LevelPlan& P = op->levels[lev];
      HPS_TRY(run_copy32(op, P.copyHint, nrhs, P.hint32, (long long)NR * P.m, op->h32[lev + 1],
                         (long long)nd * NR * P.nbc, nullptr, 0, P.nm, st));
      HPS_TRY(run_gemm32(op, P.gemmGt32, st, nrhs));
      if (lev > 0) HPS_TRY(run_gemm32(op, P.gemmHp32, st, nrhs));
    }
    HPS_HIP_TRY(hipMemsetAsync(op->g32[0], 0, sizeof(float) * NR * op->nbl[0], st));
    for (int lev = 0; lev < L; ++lev) {
      LevelPlan& P = op->levels[lev];
      HPS_TRY(run_gemm32(op, P.gemmDown32, st, nrhs));
      HPS_TRY(run_copy32(op, P.copyGchild, nrhs, op->g32[lev + 1], (long long)nd * NR * P.nbc, op->g32[lev],
                         (long long)NR * P.nbp, P.gint32, (long long)NR * P.m, P.nm, st));
    }
    HPS_TRY(refine_update_launch(op->g32[L], op->Y32, op->v32, op->cst->Ii, op->ni, op->nb, op->npts, nl, nrhs, NR,
                                 op->gam, u, st));
  }
  stage_end(op, st);
  return HPS_OK;
}

// After a queued build: synchronize, then check the pivots and the
// merge-inverse probes (see hps_level_info).  *retry is set when a
// block-eliminated inverse stayed inaccurate (or had a zero pivot inside a
// block) and pivoting over all of D can redo it.
int check_build(hps_op* op, bool* retry) {
  *retry = false;
  std::vector<double> status;
  HPS_TRY(download_status(op, &status));
  int hflag[4];
  std::memcpy(hflag, status.data(), sizeof(hflag));
  if (hflag[0]) {
    set_error(std::string("zero or non-finite pivot in ") +
              ((hflag[0] & 1) ? "a leaf factorization (L_ii)" : "a merge matrix D"));
    return HPS_ESINGULAR;
  }
  op->info_ready = false;
  HPS_TRY(collect_info(op, &status));
  int bad = -1;
  for (int lev = 0; lev < (int)op->info.size(); ++lev)
    if (op->info[lev].block_inverse && (hflag[1] || !(op->info[lev].residual <= kNsAccept))) bad = lev;
  if (bad < 0) return HPS_OK;
  bool full_ok = true;
  for (const auto& I : op->info) full_ok = full_ok && I.m <= 16384;
  if (full_ok) {
    *retry = true;
    return HPS_OK;
  }
  const hps_level_info_t& I = op->info[bad];
  char buf[256];
  std::snprintf(buf, sizeof(buf),
                "merge level %d node %lld: inverse of D (m = %d) by block elimination has probe residual "
                "%.2e after %d Newton-Schulz steps%s, and m exceeds the whole-D pivoting limit (16384)",
                bad, I.worst_node, I.m, I.residual, I.ns_steps, hflag[1] ? " (zero pivot in a block)" : "");
  set_error(buf);
  return HPS_ESINGULAR;
}

int check_tree(const hps_tree_t* t, int p) {
  if (!t) { set_error("tree is NULL"); return HPS_EINVAL; }
  if (t->dim != 2 && t->dim != 3) { set_error("dim must be 2 or 3"); return HPS_EINVAL; }
  if (t->depth < 1 || (t->dim == 2 && t->depth > 12) || (t->dim == 3 && t->depth > 5)) {
    set_error("depth out of range");
    return HPS_EINVAL;
  }
  if (!(t->hi > t->lo) || !std::isfinite(t->lo) || !std::isfinite(t->hi)) {
    set_error("domain must satisfy lo < hi");
    return HPS_EINVAL;
  }
  if (p < 4 || p > 16) { set_error("p must be in [4, 16]"); return HPS_EINVAL; }
  return HPS_OK;
}

}  // namespace

// helpers for the other host sources (adaptive.cpp)
void* op_alloc_x(hps_op* op, size_t bytes, bool resident) { return op_alloc(op, bytes, resident); }
int add_gemm_x(hps_op* op, std::vector<GemmGroup> groups, GemmCall* call) {
  return add_gemm(op, std::move(groups), call);
}
void add_copy_x(hps_op* op, const std::vector<BlockOp>& ops, CopyCall* call) { add_copy(op, ops, call); }
int run_gemm_x(hps_op* op, const GemmCall& c, hipStream_t st, int n_override) {
  if (c.count == 0) return HPS_OK;
  return run_gemm(op, c, st, n_override);
}
int run_copy_x(hps_op* op, const CopyCall& c, int ncols_rt, double* dst, const double* s0, const double* s1,
               hipStream_t st) {
  if (c.ntasks == 0) return HPS_OK;
  return run_copy(op, c, ncols_rt, dst, 0, s0, 0, s1, 0, 1, st);
}
int plan_gj_x(hps_op* op, GJPlan* g, double* A, double* Z, int m, long long batch) {
  return plan_gj(op, g, A, Z, m, batch, false);
}
int run_gj_x(hps_op* op, const GJPlan& g, hipStream_t st) { return run_gj(op, g, st); }
int get_consts_x(int d, int p, double r, DevConsts** out) { return get_consts(d, p, r, out); }
int finish_plan_x(hps_op* op) { return finish_plan(op); }
}  // namespace hps

using namespace hps;

extern "C" {

const char* hps_last_error(void) { return g_err.c_str(); }

int hps_sizes(const hps_tree_t* tree, int p, hps_sizes_t* out) {
  HPS_TRY(check_tree(tree, p));
  if (!out) { set_error("out is NULL"); return HPS_EINVAL; }
  const int d = tree->dim, q = p - 2;
  out->n_leaves = 1LL << (d * tree->depth);
  out->pts_per_leaf = d == 2 ? p * p : p * p * p;
  out->n_terms = n_terms(d);
  out->n_root_bdry = n_root_bdry(d, tree->depth, p);
  out->n_interior = d == 2 ? q * q : q * q * q;
  out->n_leaf_bdry = d == 2 ? 4 * q : 6 * q * q;
  out->n_levels = tree->depth;
  const long long nface = d == 2 ? (long long)q << (tree->depth - 1) : (long long)q * q << (2 * (tree->depth - 1));
  out->root_D = (d == 2 ? 4 : 12) * nface;
  return HPS_OK;
}

int hps_leaf_points(const hps_tree_t* tree, int p, double* xyz) {
  HPS_TRY(check_tree(tree, p));
  if (!xyz) { set_error("xyz is NULL"); return HPS_EINVAL; }
  leaf_points(tree->dim, tree->depth, tree->lo, tree->hi, p, xyz);
  return HPS_OK;
}

int hps_boundary_points(const hps_tree_t* tree, int p, double* xyz) {
  HPS_TRY(check_tree(tree, p));
  if (!xyz) { set_error("xyz is NULL"); return HPS_EINVAL; }
  boundary_points(tree->dim, tree->depth, tree->lo, tree->hi, p, xyz);
  return HPS_OK;
}

size_t hps_op_footprint(const hps_tree_t* tree, int p, int flags) {
  if (check_tree(tree, p) != HPS_OK) return 0;
  const int d = tree->dim, L = tree->depth, q = p - 2;
  const long long nl = 1LL << (d * L);
  const long long ni = d == 2 ? q * q : q * q * q, nb = d == 2 ? 4 * q : 6 * q * q;
  size_t bytes = (size_t)nl * (ni * ni + ni * nb) * 8 + (size_t)nl * ni * 8;  // LU, Y, perm+pos
  long long n = d == 2 ? q : q * q;
  for (int lev = L - 1; lev >= 0; --lev) {
    const long long nm = 1LL << (d * lev);
    const long long m = (d == 2 ? 4 : 12) * n, nbp = 2 * d * n * (1 << (d - 1)), dn = d * n;
    bytes += (size_t)nm * (m * m + m * nbp + (1 << d) * dn * dn) * 8;
    if (lev == 0 && (flags & HPS_FLAG_ROOT_T)) bytes += (size_t)nbp * nbp * 8;
    n *= (1 << (d - 1));
  }
  return bytes;
}

size_t hps_op_bytes(const hps_op_t* op) { return op ? op->resident + (op->sub ? op->sub->resident : 0) : 0; }

int hps_set_allocator(hps_alloc_fn alloc, hps_free_fn free, void* ctx) {
  if ((alloc == nullptr) != (free == nullptr)) {
    set_error("alloc and free must both be set or both be NULL");
    return HPS_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_pool_mu);
  g_cb_alloc = alloc;
  g_cb_free = free;
  g_cb_ctx = alloc ? ctx : nullptr;
  return HPS_OK;
}

void hps_mem_stats(size_t* in_use, size_t* peak, int reset_peak) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if (in_use) *in_use = g_in_use;
  if (peak) *peak = g_peak;
  if (reset_peak) g_peak = g_in_use;
}

int hps_level_info(hps_op_t* op, hps_level_info_t* out, int cap) {
  if (op && op->ad) { set_error("merge-level probe information is not kept for adaptive operators"); return -HPS_EUNSUPPORTED; }
  if (!op || (cap > 0 && !out)) { set_error("op must be non-NULL (and out when cap > 0)"); return -HPS_EINVAL; }
  if (op->iti) { set_error("ItI merges invert W with pivoting over all of W and run no probes"); return -HPS_EUNSUPPORTED; }
  const int rc = collect_info(op);
  if (rc != HPS_OK) return -rc;
  const int n = std::min(cap, (int)op->info.size());
  for (int i = 0; i < n; ++i) out[i] = op->info[i];
  return n;
}

int hps_build(const hps_tree_t* tree, int p, const double* coeffs, int flags, void* stream, hps_op_t** out) {
  if (out) *out = nullptr;
  HPS_TRY(check_tree(tree, p));
  if (!coeffs || !out) { set_error("coeffs and out must not be NULL"); return HPS_EINVAL; }
  hps_op* op = new hps_op();
  op->tree = *tree;
  op->p = p;
  op->d = tree->dim;
  op->nd = 1 << op->d;
  op->flags = flags;
  op->nl = 1LL << (op->d * tree->depth);
  const LeafOps& o = leaf_ops(op->d, p);
  op->npts = o.npts;
  op->ni = o.n_i;
  op->ne = o.n_e;
  op->nb = o.n_b;
  op->r = (tree->hi - tree->lo) / 2.0 / (double)(1LL << tree->depth);
  op->stream = (hipStream_t)stream;
  int rc = get_consts(op->d, p, op->r, &op->cst);
  if (rc == HPS_OK) rc = plan_op(op);
  if (rc == HPS_OK) rc = run_build(op, coeffs, op->stream);
  bool retry_full_pivot = false;
  if (rc == HPS_OK && !(flags & HPS_FLAG_NO_CHECK)) rc = check_build(op, &retry_full_pivot);
  if (retry_full_pivot) {
    // rare path: redo the whole build with partial pivoting over every D
    (void)hipStreamSynchronize(op->stream);
    hps_free(op);
    return hps_build(tree, p, coeffs, flags | HPS_FLAG_FULL_PIVOT, stream, out);
  }
  if (rc == HPS_OK && (flags & (HPS_FLAG_FP32_COPY | HPS_FLAG_FP32_ONLY))) rc = setup_fp32(op, coeffs, op->stream);
  if (rc == HPS_OK && (flags & HPS_FLAG_FP32_ONLY)) rc = drop_fp64(op);
  if (rc != HPS_OK) {
    if (rc != HPS_EDEVICE) (void)hipStreamSynchronize(op->stream);
    hps_free(op);
    return rc;
  }
  *out = op;
  return HPS_OK;
}

// The second stream of hps_build_solve, one per device, created at its first
// use and kept for the process (creating a queue per call costs more than the
// overlap gains).  It runs on every other CU: its long source-solve waves
// would otherwise hold every CU, and the build's products and chain steps
// beside them would wait for free ones.
static hipStream_t side_stream() {
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  auto it = streams.find(dev);
  if (it != streams.end()) return it->second;
  hipStream_t s = nullptr;
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu >= 16) {
    std::vector<uint32_t> mask((size_t)(ncu + 31) / 32, 0u);
    for (int cu = 0; cu < ncu; ++cu)
      if (cu % 2 == 0) mask[(size_t)cu / 32] |= 1u << (cu % 32);
    if (hipExtStreamCreateWithCUMask(&s, (uint32_t)mask.size(), mask.data()) != hipSuccess) {
      (void)hipGetLastError();
      s = nullptr;
    }
  }
  if (!s && hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
  streams[dev] = s;
  return s;
}

// the fork follows the last merge level with at least this many nodes: the
// root's children, so the leaf solves run beside the root merge, whose
// Gauss-Jordan chains leave most of the GPU idle (forks after the 16- and
// 64-node levels measured 0.25 ms slower)
constexpr long long kForkNodes = 4;
// the second stream's leaf solves keep at most this many workgroups on a CU:
// at full occupancy they fill its registers for their whole run, and the
// build's copies and products placed on that CU wait until they finish; the
// Gauss-Jordan kernels raise their waves' issue priority, so that the chain
// is not slowed by the leaf solves sharing its SIMDs (2 measured best; 4 slows
// the chain, 1 makes the leaf solves outlast the window)
constexpr int kSideWgPerCu = 2;

int hps_build_solve(const hps_tree_t* tree, int p, const double* coeffs, int flags, const double* bdry,
                    const double* src, double* u, int nrhs, void* stream, hps_op_t** out) {
  if (out) *out = nullptr;
  HPS_TRY(check_tree(tree, p));
  if (!coeffs || !out || !bdry || !u || nrhs < 1) {
    set_error("coeffs, bdry, u and out must be non-NULL and nrhs >= 1");
    return HPS_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  auto build_then_solve = [&](int fl) -> int {
    HPS_TRY(hps_build(tree, p, coeffs, fl, stream, out));
    const int rc = hps_solve(*out, bdry, src, u, nrhs, HPS_FP64, stream);
    if (rc != HPS_OK) {
      hps_free(*out);
      *out = nullptr;
    }
    return rc;
  };
  if (!src) return build_then_solve(flags);
  hipError_t pending = hipGetLastError();
  if (pending != hipSuccess) {
    set_error(std::string("earlier device error: ") + hipGetErrorString(pending));
    return HPS_EDEVICE;
  }
  hps_op* op = new hps_op();
  op->tree = *tree;
  op->p = p;
  op->d = tree->dim;
  op->nd = 1 << op->d;
  op->flags = flags;
  op->nl = 1LL << (op->d * tree->depth);
  const LeafOps& o = leaf_ops(op->d, p);
  op->npts = o.npts;
  op->ni = o.n_i;
  op->ne = o.n_e;
  op->nb = o.n_b;
  op->r = (tree->hi - tree->lo) / 2.0 / (double)(1LL << tree->depth);
  op->stream = st;
  int rc = get_consts(op->d, p, op->r, &op->cst);
  if (rc == HPS_OK) rc = plan_op(op);
  if (rc != HPS_OK) {
    hps_free(op);
    return rc;
  }
  const int L = op->tree.depth, k = std::min(op->NR, nrhs);
  // The source's leaf part (and the upward pass through the levels already
  // built) goes to a second stream once the build has passed the last level
  // with at least kForkNodes nodes: the levels above it are Gauss-Jordan
  // chains on a few large matrices that leave most of the GPU idle.  Only products that
  // do not split K (the split-K workspace is shared) go there.
  int fork = L;
  for (int lev = L - 1; lev >= 0; --lev)
    if (op->levels[lev].nm >= kForkNodes) fork = lev;
  // the side stream's upward pass covers levels up_lo .. L - 1: the built
  // levels from the leaves up to the first one whose products split K
  bool overlap = op->gemmHleaf.nrblocks == 0 && (op->d == 2 || op->gemmVleaf.nrblocks == 0);
  int up_lo = L;
  while (up_lo > fork && op->levels[up_lo - 1].gemmGt.nrblocks == 0 && op->levels[up_lo - 1].gemmHp.nrblocks == 0)
    --up_lo;
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, side_ev = nullptr;
  if (overlap) {
    side = side_stream();
    if (!side || hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&side_ev, hipEventDisableTiming) != hipSuccess)
      overlap = false;
  }
  const SolveCtx c = own_ctx(op);
  bool forked = false;
  std::function<int(int)> after = [&](int lev) -> int {
    if (!overlap || lev != fork) return HPS_OK;
    HPS_HIP_TRY(hipEventRecord(fork_ev, st));
    HPS_HIP_TRY(hipStreamWaitEvent(side, fork_ev, 0));
    HPS_TRY(run_solve_leaf_src(op, c, src, k, side, kSideWgPerCu));
    if (up_lo < L) HPS_TRY(run_solve_levels_up(op, c, L - 1, up_lo, k, side));
    HPS_HIP_TRY(hipEventRecord(side_ev, side));
    forked = true;
    return HPS_OK;
  };
  rc = run_build(op, coeffs, st, true, &after);
  if (rc == HPS_OK) {
    if (forked) {
      if (hipStreamWaitEvent(st, side_ev, 0) != hipSuccess) { set_error("stream wait failed"); rc = HPS_EDEVICE; }
      if (rc == HPS_OK) rc = run_copy(op, op->copyRoot, k, c.at(op->g[0]), 0, bdry, 0, nullptr, 0, 1, st);
      if (rc == HPS_OK && up_lo > 0) rc = run_solve_levels_up(op, c, up_lo - 1, 0, k, st);
      if (rc == HPS_OK) rc = run_solve_down(op, c, true, u, k, st);
    } else {
      rc = run_solve_chunk(op, c, bdry, src, u, k, false, st);
    }
  }
  if (side) (void)hipStreamSynchronize(side);
  if (fork_ev) (void)hipEventDestroy(fork_ev);
  if (side_ev) (void)hipEventDestroy(side_ev);
  bool retry_full_pivot = false;
  if (rc == HPS_OK && !(flags & HPS_FLAG_NO_CHECK)) rc = check_build(op, &retry_full_pivot);
  if (retry_full_pivot) {
    (void)hipStreamSynchronize(st);
    hps_free(op);
    return build_then_solve(flags | HPS_FLAG_FULL_PIVOT);
  }
  const long long nbr = op->nbl[0], field = op->nl * op->npts;
  for (int r0 = k; rc == HPS_OK && r0 < nrhs; r0 += op->NR) {
    const int kk = std::min(op->NR, nrhs - r0);
    rc = run_solve_chunk(op, c, bdry + r0 * nbr, src + r0 * field, u + r0 * field, kk, false, st);
  }
  if (rc == HPS_OK && (flags & (HPS_FLAG_FP32_COPY | HPS_FLAG_FP32_ONLY))) rc = setup_fp32(op, coeffs, st);
  if (rc == HPS_OK && (flags & HPS_FLAG_FP32_ONLY)) rc = drop_fp64(op);
  if (rc != HPS_OK) {
    if (rc != HPS_EDEVICE) (void)hipStreamSynchronize(st);
    hps_free(op);
    return rc;
  }
  *out = op;
  return HPS_OK;
}

int hps_build_subtrees(const hps_tree_t* tree, int p, const double* coeffs, int flags, int subtree_depth,
                       void* stream, hps_op_t** out) {
  if (out) *out = nullptr;
  HPS_TRY(check_tree(tree, p));
  if (!coeffs || !out) { set_error("coeffs and out must not be NULL"); return HPS_EINVAL; }
  if (tree->dim != 2) { set_error("subtree recomputation is implemented for 2D trees"); return HPS_EUNSUPPORTED; }
  if (subtree_depth < 1 || subtree_depth >= tree->depth) {
    set_error("subtree_depth must satisfy 1 <= subtree_depth < depth");
    return HPS_EINVAL;
  }
  if (flags & (HPS_FLAG_FP32_COPY | HPS_FLAG_FP32_ONLY | HPS_FLAG_ROOT_T)) {
    set_error("HPS_FLAG_FP32_COPY and HPS_FLAG_ROOT_T are not available with subtree recomputation");
    return HPS_EUNSUPPORTED;
  }
  const int Ls = subtree_depth, Lt = tree->depth - Ls;
  const LeafOps& o = leaf_ops(2, p);
  hipStream_t st = (hipStream_t)stream;
  const int keep = flags & (HPS_FLAG_FULL_PIVOT | HPS_FLAG_TEST_NO_REFINE);
  // one subtree's plan: a depth-Ls tree over the subtree's box (every subtree
  // has the same leaf size, so the plan serves all of them), with its root T
  // and its root's outgoing source flux
  hps_op* sub = new hps_op();
  sub->tree = *tree;
  sub->tree.depth = Ls;
  sub->tree.hi = tree->lo + (tree->hi - tree->lo) / (double)(1LL << Lt);
  sub->p = p;
  sub->d = 2;
  sub->nd = 4;
  sub->flags = keep | HPS_FLAG_ROOT_T;
  sub->nl = 1LL << (2 * Ls);
  sub->npts = o.npts;
  sub->ni = o.n_i;
  sub->ne = o.n_e;
  sub->nb = o.n_b;
  sub->r = (tree->hi - tree->lo) / 2.0 / (double)(1LL << tree->depth);
  sub->stream = st;
  sub->root_h = true;
  sub->rstride = (1LL << (2 * tree->depth)) * o.npts;
  int rc = get_consts(2, p, sub->r, &sub->cst);
  if (rc == HPS_OK) rc = plan_op(sub);
  if (rc != HPS_OK) { hps_free(sub); return rc; }
  // the top levels: leaves are the subtree roots
  hps_op* top = new hps_op();
  top->tree = *tree;
  top->tree.depth = Lt;
  top->p = p;
  top->d = 2;
  top->nd = 4;
  top->flags = keep | (flags & HPS_FLAG_TIMING);
  top->nl = 1LL << (2 * Lt);
  top->ext_side = (p - 2) << Ls;
  top->nb = 4 * top->ext_side;
  top->r = sub->r;
  top->stream = st;
  top->sub = sub;
  top->full_depth = tree->depth;
  rc = plan_op(top);
  const long long ncoef = (1LL << (2 * tree->depth)) * 6 * o.npts;
  if (rc == HPS_OK) {
    top->sub_coef = (double*)op_alloc(top, sizeof(double) * ncoef);
    if (!top->sub_coef) { set_error("device allocation failed (coefficient copy)"); rc = HPS_ENOMEM; }
  }
  if (rc == HPS_OK) {
    const hipError_t e = hipMemcpyAsync(top->sub_coef, coeffs, sizeof(double) * ncoef, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) { set_error(std::string("coefficient copy failed: ") + hipGetErrorString(e)); rc = HPS_EDEVICE; }
  }
  const bool check = !(flags & HPS_FLAG_NO_CHECK);
  bool retry = false;
  const long long coef_stride = sub->nl * 6 * o.npts, nbs = top->nb;
  for (long long j = 0; rc == HPS_OK && !retry && j < top->nl; ++j) {
    rc = run_build(sub, top->sub_coef + j * coef_stride, st);
    if (rc == HPS_OK) {
      const hipError_t e = hipMemcpyAsync(top->Tleaf + j * nbs * nbs, sub->levels[0].Tp, sizeof(double) * nbs * nbs,
                                          hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) { set_error(std::string("subtree copy failed: ") + hipGetErrorString(e)); rc = HPS_EDEVICE; }
    }
    if (rc == HPS_OK && check) rc = check_build(sub, &retry);
  }
  if (rc == HPS_OK && !retry) rc = run_build(top, nullptr, st);
  if (rc == HPS_OK && !retry && check) rc = check_build(top, &retry);
  if (rc == HPS_OK && retry) {
    hps_free(top);
    return hps_build_subtrees(tree, p, coeffs, flags | HPS_FLAG_FULL_PIVOT, subtree_depth, stream, out);
  }
  if (rc != HPS_OK) {
    if (rc != HPS_EDEVICE) (void)hipStreamSynchronize(st);
    hps_free(top);
    return rc;
  }
  *out = top;
  return HPS_OK;
}

int hps_build_iti(const hps_tree_t* tree, int p, double eta, const double* coeffs, int flags, void* stream,
                  hps_op_t** out) {
  if (out) *out = nullptr;
  HPS_TRY(check_tree(tree, p));
  if (!coeffs || !out) { set_error("coeffs and out must not be NULL"); return HPS_EINVAL; }
  if (tree->dim != 2) { set_error("the ItI variant is implemented for 2D trees"); return HPS_EUNSUPPORTED; }
  if (!(eta > 0.0) || !std::isfinite(eta)) { set_error("eta must be positive and finite"); return HPS_EINVAL; }
  if (flags & (HPS_FLAG_FP32_COPY | HPS_FLAG_FP32_ONLY | HPS_FLAG_ROOT_T)) {
    set_error("HPS_FLAG_FP32_COPY and HPS_FLAG_ROOT_T are not available for the ItI variant");
    return HPS_EUNSUPPORTED;
  }
  hps_op* op = new hps_op();
  op->tree = *tree;
  op->p = p;
  op->d = 2;
  op->nd = 4;
  op->flags = flags & (HPS_FLAG_NO_CHECK | HPS_FLAG_TIMING);
  op->nl = 1LL << (2 * tree->depth);
  op->npts = 2 * p * p;
  op->ni = 2 * (p - 2) * (p - 2);
  op->ne = 2 * (4 * p - 4);
  op->nb = 2 * 4 * (p - 2);
  op->r = (tree->hi - tree->lo) / 2.0 / (double)(1LL << tree->depth);
  op->stream = (hipStream_t)stream;
  op->iti = true;
  op->eta = eta;
  int rc = get_consts(2, p, op->r, &op->cst);
  if (rc == HPS_OK) rc = get_iti_consts(p, op->r, eta, &op->ic);
  if (rc == HPS_OK) rc = plan_iti(op);
  if (rc == HPS_OK) rc = run_build_iti(op, coeffs, op->stream);
  if (rc == HPS_OK && !(flags & HPS_FLAG_NO_CHECK)) {
    int hflag[4] = {0, 0, 0, 0};
    hipError_t e = hipMemcpyAsync(hflag, op->flag, sizeof(hflag), hipMemcpyDeviceToHost, op->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(op->stream);
    if (e != hipSuccess) {
      set_error(std::string("build failed on the device: ") + hipGetErrorString(e));
      rc = HPS_EDEVICE;
    } else if (hflag[0] || hflag[1]) {
      set_error("zero or non-finite pivot in an ItI leaf matrix B or a merge matrix W");
      rc = HPS_ESINGULAR;
    }
  }
  if (rc != HPS_OK) {
    if (rc != HPS_EDEVICE) (void)hipStreamSynchronize(op->stream);
    hps_free(op);
    return rc;
  }
  *out = op;
  return HPS_OK;
}

int hps_solve(hps_op_t* op, const double* bdry, const double* src, double* u, int nrhs, int precision, void* stream) {
  if (!op || !bdry || !u || nrhs < 1) { set_error("op, bdry, u must be non-NULL and nrhs >= 1"); return HPS_EINVAL; }
  if (precision != HPS_FP64 && precision != HPS_FP32_REFINED) { set_error("unknown precision"); return HPS_EINVAL; }
  if (precision == HPS_FP32_REFINED && !op->fp32) {
    set_error("HPS_FP32_REFINED needs an operator built with HPS_FLAG_FP32_COPY");
    return HPS_EINVAL;
  }
  if (precision == HPS_FP64 && op->fp64_dropped) {
    set_error("the fp64 operators were freed (HPS_FLAG_FP32_ONLY): solve with HPS_FP32_REFINED");
    return HPS_EUNSUPPORTED;
  }
  hipError_t pending = hipGetLastError();
  if (pending != hipSuccess) {
    set_error(std::string("earlier device error: ") + hipGetErrorString(pending));
    return HPS_EDEVICE;
  }
  hipStream_t st = (hipStream_t)stream;
  clear_stages(op);
  if (op->ad) {
    if (precision != HPS_FP64) { set_error("adaptive operators solve in fp64"); return HPS_EUNSUPPORTED; }
    return adaptive_solve(op, bdry, src, u, nrhs, st);
  }
  if (op->iti) {
    const long long nbr = op->nbl[0], field = op->nl * op->npts;
    for (int r0 = 0; r0 < nrhs; r0 += op->NR) {
      const int k = std::min(op->NR, nrhs - r0);
      HPS_TRY(run_solve_iti_chunk(op, bdry + r0 * nbr, src ? src + r0 * field : nullptr, u + r0 * field, k, st));
    }
    return HPS_OK;
  }
  if (op->sub) {
    const long long nbr = op->nbl[0], field = op->sub->rstride;
    for (int r0 = 0; r0 < nrhs; r0 += op->NR) {
      const int k = std::min(op->NR, nrhs - r0);
      HPS_TRY(run_solve_subtrees(op, bdry + r0 * nbr, src ? src + r0 * field : nullptr, u + r0 * field, k, st));
    }
    return HPS_OK;
  }
  const long long nbr = op->nbl[0], field = op->nl * op->npts;
  for (int r0 = 0; r0 < nrhs; r0 += op->NR) {
    const int k = std::min(op->NR, nrhs - r0);
    if (precision == HPS_FP32_REFINED)
      HPS_TRY(run_solve_refined_chunk(op, bdry + r0 * nbr, src ? src + r0 * field : nullptr, u + r0 * field, k, st));
    else
      HPS_TRY(run_solve_chunk(op, own_ctx(op), bdry + r0 * nbr, src ? src + r0 * field : nullptr, u + r0 * field, k,
                              false, st));
  }
  return HPS_OK;
}

int hps_solve_noalloc(hps_op_t* op, const double* bdry, const double* src, double* u, int nrhs, void* stream) {
  if (op && op->ad) { set_error("the allocation-free solve serves fp64 DtN operators built by hps_build"); return HPS_EUNSUPPORTED; }
  if (!op || !bdry || !u || nrhs < 1) { set_error("op, bdry, u must be non-NULL and nrhs >= 1"); return HPS_EINVAL; }
  if (op->sub || op->iti || op->fp64_dropped) {
    set_error("the allocation-free solve serves fp64 DtN operators built by hps_build");
    return HPS_EUNSUPPORTED;
  }
  if (!op->static_ok) {
    char buf[200];
    std::snprintf(buf, sizeof(buf),
                  "solve workspace of this operator (%.1f MiB) exceeds the static workspace (%.1f MiB)",
                  (double)op->static_need / 1048576.0, (double)HPS_STATIC_WS_BYTES / 1048576.0);
    set_error(buf);
    return HPS_EINVAL;
  }
  hipError_t pending = hipGetLastError();
  if (pending != hipSuccess) {
    set_error(std::string("earlier device error: ") + hipGetErrorString(pending));
    return HPS_EDEVICE;
  }
  hipStream_t st = (hipStream_t)stream;
  const SolveCtx c{op, op->dgroups_static, op->static_base};
  const long long nbr = op->nbl[0], field = op->nl * op->npts;
  for (int r0 = 0; r0 < nrhs; r0 += op->NR) {
    const int k = std::min(op->NR, nrhs - r0);
    HPS_TRY(run_solve_chunk(op, c, bdry + r0 * nbr, src ? src + r0 * field : nullptr, u + r0 * field, k, true, st));
  }
  return HPS_OK;
}

int hps_refine_sweeps(hps_op_t* op, int sweeps) {
  if (op && op->ad) { set_error("adaptive operators have no mixed-precision solve"); return -HPS_EUNSUPPORTED; }
  if (!op || sweeps < 0 || sweeps > 64) { set_error("op must be non-NULL and 0 <= sweeps <= 64"); return -HPS_EINVAL; }
  const int old = op->refine_sweeps;
  if (sweeps > 0) op->refine_sweeps = sweeps;
  return old;
}

int hps_solve_adjoint(hps_op_t* op, const double* w, double* lam_src, double* lam_bdry, int nrhs, void* stream) {
  if (op && op->ad) { set_error("the adjoint solve is not available for adaptive operators"); return HPS_EUNSUPPORTED; }
  if (!op || !w || !lam_src || nrhs < 1) { set_error("op, w, lam_src must be non-NULL and nrhs >= 1"); return HPS_EINVAL; }
  if (op->iti) { set_error("the adjoint solve is not available for the ItI variant"); return HPS_EUNSUPPORTED; }
  if (op->fp64_dropped) { set_error("the adjoint solve needs the fp64 operators (freed by HPS_FLAG_FP32_ONLY)"); return HPS_EUNSUPPORTED; }
  hipError_t pending = hipGetLastError();
  if (pending != hipSuccess) {
    set_error(std::string("earlier device error: ") + hipGetErrorString(pending));
    return HPS_EDEVICE;
  }
  hipStream_t st = (hipStream_t)stream;
  clear_stages(op);
  const long long nbr = op->nbl[0], field = op->nl * op->npts, sfield = op->sub ? op->sub->rstride : 0;
  for (int r0 = 0; r0 < nrhs; r0 += op->NR) {
    const int k = std::min(op->NR, nrhs - r0);
    if (op->sub)
      HPS_TRY(run_adjoint_subtrees(op, w + r0 * sfield, lam_src + r0 * sfield, lam_bdry ? lam_bdry + r0 * nbr : nullptr,
                                   k, st));
    else
      HPS_TRY(run_adjoint_chunk(op, w + r0 * field, lam_src + r0 * field, lam_bdry ? lam_bdry + r0 * nbr : nullptr, k,
                                st));
  }
  return HPS_OK;
}

int hps_coeff_grad(hps_op_t* op, const double* u, const double* lam, int nrhs, double* grad, void* stream) {
  if (op && op->ad) { set_error("the coefficient gradient is not available for adaptive operators"); return HPS_EUNSUPPORTED; }
  if (!op || !u || !lam || !grad || nrhs < 1) {
    set_error("op, u, lam, grad must be non-NULL and nrhs >= 1");
    return HPS_EINVAL;
  }
  if (op->iti) { set_error("the coefficient gradient is not available for the ItI variant"); return HPS_EUNSUPPORTED; }
  // the gradient needs only the leaf differentiation matrices (the same for
  // every leaf of the tree, so a subtree plan's serve for all leaves)
  const hps_op* lo = op->sub ? op->sub : op;
  const long long nl = op->sub ? op->sub->rstride / op->sub->npts : op->nl;
  return coeff_grad_launch(op->d, op->p, u, lam, lo->cst->D1, lo->cst->D2, nl, nrhs, grad, (hipStream_t)stream);
}

int hps_interp_weights(const hps_tree_t* tree, int p, const double* x, long long m, long long* leaf, double* w) {
  HPS_TRY(check_tree(tree, p));
  if (m < 0 || (m > 0 && (!x || !leaf || !w))) { set_error("x, leaf, w must be non-NULL and m >= 0"); return HPS_EINVAL; }
  if (interp_weights(tree->dim, tree->depth, tree->lo, tree->hi, p, x, m, leaf, w) != 0) {
    set_error("a point lies outside the domain");
    return HPS_EINVAL;
  }
  return HPS_OK;
}

int hps_stage_times(hps_op_t* op, const char** names, double* ms, int cap) {
  if (!op) { set_error("op is NULL"); return -HPS_EINVAL; }
  int n = 0;
  for (auto& s : op->stages) {
    if (n >= cap) break;
    if (hipEventSynchronize(s.b) != hipSuccess) { set_error("event sync failed"); return -HPS_EDEVICE; }
    float t = 0.f;
    if (hipEventElapsedTime(&t, s.a, s.b) != hipSuccess) t = -1.f;
    if (names) names[n] = s.name;
    if (ms) ms[n] = t;
    ++n;
  }
  return n;
}

void hps_free(hps_op_t* op) {
  if (!op) return;
  // solves, adjoint solves and batches may have used the operator on any
  // stream: wait for all queued device work before its memory is recycled
  (void)hipDeviceSynchronize();
  clear_stages(op);
  if (op->sub) hps_free(op->sub);
  if (op->ad) adaptive_free(op->ad);
  for (auto& a : op->allocs) op_dfree(a);
  delete op;
}

int hps_debug_gemm_f32(int m, int n, int k, float alpha, const float* a, int lda, int trans_a, const float* b,
                       int ldb, int trans_b, float beta, float* c, int ldc, void* stream) {
  if (m < 0 || n < 0 || k < 0 || !a || !b || !c) { set_error("bad GEMM arguments"); return HPS_EINVAL; }
  GemmGroupF32 g;
  std::memset(&g, 0, sizeof(g));
  g.A = a; g.B = b; g.C = c; g.C0 = c;
  g.lda = lda; g.ldb = ldb; g.ldc = ldc; g.ldc0 = ldc;
  g.M = m; g.N = n; g.K = k; g.nseg = 1;
  g.alpha = alpha; g.beta = beta; g.batch = 1;
  std::vector<GemmGroupF32> gs = {g};
  const long long ws = gemm_plan_split_f32(gs);
  const long long nblocks = gemm_prepare_f32(gs);
  const long long nrblocks = gemm_rblocks_f32(gs);
  GemmGroupF32* dg = nullptr;
  float* part = nullptr;
  HPS_HIP_TRY(hipMalloc(&dg, sizeof(GemmGroupF32)));
  if (ws > 0 && hipMalloc(&part, sizeof(float) * ws) != hipSuccess) {
    (void)hipFree(dg);
    set_error("device allocation failed");
    return HPS_ENOMEM;
  }
  if (gs[0].ksplit > 1) gs[0].part = part + gs[0].part_off;
  hipStream_t st = (hipStream_t)stream;
  int rc = HPS_OK;
  if (hipMemcpyAsync(dg, gs.data(), sizeof(GemmGroupF32), hipMemcpyHostToDevice, st) != hipSuccess) rc = HPS_EDEVICE;
  if (rc == HPS_OK) rc = gemm_launch_f32(dg, 1, nblocks, nrblocks, trans_a != 0, trans_b != 0, st, n);
  (void)hipStreamSynchronize(st);
  (void)hipFree(dg);
  if (part) (void)hipFree(part);
  return rc;
}

int hps_debug_gemm(int m, int n, int k, double alpha, const double* a, int lda, int trans_a, const double* b, int ldb,
                   int trans_b, double beta, double* c, int ldc, void* stream) {
  if (m < 0 || n < 0 || k < 0 || !a || !b || !c) { set_error("bad GEMM arguments"); return HPS_EINVAL; }
  std::vector<GemmGroup> gs = {make_group(a, 0, lda, b, 0, ldb, c, 0, ldc, m, n, k, alpha, beta, 1, c, 0, ldc)};
  const long long ws = gemm_plan_split(gs);
  const long long nblocks = gemm_prepare(gs);
  const long long nrblocks = gemm_rblocks(gs);
  GemmGroup* dg = nullptr;
  double* part = nullptr;
  HPS_HIP_TRY(hipMalloc(&dg, sizeof(GemmGroup)));
  if (ws > 0 && hipMalloc(&part, sizeof(double) * ws) != hipSuccess) {
    (void)hipFree(dg);
    set_error("device allocation failed");
    return HPS_ENOMEM;
  }
  if (gs[0].ksplit > 1) gs[0].part = part + gs[0].part_off;
  hipStream_t st = (hipStream_t)stream;
  int rc = HPS_OK;
  if (hipMemcpyAsync(dg, gs.data(), sizeof(GemmGroup), hipMemcpyHostToDevice, st) != hipSuccess) rc = HPS_EDEVICE;
  if (rc == HPS_OK) rc = gemm_launch(dg, 1, nblocks, nrblocks, trans_a != 0, trans_b != 0, st, n);
  (void)hipStreamSynchronize(st);
  (void)hipFree(dg);
  if (part) (void)hipFree(part);
  return rc;
}

long long hps_debug_download(const hps_op_t* op, int which, int level, double* out, long long cap) {
  if (op && op->ad) { set_error("internal buffers of adaptive operators are not exposed"); return -HPS_EUNSUPPORTED; }
  if (!op || !out) { set_error("op and out must not be NULL"); return -HPS_EINVAL; }
  if (hipStreamSynchronize(op->stream) != hipSuccess) { set_error("stream sync failed"); return -HPS_EDEVICE; }
  const void* src = nullptr;
  long long n = 0;
  bool ints = false;
  const int L = op->tree.depth;
  if (which >= 4 && (level < 0 || level >= L)) { set_error("level out of range"); return -HPS_EINVAL; }
  switch (which) {
    case 0: src = op->LU; n = op->iti ? op->nl * op->npts * op->npts : op->nl * op->ni * op->ni; break;
    case 1: src = op->perm; n = op->nl * op->ni; ints = true; break;
    case 2: src = op->Y; n = op->iti ? op->nl * op->npts * op->nb : op->nl * op->ni * op->nb; break;
    case 3: src = op->Tleaf; n = op->nl * op->nb * op->nb; break;
    case 4: src = op->levels[level].Z; n = op->levels[level].nm * op->levels[level].m * op->levels[level].m; break;
    case 5: src = op->levels[level].S; n = op->levels[level].nm * op->levels[level].m * op->levels[level].nbp; break;
    case 6:
      src = op->levels[level].Tp;
      n = op->levels[level].nm * op->levels[level].nbp * op->levels[level].nbp;
      break;
    default: set_error("unknown buffer id"); return -HPS_EINVAL;
  }
  if (!src) { set_error("buffer not formed"); return -HPS_EINVAL; }
  if (n > cap) { set_error("output capacity too small"); return -HPS_EINVAL; }
  if (ints) {
    std::vector<int> tmp(n);
    if (hipMemcpy(tmp.data(), src, n * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return -HPS_EDEVICE;
    for (long long i = 0; i < n; ++i) out[i] = tmp[i];
  } else if (hipMemcpy(out, src, n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
    set_error("copy failed");
    return -HPS_EDEVICE;
  }
  return n;
}

int hps_precompute_matrix(int dim, int p, int which, double* out, long long cap, int* rows, int* cols) {
  if ((dim != 2 && dim != 3) || p < 4 || p > 16 || !out || !rows || !cols) {
    set_error("bad arguments");
    return HPS_EINVAL;
  }
  const LeafOps& o = leaf_ops(dim, p);
  std::vector<double> v;
  int r = 0, c = 0;
  switch (which) {
    case 0: v = o.cheb; r = 1; c = p; break;
    case 1: v = o.gl; r = 1; c = o.q; break;
    case 2: v = o.glw; r = 1; c = o.q; break;
    case 3: v = o.D; r = p; c = p; break;
    case 4: v = o.P; r = o.n_e; c = o.n_b; break;
    case 5: v = o.Qref; r = o.n_b; c = o.npts; break;
    case 6: v.assign(o.Ii.begin(), o.Ii.end()); r = 1; c = o.n_i; break;
    case 7: v.assign(o.Ie.begin(), o.Ie.end()); r = 1; c = o.n_e; break;
    default: set_error("unknown matrix id"); return HPS_EINVAL;
  }
  if ((long long)v.size() > cap) { set_error("output capacity too small"); return HPS_EINVAL; }
  std::memcpy(out, v.data(), v.size() * sizeof(double));
  *rows = r;
  *cols = c;
  return HPS_OK;
}

}  // extern "C"
