// Internal definitions shared by the host sources of the library: the
// operator record and the launch plans its build and solve replay.
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <vector>

#include "../../include/hps.h"
#include "common.hpp"

#define HPS_TRY(expr)              \
  do {                             \
    int _rc = (expr);              \
    if (_rc != HPS_OK) return _rc; \
  } while (0)

namespace hps {

// Per-(dim, p, leaf size) constants resident on the device.
struct DevConsts {
  double *D1 = nullptr, *D2 = nullptr, *Mt = nullptr, *QeP = nullptr, *Qi = nullptr, *P = nullptr;
  int *Ii = nullptr, *Ie = nullptr, *PosI = nullptr;
};

// Per-(p, leaf size, eta) constants of the ItI variant, in the real
// representation of complex matrices (see iti.hip): Robin rows G
// (2(4p-4) x 2p^2), P (2(4p-4) x 8q), Q H (8q x 2p^2), all column-major;
// interior points Ii, their real indices Iir (2 per point) and the identity
// index list of a leaf's 2p^2 reals.
struct ItiConsts {
  double *Gr = nullptr, *Pr = nullptr, *QHr = nullptr;
  int *Ii = nullptr, *Iir = nullptr, *ident = nullptr;
};

struct GemmCall {
  int first = 0, count = 0;
  long long nblocks = 0, nrblocks = 0;  // GEMM and split-K reduction workgroups
  bool ta = false, tb = false;
};
struct CopyCall {
  int first_task = 0, ntasks = 0;
};

// Batched inversion of m x m matrices held in `A` (overwritten) into `Z`.
struct GJPlan {
  int m = 0;
  long long batch = 0;
  double *A = nullptr, *Z = nullptr;
  int* flag = nullptr;  // pivot failure flag the kernels set
  bool small = true;
  int nb = 0;
  int *pos = nullptr, *piv = nullptr;
  double* W = nullptr;
  // two-level form (large m): column blocks of ob columns, the inner panels
  // update only their block, then one GEMM pair per block updates the rest
  int ob = 0;
  double *Wk = nullptr, *Pk = nullptr;
  std::vector<GemmCall> blk;
};

struct LevelPlan {
  int lev = 0;
  long long nm = 0;
  int n = 0, m = 0, nbc = 0, nbp = 0, dn = 0;
  double *Z = nullptr, *S = nullptr, *Bnz = nullptr, *Tp = nullptr, *Dbuf = nullptr;
  GJPlan gj;
  CopyCall copyD, fillT, copyB;
  GemmCall gemmS, gemmT;
  // solve
  double *hint = nullptr, *gt = nullptr, *gint = nullptr;
  CopyCall copyHint, copyGchild;
  GemmCall gemmGt, gemmHp, gemmDown;
  // adjoint
  CopyCall copyPext;
  GemmCall gemmSt, gemmBt1, gemmBt2, gemmZt;
  // block inversion of D for large merges: interfaces ordered [P1 | P2 | R]
  // with D(P1, P2) = 0; sizes s = |P_b| n, r = |R| n
  bool schur = false;
  int sP = 0, sR = 0;
  double *Ablk = nullptr, *Ainv = nullptr, *Xs = nullptr, *Ys = nullptr, *Sc = nullptr, *Scinv = nullptr;
  GJPlan gjA, gjS;
  CopyCall copyA, copyScZ;
  GemmCall gemmXY, gemmSc, gemmZ1, gemmZPP;
  // accuracy guard with a few probe vectors x (the columns of op->probe_x):
  // block-eliminated levels probe the right residual, y = Z x, r = D y - x
  // (D stays intact); whole-D levels, whose Gauss-Jordan overwrites D, the
  // left one, y = D x before the inversion, r = Z y - x.  rho = |r|_inf /
  // |x|_inf per node after the inversion and after each Newton-Schulz step
  // (rho[k * nm + node]).  The steps W = D Z, Zns = 2 Z - Z W run on the
  // block-eliminated levels only, for the nodes whose gate the previous probe
  // switched on.
  double *py = nullptr, *pr = nullptr, *rho = nullptr, *Wns = nullptr, *Zns = nullptr;
  int* gate = nullptr;
  GemmCall probe1, probe2, nsW, nsZ;
  // ItI merges (dense blocks of the real representation): D = I + [[0, D12],
  // [D21, 0]], W = I - D12 D21 (in Dbuf), its inverse, the coupling C;
  // Z = D^{-1}, S = -Z C, Bnz holds the whole B, copyHext the children's
  // exterior outgoing data
  double *D12 = nullptr, *D21 = nullptr, *Winv = nullptr, *Cm = nullptr;
  CopyCall copyD21, copyZ11, copyC, copyHext;
  GemmCall gemmW;
  // fp32 copies for the mixed-precision solve
  float *Z32 = nullptr, *S32 = nullptr, *Bnz32 = nullptr;
  float *hint32 = nullptr, *gt32 = nullptr, *gint32 = nullptr;
  GemmCall gemmGt32, gemmHp32, gemmDown32;
};

struct Alloc {
  void* p;
  size_t bytes;
  hps_free_fn cb_free;  // non-NULL: the block came from an allocator callback
  void* cb_ctx;
};

struct TimedStage {
  const char* name;
  hipEvent_t a, b;
};

}  // namespace hps

namespace hps {
struct AdaptivePlan;  // adaptive 3D operators (adaptive.cpp)
void adaptive_free(AdaptivePlan* A);
int adaptive_solve(hps_op* op, const double* bdry, const double* src, double* u, int nrhs, hipStream_t st);
}  // namespace hps

struct hps_op {
  hps_tree_t tree{};
  int p = 0, d = 0, flags = 0, nd = 0;
  long long nl = 0;
  int npts = 0, ni = 0, ne = 0, nb = 0;
  double r = 0.0;
  hps::DevConsts* cst = nullptr;
  hipStream_t stream = nullptr;
  double *LU = nullptr, *Y = nullptr, *Tleaf = nullptr;
  // 3D leaves: LU holds L_ii^{-1}; Lbuf / Rbuf are build workspace, fint the
  // gathered interior sources
  double *Lbuf = nullptr, *Rbuf = nullptr, *fint = nullptr;
  hps::GJPlan leaf_gj;
  hps::GemmCall gemmYleaf, gemmVleaf;
  int *perm = nullptr, *pos = nullptr, *flag = nullptr;
  std::vector<hps::LevelPlan> levels;  // index = tree level of the parents
  // solve workspace: one block holding g, h, v (3D: fint) and every level's
  // hint, gt, gint; ws_take hands out its pieces in plan order
  char* ws_base = nullptr;
  long long ws_bytes = 0;
  std::function<double*(long long)> ws_take;
  // allocation-free solve: the solve's GEMM descriptors rebased onto the
  // device's static workspace (static_ok when ws + split-K parts fit in it)
  bool static_ok = false;
  char* static_base = nullptr;
  long long static_need = 0;
  std::vector<hps::GemmGroup> hgroups_static;
  hps::GemmGroup* dgroups_static = nullptr;
  // subtree recomputation (hps_build_subtrees): this operator keeps the top
  // levels resident; its leaves are the roots of complete subtrees of depth
  // sub->tree.depth, whose operators are rebuilt from the kept coefficients
  // (sub_coef) whenever a solve needs them
  int ext_side = 0;           // Gauss points per side of a top-level leaf (0: ordinary leaves)
  bool root_h = false;        // the source pass also forms the root's outgoing flux h[0]
  long long rstride = 0;      // right-hand-side stride of src / u (0: nl * npts)
  hps_op* sub = nullptr;      // one subtree's plan, rebuilt for each subtree in turn
  int full_depth = 0;         // depth of the whole tree
  double* sub_coef = nullptr; // device copy of every leaf's coefficients
  // merge-level build workspace.  Levels are built one after another on one
  // stream, so each level takes its transient buffers (gathered D, block
  // elimination and Newton-Schulz blocks, Gauss-Jordan panels, probe
  // products) from the start of lvl_ws, sized for the largest level; the
  // leaves' T sit in Tbuf[0] and the levels' T (below the root) alternate
  // between Tbuf[1] and Tbuf[0]
  char* lvl_ws = nullptr;
  long long lvl_ws_bytes = 0, lvl_cur = 0;
  double* Tbuf[2] = {nullptr, nullptr};
  // ItI variant (hps_build_iti): complex data in the real representation;
  // npts, ni, nb count reals (2 per complex value); LU holds (S B)^{-1} per
  // leaf, S the row equilibration (Robin rows folded into G and P, interior
  // row scales in Rbuf),
  // uws the leaf solutions before they are scattered to the caller's layout,
  // ident an identity matrix (ident_ld x ident_ld) for W = I - D12 D21
  bool iti = false;
  double eta = 0.0;
  hps::ItiConsts* ic = nullptr;
  double *uws = nullptr, *ident = nullptr;
  int ident_ld = 0;
  hps::GemmCall gemmUleaf, gemmUleaf0;
  std::vector<double*> g, h;           // per tree level 0..L: [nodes][NR][nb(level)]
  std::vector<int> nbl;                // boundary size per tree level
  double* v = nullptr;                 // [nl][NR][ni]
  int NR = 16;
  std::vector<hps::GemmGroup> hgroups;
  hps::GemmGroup* dgroups = nullptr;
  std::vector<hps::BlockOp> hops;
  hps::BlockOp* dops = nullptr;
  std::vector<hps::CopyItem> hitems;
  hps::CopyItem* ditems = nullptr;
  std::vector<hps::CopyTask> htasks;
  hps::CopyTask* dtasks = nullptr;
  hps::GemmCall gemmTleaf, gemmHleaf;
  hps::GemmCall adjYt, adjPt, adjQt, adjLinvT;  // adjoint leaf products
  double* wext = nullptr;                       // [nl][NR][ne]
  hps::CopyCall copyRoot;
  // mixed-precision solve (HPS_FLAG_FP32_COPY): fp32 operator copies and
  // workspaces, fp64 iterate and residuals, leaf adjacency
  bool fp32 = false;
  bool fp64_dropped = false;                   // HPS_FLAG_FP32_ONLY: fp64 solve operators freed
  int refine_sweeps = 3;
  double* coef = nullptr;                      // [nl][n_terms][npts]
  double* C2G = nullptr;                       // q x p row-major
  float *LU32 = nullptr, *Y32 = nullptr, *Qi32 = nullptr;
  std::vector<float*> g32, h32;
  float *v32 = nullptr, *hx32 = nullptr;
  double *gam = nullptr, *r1 = nullptr, *Qu = nullptr;
  int* nbr = nullptr;                          // [nl][4]: neighbour leaf*4 + face, or -1
  long long* bidx = nullptr;                   // [nl][4]: root-boundary offset, or -1
  std::vector<hps::GemmGroupF32> hgroups32;
  hps::GemmGroupF32* dgroups32 = nullptr;
  hps::GemmCall gemmHleaf32;
  long long split_elems = 0;                   // split-K workspace (elements), fp64 and fp32
  double* splitws = nullptr;
  float* splitws32 = nullptr;
  // merge-inverse probe vectors x (device, kProbes columns of the length of
  // the largest D) and 1 / |x|_inf; per-level results of the probes, filled
  // when the build is checked (host)
  double* probe_x = nullptr;
  int probe_ld = 0;
  double probe_inv_xmax = 1.0;
  bool info_ready = false;
  std::vector<hps_level_info_t> info;
  // build status block (device): the 4 pivot-failure flags, then every merge
  // level's probe residuals (rho_n doubles), so that one download checks a build
  double* rho_all = nullptr;
  long long rho_n = 0, rho_used = 0;
  std::vector<hps::Alloc> allocs;
  size_t resident = 0;
  std::vector<hps::TimedStage> stages;
  // adaptive 3D operator (hps_build_adaptive): its tree, plans and arenas
  hps::AdaptivePlan* ad = nullptr;
};

namespace hps {
long long gemm_prepare(std::vector<GemmGroup>& groups);
long long gemm_prepare_f32(std::vector<GemmGroupF32>& groups);
long long gemm_rblocks(const std::vector<GemmGroup>& groups);
long long gemm_rblocks_f32(const std::vector<GemmGroupF32>& groups);
long long gemm_plan_split(std::vector<GemmGroup>& groups);
long long gemm_plan_split_f32(std::vector<GemmGroupF32>& groups);
int gemm_launch_f32(const GemmGroupF32* dev_groups, int ngroups, long long nblocks, long long nrblocks, bool ta,
                    bool tb, hipStream_t st, int n_override);
int gemm_launch(const GemmGroup* dev_groups, int ngroups, long long nblocks, long long nrblocks, bool ta, bool tb,
                hipStream_t st, int n_override);
}  // namespace hps
