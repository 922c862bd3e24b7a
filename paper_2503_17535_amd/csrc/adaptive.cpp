// Adaptive 3D HPS (Section 4.2): octrees refined by the eight-child
// interpolation criterion with a face level restriction, leaf stage per leaf
// size, non-uniform merges and the adaptive downward pass.
//
// Tree: leaves (level, ix, iy, iz) over the cube [lo, hi]^3 in depth-first
// order (children in the merge's child order).  Every node boundary is a list
// of Gauss panels (q x q points, q = p - 2): a leaf has one per face; a merged
// node inherits its children's exterior panels, face by face, children on a
// face in sub-face order.  An interior interface of a merge is discretized on
// the coarser of its two sides, square by square (a square that is a panel of
// either side is an interface panel; otherwise its quadrants are walked).
// Because every node lists the panels inside any square of a face
// contiguously and in quadrant order, a fine side meets each coarse interface
// panel with four consecutive panels: its Dirichlet data there are the coarse
// panel's interpolant (UP, 4q^2 x q^2) and its Neumann data enter the balance
// at the coarse Gauss points through the fine panels' interpolants (DOWN,
// q^2 x 4q^2).
//
// Device work per merge level (all nodes of the level in each launch):
//   X_c = T_c E_c, Tp_c = R_c X_c for children with projected panels
//     (block copies of the identity runs, grouped GEMMs with UP / DOWN),
//   D, C, B, A gathered from the Tp_c (parent boundary order for the
//     exterior, so that T = A + B S needs no permutation),
//   Z = D^{-1} (Gauss-Jordan with partial pivoting over all of D, per node),
//   S = -Z C, T = A + B S.
// Solve: leaf sources -> v = L_ii^{-1} f, h = Q_i v per leaf size; upward
// h_int = sum R_c h_c, gt = -Z h_int, h = h_ext + B gt; downward
// g_int = S g + gt, child data E_c [g_ext; g_int]; leaves u = Y g + v.
// Leaves are processed in slots grouped by level (one leaf operator set per
// leaf size); coefficients, sources and solutions are permuted between the
// caller's depth-first order and the slots on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <set>
#include <vector>

#include "../../include/hps.h"
#include "op.hpp"
#include "precompute.hpp"

namespace hps {

// helpers of api.cpp
void* op_alloc_x(hps_op* op, size_t bytes, bool resident);
int add_gemm_x(hps_op* op, std::vector<GemmGroup> groups, GemmCall* call);
void add_copy_x(hps_op* op, const std::vector<BlockOp>& ops, CopyCall* call);
int run_gemm_x(hps_op* op, const GemmCall& c, hipStream_t st, int n_override);
int run_copy_x(hps_op* op, const CopyCall& c, int ncols_rt, double* dst, const double* s0, const double* s1,
               hipStream_t st);
int plan_gj_x(hps_op* op, GJPlan* g, double* A, double* Z, int m, long long batch);
int run_gj_x(hps_op* op, const GJPlan& g, hipStream_t st);
int get_consts_x(int d, int p, double r, DevConsts** out);
int finish_plan_x(hps_op* op);
int leaf3d_assemble_launch(const double* coeffs, const double* D1, const double* D2, const double* Mt, int p,
                           double* Lii, double* R, long long nl, hipStream_t st);
int leaf_gather_int_launch(const double* src, const int* Ii, int ni, int npts, long long nl, int nrhs, int NRcap,
                           double* fint, hipStream_t st);
int leaf_out_launch(const double* Y, const double* P, const double* g, const double* v, const int* Ii, const int* Ie,
                    int NI, int NE, int NB, int npts, long long nl, int nrhs, int NRcap, double* u, hipStream_t st,
                    long long rstride);
int adaptive_permute_launch(const double* src, double* dst, const int* idx, long long len, long long n, int nrhs,
                            long long src_rstride, long long dst_rstride, hipStream_t st);
int adaptive_check_launch(const double* f0, const double* f1, const double* E, int p, long long nl, double* err,
                          double* fmax, hipStream_t st);

namespace {

using Key = std::array<int, 4>;  // level, ix, iy, iz

Key child_key(const Key& k, int c, const MergeGeom& G) {
  return {k[0] + 1, 2 * k[1] + G.child_off[c][0], 2 * k[2] + G.child_off[c][1], 2 * k[3] + G.child_off[c][2]};
}
Key parent_key(const Key& k) { return {k[0] - 1, k[1] >> 1, k[2] >> 1, k[3] >> 1}; }

// Leaves in depth-first order; false if they do not tile the cube exactly.
bool dfs_order(const std::set<Key>& leaves, std::vector<Key>& out, std::set<Key>* internal_out = nullptr) {
  const MergeGeom& G = merge_geom(3);
  std::set<Key> internal;
  for (const Key& k : leaves) {
    if (k[0] < 0 || k[0] > 20) return false;
    const int n = 1 << k[0];
    if (k[1] < 0 || k[2] < 0 || k[3] < 0 || k[1] >= n || k[2] >= n || k[3] >= n) return false;
    Key a = k;
    while (a[0] > 0) {
      a = parent_key(a);
      internal.insert(a);
    }
  }
  for (const Key& k : leaves)
    if (internal.count(k)) return false;  // a leaf inside another leaf
  out.clear();
  std::vector<Key> stack = {Key{0, 0, 0, 0}};
  while (!stack.empty()) {
    Key k = stack.back();
    stack.pop_back();
    if (leaves.count(k)) {
      out.push_back(k);
    } else if (internal.count(k)) {
      for (int c = 7; c >= 0; --c) stack.push_back(child_key(k, c, G));
    } else {
      return false;  // a hole
    }
  }
  if (out.size() != leaves.size()) return false;
  if (internal_out) *internal_out = internal;
  return true;
}

// fine-grid box of a node
struct Box {
  long long lo[3], s;
};
Box fine_box(const Key& k, int maxl) {
  Box b;
  b.s = 1LL << (maxl - k[0]);
  for (int a = 0; a < 3; ++a) b.lo[a] = (long long)k[1 + a] * b.s;
  return b;
}

// pairs of leaves sharing a face of positive area whose levels differ by 2 or more
std::vector<int> unbalanced(const std::vector<Key>& lv) {
  int maxl = 0;
  for (const Key& k : lv) maxl = std::max(maxl, k[0]);
  const size_t n = lv.size();
  std::vector<Box> bx(n);
  for (size_t i = 0; i < n; ++i) bx[i] = fine_box(lv[i], maxl);
  // bucket leaves by each face plane for the neighbour search
  std::map<std::pair<int, long long>, std::vector<int>> lo_plane, hi_plane;
  for (size_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      lo_plane[{a, bx[i].lo[a]}].push_back((int)i);
      hi_plane[{a, bx[i].lo[a] + bx[i].s}].push_back((int)i);
    }
  std::vector<int> split;
  for (size_t i = 0; i < n; ++i) {
    bool bad = false;
    for (int a = 0; a < 3 && !bad; ++a)
      for (int side = 0; side < 2 && !bad; ++side) {
        const long long plane = bx[i].lo[a] + (side ? bx[i].s : 0);
        auto& cand = side ? lo_plane : hi_plane;
        auto it = cand.find({a, plane});
        if (it == cand.end()) continue;
        for (int j : it->second) {
          if (lv[j][0] < lv[i][0] + 2) continue;
          bool ov = true;
          for (int b = 0; b < 3; ++b) {
            if (b == a) continue;
            const long long l0 = std::max(bx[i].lo[b], bx[j].lo[b]);
            const long long l1 = std::min(bx[i].lo[b] + bx[i].s, bx[j].lo[b] + bx[j].s);
            if (l1 <= l0) ov = false;
          }
          if (ov) { bad = true; break; }
        }
      }
    if (bad) split.push_back((int)i);
  }
  return split;
}

// 1D barycentric interpolation matrix (rows: targets y, columns: nodes x), row-major
std::vector<double> interp1d(const std::vector<double>& x, const std::vector<double>& y) {
  const size_t n = x.size();
  std::vector<double> w(n, 1.0);
  for (size_t j = 0; j < n; ++j)
    for (size_t k = 0; k < n; ++k)
      if (k != j) w[j] /= (x[j] - x[k]);
  std::vector<double> M(y.size() * n, 0.0);
  for (size_t i = 0; i < y.size(); ++i) {
    int hit = -1;
    for (size_t j = 0; j < n; ++j)
      if (std::fabs(y[i] - x[j]) < 1e-15) hit = (int)j;
    if (hit >= 0) { M[i * n + hit] = 1.0; continue; }
    double s = 0.0;
    for (size_t j = 0; j < n; ++j) s += w[j] / (y[i] - x[j]);
    for (size_t j = 0; j < n; ++j) M[i * n + j] = (w[j] / (y[i] - x[j])) / s;
  }
  return M;
}

struct Panel {
  int face;           // face of the owning node
  int axis, a0, b0;   // normal axis; square corner in the tangential axes
  long long plane;    // fine-grid coordinate of the plane
  int s;              // side length on the fine grid
};

struct Seg {  // child panels [src, src + cnt) -> projected panels [dst, dst + cnt), or 4 -> 1
  int src, dst, cnt;
  bool proj;
};

struct Kid {
  int node = -1;
  bool proj = false;
  std::vector<Seg> segs;
  long long np = 0;                   // projected points
  int f0[6] = {0}, f1[6] = {0};       // projected panel range of each face
  double *X = nullptr, *Tp = nullptr; // device (proj only)
  double* gp = nullptr;               // [NR][np] vector workspace (proj only)
};

struct Node {
  Key key{};
  int parent = -1;
  int kid[8];
  bool leaf = true;
  int slot = -1;
  std::vector<Panel> bdry;
  long long n = 0;
  double* T = nullptr;
  double *g = nullptr, *h = nullptr;  // [NR][n]
  Kid kids[8];
  long long m = 0;
  int mo[13] = {0};   // interface panel offsets (panels)
  long long goff[25]; // parent group point offsets
  double *D = nullptr, *Z = nullptr, *C = nullptr, *S = nullptr, *B = nullptr, *A = nullptr;
  double *hint = nullptr, *gt = nullptr, *gint = nullptr, *hext = nullptr;
};

struct Level {
  std::vector<int> nodes;
  std::vector<GJPlan> gjs;  // one batched inverse per merge size of the level
  CopyCall pcols, prows, assemble;
  GemmCall gcols, grows, gemmS, gemmT;
  CopyCall uprows, uphint, uphext;
  GemmCall guprows, gemmGt, gemmH;
  GemmCall gemmDown;
  CopyCall downgp, downg;
  GemmCall gdown;
};

struct LeafGroup {
  int level = 0;
  long long s0 = 0, cnt = 0;
  DevConsts* cst = nullptr;
  GJPlan gj;
  GemmCall gemmY, gemmT, gemmV, gemmH;
};

}  // namespace

struct AdaptivePlan {
  double lo = 0.0, hi = 1.0;
  int p = 0, q = 0, q2 = 0, maxl = 0;
  std::vector<Node> nodes;      // node 0 = root
  std::vector<int> slot_node;   // slot -> node
  std::vector<int> slot_dfs;    // slot -> depth-first leaf index
  int *d_slot_dfs = nullptr, *d_dfs_slot = nullptr;
  std::vector<LeafGroup> groups;
  std::vector<Level> levels;    // deepest first
  double *Tall = nullptr, *Wall = nullptr, *Vall = nullptr;
  double *UP = nullptr, *DOWN = nullptr;
  double *coefslot = nullptr, *srcslot = nullptr, *uslot = nullptr;
  double *gleaf = nullptr, *hleaf = nullptr, *vleaf = nullptr;
  long long root_n = 0, max_m = 0, total_m = 0;
};

namespace {

// ---------------------------------------------------------------------------
// tree structure and panels (no device work)
// ---------------------------------------------------------------------------
int build_structure(AdaptivePlan& A, const std::vector<Key>& dfs) {
  const MergeGeom& G = merge_geom(3);
  A.maxl = 0;
  for (const Key& k : dfs) A.maxl = std::max(A.maxl, k[0]);
  std::set<Key> leafset(dfs.begin(), dfs.end());
  // nodes: breadth-first from the root (parents before children)
  std::map<Key, int> index;
  A.nodes.clear();
  A.nodes.push_back(Node());
  A.nodes[0].key = {0, 0, 0, 0};
  index[A.nodes[0].key] = 0;
  for (size_t i = 0; i < A.nodes.size(); ++i) {
    const Key k = A.nodes[i].key;
    for (int c = 0; c < 8; ++c) A.nodes[i].kid[c] = -1;
    if (leafset.count(k)) continue;
    A.nodes[i].leaf = false;
    for (int c = 0; c < 8; ++c) {
      Node nd;
      nd.key = child_key(k, c, G);
      nd.parent = (int)i;
      index[nd.key] = (int)A.nodes.size();
      A.nodes[i].kid[c] = (int)A.nodes.size();
      A.nodes.push_back(nd);
    }
  }
  // leaf slots grouped by level, depth-first within a level
  A.slot_node.clear();
  A.slot_dfs.clear();
  A.groups.clear();
  for (int l = 0; l <= A.maxl; ++l) {
    LeafGroup grp;
    grp.level = l;
    grp.s0 = (long long)A.slot_node.size();
    for (size_t i = 0; i < dfs.size(); ++i)
      if (dfs[i][0] == l) {
        const int nd = index[dfs[i]];
        A.nodes[nd].slot = (int)A.slot_node.size();
        A.slot_node.push_back(nd);
        A.slot_dfs.push_back((int)i);
      }
    grp.cnt = (long long)A.slot_node.size() - grp.s0;
    if (grp.cnt > 0) A.groups.push_back(grp);
  }
  // boundaries, deepest nodes first
  std::vector<int> order(A.nodes.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return A.nodes[a].key[0] > A.nodes[b].key[0]; });
  A.levels.clear();
  A.max_m = 0;
  A.total_m = 0;
  std::map<int, int> level_of;  // tree level -> index in A.levels
  for (int ni : order) {
    Node& nd = A.nodes[ni];
    if (nd.leaf) {
      const Box b = fine_box(nd.key, A.maxl);
      for (int f = 0; f < 6; ++f) {
        const FaceDesc& fd = G.faces[f];
        Panel pn;
        pn.face = f;
        pn.axis = fd.axis;
        pn.plane = b.lo[fd.axis] + (fd.side ? b.s : 0);
        pn.a0 = (int)b.lo[fd.tang[0]];
        pn.b0 = (int)b.lo[fd.tang[1]];
        pn.s = (int)b.s;
        nd.bdry.push_back(pn);
      }
      nd.n = (long long)nd.bdry.size() * A.q2;
      continue;
    }
    // children's panels per face
    auto face_range = [&](int c, int f, int& k0, int& k1) {
      const std::vector<Panel>& bd = A.nodes[nd.kid[c]].bdry;
      k0 = -1;
      k1 = -1;
      for (int k = 0; k < (int)bd.size(); ++k)
        if (bd[k].face == f) {
          if (k0 < 0) k0 = k;
          k1 = k + 1;
        }
    };
    for (int c = 0; c < 8; ++c) {
      Kid& kc = nd.kids[c];
      kc = Kid();
      kc.node = nd.kid[c];
    }
    // interfaces: coarse squares, and each side's segments on its face
    std::vector<Seg> face_segs[8][6];
    bool face_done[8][6] = {{false}};
    long long moff = 0;
    for (int i = 0; i < 12; ++i) {
      const int c1 = G.iface[i][0], f1 = G.iface[i][1], c2 = G.iface[i][2], f2 = G.iface[i][3];
      int a0, a1, b0, b1;
      face_range(c1, f1, a0, a1);
      face_range(c2, f2, b0, b1);
      const std::vector<Panel>& P1 = A.nodes[nd.kid[c1]].bdry;
      const std::vector<Panel>& P2 = A.nodes[nd.kid[c2]].bdry;
      std::map<std::array<int, 3>, int> s1, s2;
      for (int k = a0; k < a1; ++k) s1[{P1[k].a0, P1[k].b0, P1[k].s}] = k;
      for (int k = b0; k < b1; ++k) s2[{P2[k].a0, P2[k].b0, P2[k].s}] = k;
      // the interface square = the child's face square
      int sa = INT32_MAX, sb = INT32_MAX, se = 0;
      for (int k = a0; k < a1; ++k) {
        sa = std::min(sa, P1[k].a0);
        sb = std::min(sb, P1[k].b0);
        se = std::max(se, P1[k].a0 + P1[k].s);
      }
      std::vector<std::array<int, 3>> coarse;
      std::vector<std::array<int, 3>> stack = {{sa, sb, se - sa}};
      while (!stack.empty()) {
        const std::array<int, 3> sq = stack.back();
        stack.pop_back();
        if (s1.count(sq) || s2.count(sq)) { coarse.push_back(sq); continue; }
        const int h = sq[2] / 2;
        if (h == 0) { set_error("adaptive tree: interface sides do not meet on common squares"); return HPS_EINVAL; }
        static const int quad[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
        for (int j = 3; j >= 0; --j) stack.push_back({sq[0] + quad[j][0] * h, sq[1] + quad[j][1] * h, h});
      }
      nd.mo[i] = (int)moff;
      moff += (long long)coarse.size();
      // segments of each side: walk its face panels against the coarse list
      for (int side = 0; side < 2; ++side) {
        const int c = side ? c2 : c1, f = side ? f2 : f1;
        const std::map<std::array<int, 3>, int>& sm = side ? s2 : s1;
        const std::vector<Panel>& P = side ? P2 : P1;
        std::vector<Seg>& segs = face_segs[c][f];
        int dst = 0;
        for (const auto& sq : coarse) {
          auto it = sm.find(sq);
          if (it != sm.end()) {
            if (!segs.empty() && !segs.back().proj && segs.back().src + segs.back().cnt == it->second &&
                segs.back().dst + segs.back().cnt == dst)
              segs.back().cnt++;
            else
              segs.push_back({it->second, dst, 1, false});
          } else {
            // the four quadrants, consecutive and in quadrant order
            const int h = sq[2] / 2;
            static const int quad[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
            int k0 = -1;
            for (int j = 0; j < 4; ++j) {
              auto jt = sm.find({sq[0] + quad[j][0] * h, sq[1] + quad[j][1] * h, h});
              if (jt == sm.end() || (j > 0 && jt->second != k0 + j)) {
                set_error("adaptive tree: level restriction violated across an interface (leaves more than one "
                          "level apart share a face)");
                return HPS_EINVAL;
              }
              if (j == 0) k0 = jt->second;
            }
            (void)P;
            segs.push_back({k0, dst, 4, true});
          }
          ++dst;
        }
        face_done[c][f] = true;
      }
    }
    nd.m = moff * A.q2;
    A.max_m = std::max(A.max_m, nd.m);
    A.total_m += nd.m;
    // each child's projected layout: faces in order; exterior faces unchanged
    for (int c = 0; c < 8; ++c) {
      Kid& kc = nd.kids[c];
      int cur = 0;
      for (int f = 0; f < 6; ++f) {
        int k0, k1;
        face_range(c, f, k0, k1);
        kc.f0[f] = cur;
        if (face_done[c][f]) {
          // the child's own panels in its own order unless a segment says otherwise
          const std::vector<Seg>& fs = face_segs[c][f];
          if (!(fs.size() == 1 && !fs[0].proj && fs[0].src == k0 && fs[0].dst == 0 && fs[0].cnt == k1 - k0))
            kc.proj = true;
          for (Seg s : fs) {
            s.dst += cur;
            kc.segs.push_back(s);
          }
          int cnt = 0;
          for (const Seg& s : face_segs[c][f]) cnt += s.proj ? 1 : s.cnt;
          cur += cnt;
        } else {
          kc.segs.push_back({k0, cur, k1 - k0, false});
          cur += k1 - k0;
        }
        kc.f1[f] = cur;
      }
      kc.np = (long long)cur * A.q2;
    }
    // parent boundary: faces in order, the children on a face in sub-face order
    long long off = 0;
    for (int g = 0; g < 24; ++g) {
      const int c = G.group_child[g], f = G.group_face[g];
      int k0, k1;
      face_range(c, f, k0, k1);
      nd.goff[g] = off;
      const std::vector<Panel>& bd = A.nodes[nd.kid[c]].bdry;
      for (int k = k0; k < k1; ++k) {
        Panel pn = bd[k];
        pn.face = f;
        nd.bdry.push_back(pn);
      }
      off += (long long)(k1 - k0) * A.q2;
    }
    nd.goff[24] = off;
    nd.n = off;
    auto lit = level_of.find(nd.key[0]);
    if (lit == level_of.end()) {
      level_of[nd.key[0]] = (int)A.levels.size();
      A.levels.push_back(Level());
      lit = level_of.find(nd.key[0]);
    }
    A.levels[lit->second].nodes.push_back(ni);
  }
  A.root_n = A.nodes[0].n;
  return HPS_OK;
}

GemmGroup grp(const double* Am, int lda, const double* Bm, int ldb, double* Cm, int ldc, int M, int N, int K,
              double alpha, double beta, const double* C0 = nullptr, int ldc0 = 0, long long batch = 1,
              long long sA = 0, long long sB = 0, long long sC = 0, long long sC0 = 0) {
  GemmGroup g;
  std::memset(&g, 0, sizeof(g));
  g.A = Am; g.B = Bm; g.C = Cm; g.C0 = C0;
  g.sA = sA; g.sB = sB; g.sC = sC; g.sC0 = sC0;
  g.lda = lda; g.ldb = ldb; g.ldc = ldc; g.ldc0 = ldc0 ? ldc0 : ldc;
  g.M = M; g.N = N; g.K = K; g.nseg = 1;
  g.alpha = alpha; g.beta = beta;
  g.batch = (int)batch;
  return g;
}

BlockOp blk(long long dst_off, int dst_ld, int rows, int cols) {
  BlockOp o;
  std::memset(&o, 0, sizeof(o));
  o.dst_off = dst_off;
  o.dst_ld = dst_ld;
  o.rows = rows;
  o.cols = cols;
  return o;
}
void src(BlockOp& o, long long off, int ld) {
  o.src_buf[o.nsrc] = 0;
  o.src_off[o.nsrc] = off;
  o.src_ld[o.nsrc] = ld;
  o.nsrc++;
}

// Host check of a plan before anything runs: every block copy and every
// product stays inside the arenas it addresses (runtime column counts taken
// at their maximum).  A failure is an internal planning error.
bool ops_in_range(const std::vector<BlockOp>& ops, long long dst_size, long long src_size, int ncols_rt) {
  for (const BlockOp& o : ops) {
    const long long cols = o.cols > 0 ? o.cols : ncols_rt;
    if (o.rows <= 0 || cols <= 0) continue;
    if (o.dst_off < 0 || o.rows > o.dst_ld || o.dst_off + (cols - 1) * o.dst_ld + o.rows > dst_size) return false;
    for (int k = 0; k < o.nsrc; ++k)
      if (o.src_off[k] < 0 || o.rows > o.src_ld[k] || o.src_off[k] + (cols - 1) * o.src_ld[k] + o.rows > src_size)
        return false;
  }
  return true;
}

struct Arena {
  const double* base;
  long long size;
};
bool gemms_in_range(const std::vector<GemmGroup>& gs, const std::vector<Arena>& arenas) {
  auto inside = [&](const double* p, long long extent) {
    for (const Arena& a : arenas)
      if (p >= a.base && p < a.base + a.size) return p + extent <= a.base + a.size;
    return true;  // constants outside the arenas
  };
  for (const GemmGroup& g : gs) {
    const long long b = g.batch > 0 ? g.batch - 1 : 0;
    if (g.lda < g.M || g.ldb < g.K || g.ldc < g.M) return false;
    if (!inside(g.A, b * g.sA + (long long)(g.K - 1) * g.lda + g.M)) return false;
    if (!inside(g.B, b * g.sB + (long long)(g.N - 1) * g.ldb + g.K)) return false;
    if (!inside(g.C, b * g.sC + (long long)(g.N - 1) * g.ldc + g.M)) return false;
    if (g.C0 && !inside(g.C0, b * g.sC0 + (long long)(g.N - 1) * g.ldc0 + g.M)) return false;
  }
  return true;
}

// ---------------------------------------------------------------------------
// device plan
// ---------------------------------------------------------------------------
int plan_adaptive(hps_op* op, AdaptivePlan& A) {
  const MergeGeom& G = merge_geom(3);
  const int q2 = A.q2, NR = op->NR, ni = op->ni, nb = op->nb;
  const long long nl = op->nl;
  auto alloc = [&](long long elems, bool resident) { return (double*)op_alloc_x(op, sizeof(double) * std::max(1LL, elems), resident); };
  // panel operators: UP (4q^2 x q^2), DOWN (q^2 x 4q^2), column-major
  {
    const LeafOps& o = leaf_ops(3, A.p);
    const std::vector<double>& g = o.gl;
    const int q = A.q;
    std::vector<double> ylo(q), yhi(q);
    for (int i = 0; i < q; ++i) { ylo[i] = (g[i] - 1.0) / 2.0; yhi[i] = (g[i] + 1.0) / 2.0; }
    const std::vector<double> H[2] = {interp1d(g, ylo), interp1d(g, yhi)};  // q x q row-major
    static const int quad[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
    std::vector<double> up((size_t)4 * q2 * q2), down((size_t)q2 * 4 * q2, 0.0);
    for (int j = 0; j < 4; ++j)
      for (int b = 0; b < q; ++b)
        for (int a = 0; a < q; ++a)          // fine point (a, b) of quadrant j
          for (int bb = 0; bb < q; ++bb)
            for (int aa = 0; aa < q; ++aa)   // coarse point (aa, bb)
              up[(size_t)(j * q2 + a + q * b) + (size_t)(aa + q * bb) * 4 * q2] =
                  H[quad[j][0]][a * q + aa] * H[quad[j][1]][b * q + bb];
    for (int b = 0; b < q; ++b)
      for (int a = 0; a < q; ++a) {
        // a node on the seam (the middle node of an odd rule) reads the lower quadrant
        const int s1 = g[a] > 1e-12, s2 = g[b] > 1e-12;
        int j = 0;
        for (; j < 4; ++j)
          if (quad[j][0] == s1 && quad[j][1] == s2) break;
        const std::vector<double> w1 = interp1d(g, {2.0 * g[a] + (s1 ? -1.0 : 1.0)});
        const std::vector<double> w2 = interp1d(g, {2.0 * g[b] + (s2 ? -1.0 : 1.0)});
        for (int bb = 0; bb < q; ++bb)
          for (int aa = 0; aa < q; ++aa)
            down[(size_t)(a + q * b) + (size_t)(j * q2 + aa + q * bb) * q2] = w1[aa] * w2[bb];
      }
    A.UP = alloc((long long)up.size(), true);
    A.DOWN = alloc((long long)down.size(), true);
    if (!A.UP || !A.DOWN) { set_error("device allocation failed (panel operators)"); return HPS_ENOMEM; }
    HPS_HIP_TRY(hipMemcpy(A.UP, up.data(), sizeof(double) * up.size(), hipMemcpyHostToDevice));
    HPS_HIP_TRY(hipMemcpy(A.DOWN, down.data(), sizeof(double) * down.size(), hipMemcpyHostToDevice));
  }
  // slot permutations
  {
    std::vector<int> dfs_slot(nl);
    for (long long s = 0; s < nl; ++s) dfs_slot[A.slot_dfs[s]] = (int)s;
    A.d_slot_dfs = (int*)op_alloc_x(op, sizeof(int) * nl, true);
    A.d_dfs_slot = (int*)op_alloc_x(op, sizeof(int) * nl, true);
    if (!A.d_slot_dfs || !A.d_dfs_slot) { set_error("device allocation failed (leaf order)"); return HPS_ENOMEM; }
    HPS_HIP_TRY(hipMemcpy(A.d_slot_dfs, A.slot_dfs.data(), sizeof(int) * nl, hipMemcpyHostToDevice));
    HPS_HIP_TRY(hipMemcpy(A.d_dfs_slot, dfs_slot.data(), sizeof(int) * nl, hipMemcpyHostToDevice));
  }
  // T arena: leaf T (slot order), every merged node's T but the root's, the
  // projected children's X and Tp
  long long tsz = nl * nb * nb;
  for (size_t i = 1; i < A.nodes.size(); ++i)
    if (!A.nodes[i].leaf) tsz += A.nodes[i].n * A.nodes[i].n;
  for (const Node& nd : A.nodes)
    if (!nd.leaf)
      for (const Kid& kc : nd.kids)
        if (kc.proj) tsz += A.nodes[kc.node].n * kc.np + kc.np * kc.np;
  A.Tall = alloc(tsz, true);
  // merge arena: D, Z, C, S, B, A per node
  long long wsz = 0;
  for (const Node& nd : A.nodes)
    if (!nd.leaf) wsz += 2 * nd.m * nd.m + 3 * nd.m * nd.n + nd.n * nd.n;
  A.Wall = alloc(wsz, true);
  // vector arena
  long long vsz = 0;
  for (const Node& nd : A.nodes) {
    vsz += 2 * (long long)NR * nd.n;
    if (!nd.leaf) {
      vsz += 3 * (long long)NR * nd.m + (long long)NR * nd.n;
      for (const Kid& kc : nd.kids)
        if (kc.proj) vsz += (long long)NR * kc.np;
    }
  }
  vsz += 2 * nl * NR * ni;  // v, fint
  A.Vall = alloc(vsz, false);
  op->LU = alloc(nl * ni * ni, true);
  op->Y = alloc(nl * ni * nb, true);
  long long gmax = 0;
  for (const LeafGroup& g : A.groups) gmax = std::max(gmax, g.cnt);
  op->Lbuf = alloc(gmax * ni * ni, false);
  op->Rbuf = alloc(gmax * ni * nb, false);
  A.coefslot = alloc(nl * 10 * op->npts, false);
  A.srcslot = alloc((long long)NR * nl * op->npts, false);
  A.uslot = alloc((long long)NR * nl * op->npts, false);
  op->flag = (int*)op_alloc_x(op, sizeof(int) * 4, false);
  if (!A.Tall || !A.Wall || !A.Vall || !op->LU || !op->Y || !op->Lbuf || !op->Rbuf || !A.coefslot || !A.srcslot ||
      !A.uslot || !op->flag) {
    set_error("device allocation failed (adaptive operator)");
    return HPS_ENOMEM;
  }
  // carve the arenas
  long long tc = 0, wc = 0, vc = 0;
  auto tt = [&](long long e) { double* p = A.Tall + tc; tc += e; return p; };
  auto ww = [&](long long e) { double* p = A.Wall + wc; wc += e; return p; };
  auto vv = [&](long long e) { double* p = A.Vall + vc; vc += e; return p; };
  double* Tleaf = tt(nl * nb * nb);
  A.gleaf = vv(nl * NR * nb);
  A.hleaf = vv(nl * NR * nb);
  A.vleaf = vv(nl * NR * ni);
  op->fint = vv(nl * NR * ni);
  for (long long s = 0; s < nl; ++s) {
    Node& nd = A.nodes[A.slot_node[s]];
    nd.T = Tleaf + s * nb * nb;
    nd.g = A.gleaf + s * NR * nb;
    nd.h = A.hleaf + s * NR * nb;
  }
  // D and Z of the nodes of one level with one merge size sit back to back,
  // so that one batched Gauss-Jordan inverts them all
  for (Level& L : A.levels) {
    std::map<long long, std::vector<int>> by_m;
    for (int ni_ : L.nodes) by_m[A.nodes[ni_].m].push_back(ni_);
    for (auto& kv : by_m) {
      const long long m = kv.first, cnt = (long long)kv.second.size();
      double* Dg = ww(cnt * m * m);
      double* Zg = ww(cnt * m * m);
      for (long long k = 0; k < cnt; ++k) {
        A.nodes[kv.second[k]].D = Dg + k * m * m;
        A.nodes[kv.second[k]].Z = Zg + k * m * m;
      }
      GJPlan gj;
      HPS_TRY(plan_gj_x(op, &gj, Dg, Zg, (int)m, cnt));
      gj.flag = op->flag;
      L.gjs.push_back(gj);
    }
  }
  for (size_t i = 0; i < A.nodes.size(); ++i) {
    Node& nd = A.nodes[i];
    if (nd.leaf) continue;
    if (i > 0) nd.T = tt(nd.n * nd.n);
    nd.g = vv((long long)NR * nd.n);
    nd.h = vv((long long)NR * nd.n);
    nd.C = ww(nd.m * nd.n);
    nd.S = ww(nd.m * nd.n);
    nd.B = ww(nd.n * nd.m);
    nd.A = ww(nd.n * nd.n);
    nd.hint = vv((long long)NR * nd.m);
    nd.gt = vv((long long)NR * nd.m);
    nd.gint = vv((long long)NR * nd.m);
    nd.hext = vv((long long)NR * nd.n);
    for (Kid& kc : nd.kids)
      if (kc.proj) {
        kc.X = tt(A.nodes[kc.node].n * kc.np);
        kc.Tp = tt(kc.np * kc.np);
        kc.gp = vv((long long)NR * kc.np);
      }
  }
  // leaf groups: constants per leaf size, Gauss-Jordan, products
  for (LeafGroup& lg : A.groups) {
    const double r = (A.hi - A.lo) / 2.0 / (double)(1LL << lg.level);
    HPS_TRY(get_consts_x(3, A.p, r, &lg.cst));
    HPS_TRY(plan_gj_x(op, &lg.gj, op->Lbuf, op->LU + lg.s0 * ni * ni, ni, lg.cnt));
    lg.gj.flag = op->flag;
    HPS_TRY(add_gemm_x(op, {grp(op->LU + lg.s0 * ni * ni, ni, op->Rbuf, ni, op->Y + lg.s0 * ni * nb, ni, ni, nb, ni,
                                -1.0, 0.0, nullptr, 0, lg.cnt, (long long)ni * ni, (long long)ni * nb,
                                (long long)ni * nb)},
                       &lg.gemmY));
    HPS_TRY(add_gemm_x(op, {grp(lg.cst->Qi, nb, op->Y + lg.s0 * ni * nb, ni, Tleaf + lg.s0 * nb * nb, nb, nb, nb, ni,
                                1.0, 1.0, lg.cst->QeP, nb, lg.cnt, 0, (long long)ni * nb, (long long)nb * nb, 0)},
                       &lg.gemmT));
    HPS_TRY(add_gemm_x(op, {grp(op->LU + lg.s0 * ni * ni, ni, op->fint + lg.s0 * NR * ni, ni,
                                A.vleaf + lg.s0 * NR * ni, ni, ni, NR, ni, 1.0, 0.0, nullptr, 0, lg.cnt,
                                (long long)ni * ni, (long long)NR * ni, (long long)NR * ni)},
                       &lg.gemmV));
    HPS_TRY(add_gemm_x(op, {grp(lg.cst->Qi, nb, A.vleaf + lg.s0 * NR * ni, ni, A.hleaf + lg.s0 * NR * nb, nb, nb, NR,
                                ni, 1.0, 0.0, nullptr, 0, lg.cnt, 0, (long long)NR * ni, (long long)NR * nb)},
                       &lg.gemmH));
  }
  op->cst = A.groups[0].cst;
  // merge levels
  auto toff = [&](const double* p) { return (long long)(p - A.Tall); };
  auto voff = [&](const double* p) { return (long long)(p - A.Vall); };
  for (Level& L : A.levels) {
    std::vector<BlockOp> pcols, prows, asmb, uprows, uphint, uphext, downgp, downg;
    std::vector<GemmGroup> gcols, grows, gS, gT, guprows, gGt, gH, gDown, gdown;
    for (int ni_ : L.nodes) {
      Node& nd = A.nodes[ni_];
      const int m = (int)nd.m, n = (int)nd.n;
      // projections of the children
      for (Kid& kc : nd.kids) {
        if (!kc.proj) continue;
        const Node& ch = A.nodes[kc.node];
        const int nc = (int)ch.n, np = (int)kc.np;
        for (const Seg& s : kc.segs) {
          if (!s.proj) {
            BlockOp o = blk(toff(kc.X) + (long long)s.dst * q2 * nc, nc, nc, s.cnt * q2);
            src(o, toff(ch.T) + (long long)s.src * q2 * nc, nc);
            pcols.push_back(o);
            BlockOp r = blk(toff(kc.Tp) + (long long)s.dst * q2, np, s.cnt * q2, np);
            src(r, toff(kc.X) + (long long)s.src * q2, nc);
            prows.push_back(r);
            BlockOp u = blk(voff(kc.gp) + (long long)s.dst * q2, np, s.cnt * q2, -1);
            src(u, voff(ch.h) + (long long)s.src * q2, nc);
            uprows.push_back(u);
            BlockOp d = blk(voff(ch.g) + (long long)s.src * q2, nc, s.cnt * q2, -1);
            src(d, voff(kc.gp) + (long long)s.dst * q2, np);
            downg.push_back(d);
          } else {
            gcols.push_back(grp(ch.T + (long long)s.src * q2 * nc, nc, A.UP, 4 * q2, kc.X + (long long)s.dst * q2 * nc,
                                nc, nc, q2, 4 * q2, 1.0, 0.0));
            grows.push_back(grp(A.DOWN, q2, kc.X + (long long)s.src * q2, nc, kc.Tp + (long long)s.dst * q2, np, q2,
                                np, 4 * q2, 1.0, 0.0));
            guprows.push_back(grp(A.DOWN, q2, ch.h + (long long)s.src * q2, nc, kc.gp + (long long)s.dst * q2, np, q2,
                                  NR, 4 * q2, 1.0, 0.0));
            gdown.push_back(grp(A.UP, 4 * q2, kc.gp + (long long)s.dst * q2, np, ch.g + (long long)s.src * q2, nc,
                                4 * q2, NR, q2, 1.0, 0.0));
          }
        }
      }
      // sources in projected coordinates: Tp_c (or T_c) and hp_c (or h_c)
      auto Tp = [&](int c) { const Kid& kc = nd.kids[c]; return kc.proj ? kc.Tp : A.nodes[kc.node].T; };
      auto ldp = [&](int c) { const Kid& kc = nd.kids[c]; return (int)kc.np; };
      auto hp = [&](int c) { const Kid& kc = nd.kids[c]; return kc.proj ? kc.gp : A.nodes[kc.node].h; };
      auto gpt = [&](int c) { const Kid& kc = nd.kids[c]; return kc.proj ? kc.gp : A.nodes[kc.node].g; };
      auto frow = [&](int c, int f) { return (long long)nd.kids[c].f0[f] * q2; };
      auto fcnt = [&](int c, int f) { return (nd.kids[c].f1[f] - nd.kids[c].f0[f]) * q2; };
      auto mrow = [&](int i) { return (long long)nd.mo[i] * q2; };
      auto mcnt = [&](int i) { return (int)((i < 11 ? nd.mo[i + 1] * (long long)q2 : nd.m) - (long long)nd.mo[i] * q2); };
      auto gcnt = [&](int g) { return (int)(nd.goff[g + 1] - nd.goff[g]); };
      const long long Dw = (long long)(nd.D - A.Wall), Cw = (long long)(nd.C - A.Wall);
      const long long Bw = (long long)(nd.B - A.Wall), Aw = (long long)(nd.A - A.Wall);
      // D (interface x interface)
      for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j) {
          BlockOp o = blk(Dw + mrow(i) + mrow(j) * m, m, mcnt(i), mcnt(j));
          for (int c = 0; c < 8; ++c) {
            const int fi = G.face_on_iface[c][i], fj = G.face_on_iface[c][j];
            if (fi < 0 || fj < 0) continue;
            src(o, toff(Tp(c)) + frow(c, fi) + frow(c, fj) * ldp(c), ldp(c));
          }
          asmb.push_back(o);
        }
      // C (interface x parent group), B (parent group x interface), A (group x group)
      for (int i = 0; i < 12; ++i)
        for (int g = 0; g < 24; ++g) {
          const int c = G.group_child[g], f = G.group_face[g], fi = G.face_on_iface[c][i];
          BlockOp o = blk(Cw + mrow(i) + nd.goff[g] * m, m, mcnt(i), gcnt(g));
          if (fi >= 0) src(o, toff(Tp(c)) + frow(c, fi) + frow(c, f) * ldp(c), ldp(c));
          asmb.push_back(o);
          BlockOp b = blk(Bw + nd.goff[g] + mrow(i) * n, n, gcnt(g), mcnt(i));
          if (fi >= 0) src(b, toff(Tp(c)) + frow(c, f) + frow(c, fi) * ldp(c), ldp(c));
          asmb.push_back(b);
        }
      for (int g = 0; g < 24; ++g)
        for (int g2 = 0; g2 < 24; ++g2) {
          const int c = G.group_child[g], f = G.group_face[g], c2 = G.group_child[g2], f2 = G.group_face[g2];
          BlockOp o = blk(Aw + nd.goff[g] + nd.goff[g2] * n, n, gcnt(g), gcnt(g2));
          if (c == c2) src(o, toff(Tp(c)) + frow(c, f) + frow(c, f2) * ldp(c), ldp(c));
          asmb.push_back(o);
        }
      gS.push_back(grp(nd.Z, m, nd.C, m, nd.S, m, m, n, m, -1.0, 0.0));
      if (ni_ != 0) gT.push_back(grp(nd.B, n, nd.S, m, nd.T, n, n, n, m, 1.0, 1.0, nd.A, n));
      // solve, upward: h_int, h_ext, gt, h
      for (int i = 0; i < 12; ++i) {
        BlockOp o = blk(voff(nd.hint) + mrow(i), m, mcnt(i), -1);
        for (int c = 0; c < 8; ++c) {
          const int fi = G.face_on_iface[c][i];
          if (fi >= 0) src(o, voff(hp(c)) + frow(c, fi), ldp(c));
        }
        uphint.push_back(o);
      }
      for (int g = 0; g < 24; ++g) {
        const int c = G.group_child[g], f = G.group_face[g];
        BlockOp o = blk(voff(nd.hext) + nd.goff[g], n, gcnt(g), -1);
        src(o, voff(hp(c)) + frow(c, f), ldp(c));
        uphext.push_back(o);
      }
      gGt.push_back(grp(nd.Z, m, nd.hint, m, nd.gt, m, m, NR, m, -1.0, 0.0));
      if (ni_ != 0) gH.push_back(grp(nd.B, n, nd.gt, m, nd.h, n, n, NR, m, 1.0, 1.0, nd.hext, n));
      // solve, downward: g_int = S g + gt; children's data
      gDown.push_back(grp(nd.S, m, nd.g, n, nd.gint, m, m, NR, n, 1.0, 1.0, nd.gt, m));
      for (int c = 0; c < 8; ++c) {
        for (int e = 0; e < 3; ++e) {
          const int f = G.ext_face[c][e], g = G.group_of[c][f];
          BlockOp o = blk(voff(gpt(c)) + frow(c, f), ldp(c), fcnt(c, f), -1);
          src(o, voff(nd.g) + nd.goff[g], n);
          downgp.push_back(o);
        }
        for (int k = 0; k < 3; ++k) {
          const int i = G.int_list[c][k], f = G.face_on_iface[c][i];
          BlockOp o = blk(voff(gpt(c)) + frow(c, f), ldp(c), fcnt(c, f), -1);
          src(o, voff(nd.gint) + mrow(i), m);
          downgp.push_back(o);
        }
      }
    }
    const std::vector<Arena> arenas = {{A.Tall, tsz}, {A.Wall, wsz}, {A.Vall, vsz}};
    if (!ops_in_range(pcols, tsz, tsz, 1) || !ops_in_range(prows, tsz, tsz, 1) ||
        !ops_in_range(asmb, wsz, tsz, 1) || !ops_in_range(uprows, vsz, vsz, NR) ||
        !ops_in_range(uphint, vsz, vsz, NR) || !ops_in_range(uphext, vsz, vsz, NR) ||
        !ops_in_range(downgp, vsz, vsz, NR) || !ops_in_range(downg, vsz, vsz, NR)) {
      set_error("adaptive plan: a block copy leaves its buffer (internal error)");
      return HPS_EINVAL;
    }
    for (const std::vector<GemmGroup>* gl : {&gcols, &grows, &gS, &gT, &guprows, &gGt, &gH, &gDown, &gdown})
      if (!gemms_in_range(*gl, arenas)) {
        set_error("adaptive plan: a product leaves its buffer (internal error)");
        return HPS_EINVAL;
      }
    add_copy_x(op, pcols, &L.pcols);
    add_copy_x(op, prows, &L.prows);
    add_copy_x(op, asmb, &L.assemble);
    add_copy_x(op, uprows, &L.uprows);
    add_copy_x(op, uphint, &L.uphint);
    add_copy_x(op, uphext, &L.uphext);
    add_copy_x(op, downgp, &L.downgp);
    add_copy_x(op, downg, &L.downg);
    HPS_TRY(add_gemm_x(op, gcols, &L.gcols));
    HPS_TRY(add_gemm_x(op, grows, &L.grows));
    HPS_TRY(add_gemm_x(op, gS, &L.gemmS));
    HPS_TRY(add_gemm_x(op, gT, &L.gemmT));
    HPS_TRY(add_gemm_x(op, guprows, &L.guprows));
    HPS_TRY(add_gemm_x(op, gGt, &L.gemmGt));
    HPS_TRY(add_gemm_x(op, gH, &L.gemmH));
    HPS_TRY(add_gemm_x(op, gDown, &L.gemmDown));
    HPS_TRY(add_gemm_x(op, gdown, &L.gdown));
  }
  return finish_plan_x(op);
}

int run_adaptive_build(hps_op* op, AdaptivePlan& A, const double* coeffs, hipStream_t st) {
  const long long nl = op->nl;
  const int npts = op->npts;
  HPS_HIP_TRY(hipMemsetAsync(op->flag, 0, sizeof(int) * 4, st));
  HPS_TRY(adaptive_permute_launch(coeffs, A.coefslot, A.d_slot_dfs, 10LL * npts, nl, 1, 0, 0, st));
  for (LeafGroup& lg : A.groups) {
    HPS_TRY(leaf3d_assemble_launch(A.coefslot + lg.s0 * 10 * npts, lg.cst->D1, lg.cst->D2, lg.cst->Mt, A.p, op->Lbuf,
                                   op->Rbuf, lg.cnt, st));
    HPS_TRY(run_gj_x(op, lg.gj, st));
    HPS_TRY(run_gemm_x(op, lg.gemmY, st, 0));
    HPS_TRY(run_gemm_x(op, lg.gemmT, st, 0));
  }
  for (Level& L : A.levels) {
    HPS_TRY(run_copy_x(op, L.pcols, 0, A.Tall, A.Tall, nullptr, st));
    HPS_TRY(run_gemm_x(op, L.gcols, st, 0));
    HPS_TRY(run_copy_x(op, L.prows, 0, A.Tall, A.Tall, nullptr, st));
    HPS_TRY(run_gemm_x(op, L.grows, st, 0));
    HPS_TRY(run_copy_x(op, L.assemble, 0, A.Wall, A.Tall, nullptr, st));
    for (const GJPlan& gj : L.gjs) HPS_TRY(run_gj_x(op, gj, st));
    HPS_TRY(run_gemm_x(op, L.gemmS, st, 0));
    HPS_TRY(run_gemm_x(op, L.gemmT, st, 0));
  }
  return HPS_OK;
}

int run_adaptive_solve_chunk(hps_op* op, AdaptivePlan& A, const double* bdry, const double* srcp, double* u, int nrhs,
                             hipStream_t st) {
  const long long nl = op->nl;
  const int npts = op->npts, NR = op->NR;
  const long long field = nl * npts;
  Node& root = A.nodes[0];
  HPS_HIP_TRY(hipMemcpyAsync(root.g, bdry, sizeof(double) * nrhs * root.n, hipMemcpyDeviceToDevice, st));
  if (srcp) {
    HPS_TRY(adaptive_permute_launch(srcp, A.srcslot, A.d_slot_dfs, npts, nl, nrhs, field, field, st));
    HPS_TRY(leaf_gather_int_launch(A.srcslot, op->cst->Ii, op->ni, npts, nl, nrhs, NR, op->fint, st));
    for (LeafGroup& lg : A.groups) {
      HPS_TRY(run_gemm_x(op, lg.gemmV, st, nrhs));
      HPS_TRY(run_gemm_x(op, lg.gemmH, st, nrhs));
    }
    for (Level& L : A.levels) {
      HPS_TRY(run_copy_x(op, L.uprows, nrhs, A.Vall, A.Vall, nullptr, st));
      HPS_TRY(run_gemm_x(op, L.guprows, st, nrhs));
      HPS_TRY(run_copy_x(op, L.uphint, nrhs, A.Vall, A.Vall, nullptr, st));
      HPS_TRY(run_copy_x(op, L.uphext, nrhs, A.Vall, A.Vall, nullptr, st));
      HPS_TRY(run_gemm_x(op, L.gemmGt, st, nrhs));
      HPS_TRY(run_gemm_x(op, L.gemmH, st, nrhs));
    }
  } else {
    for (Node& nd : A.nodes)
      if (!nd.leaf) HPS_HIP_TRY(hipMemsetAsync(nd.gt, 0, sizeof(double) * NR * nd.m, st));
  }
  for (auto it = A.levels.rbegin(); it != A.levels.rend(); ++it) {
    Level& L = *it;
    HPS_TRY(run_gemm_x(op, L.gemmDown, st, nrhs));
    HPS_TRY(run_copy_x(op, L.downgp, nrhs, A.Vall, A.Vall, nullptr, st));
    HPS_TRY(run_copy_x(op, L.downg, nrhs, A.Vall, A.Vall, nullptr, st));
    HPS_TRY(run_gemm_x(op, L.gdown, st, nrhs));
  }
  HPS_TRY(leaf_out_launch(op->Y, op->cst->P, A.gleaf, srcp ? A.vleaf : nullptr, op->cst->Ii, op->cst->Ie, op->ni,
                          op->ne, op->nb, npts, nl, nrhs, NR, A.uslot, st, 0));
  return adaptive_permute_launch(A.uslot, u, A.d_dfs_slot, npts, nl, nrhs, field, field, st);
}

int read_leaves(const int* leaves, long long n, std::set<Key>& out) {
  out.clear();
  for (long long i = 0; i < n; ++i) {
    Key k = {leaves[4 * i], leaves[4 * i + 1], leaves[4 * i + 2], leaves[4 * i + 3]};
    if (!out.insert(k).second) { set_error("adaptive tree: a leaf is listed twice"); return HPS_EINVAL; }
  }
  return HPS_OK;
}

long long write_leaves(const std::vector<Key>& dfs, int* out, long long cap) {
  if ((long long)dfs.size() > cap || !out) return (long long)dfs.size();
  for (size_t i = 0; i < dfs.size(); ++i)
    for (int a = 0; a < 4; ++a) out[4 * i + a] = dfs[i][a];
  return (long long)dfs.size();
}

}  // namespace

void adaptive_free(AdaptivePlan* A) { delete A; }

int adaptive_solve(hps_op* op, const double* bdry, const double* srcp, double* u, int nrhs, hipStream_t st) {
  AdaptivePlan& A = *op->ad;
  const long long field = op->nl * op->npts;
  for (int r0 = 0; r0 < nrhs; r0 += op->NR) {
    const int k = std::min(op->NR, nrhs - r0);
    HPS_TRY(run_adaptive_solve_chunk(op, A, bdry + r0 * A.root_n, srcp ? srcp + r0 * field : nullptr,
                                     u + r0 * field, k, st));
  }
  return HPS_OK;
}

long long adaptive_root_n(const hps_op* op) { return op->ad ? op->ad->root_n : 0; }

}  // namespace hps

using namespace hps;

extern "C" {

int hps_build_adaptive(const hps_atree_t* tree, int p, const double* coeffs, int flags, void* stream,
                       hps_op_t** out) {
  if (!tree || !coeffs || !out || !tree->leaves || tree->n_leaves < 1) {
    set_error("tree, its leaves, coeffs and out must be non-NULL");
    return HPS_EINVAL;
  }
  *out = nullptr;
  if (p < 4 || p > 16) { set_error("p must be in [4, 16]"); return HPS_EINVAL; }
  if (!(tree->hi > tree->lo) || !std::isfinite(tree->lo) || !std::isfinite(tree->hi)) {
    set_error("the cube needs lo < hi");
    return HPS_EINVAL;
  }
  if (flags & ~HPS_FLAG_TIMING) {
    set_error("adaptive operators take no flags but HPS_FLAG_TIMING");
    return HPS_EUNSUPPORTED;
  }
  std::set<Key> leaves;
  HPS_TRY(read_leaves(tree->leaves, tree->n_leaves, leaves));
  std::vector<Key> dfs;
  if (!dfs_order(leaves, dfs)) {
    set_error("adaptive tree: the leaves do not tile the cube (levels 0..20, coordinates in range, no overlaps)");
    return HPS_EINVAL;
  }
  for (long long i = 0; i < tree->n_leaves; ++i) {
    const Key k = {tree->leaves[4 * i], tree->leaves[4 * i + 1], tree->leaves[4 * i + 2], tree->leaves[4 * i + 3]};
    if (k != dfs[i]) { set_error("adaptive tree: leaves must be listed in depth-first order"); return HPS_EINVAL; }
  }
  if (dfs.size() == 1) { set_error("adaptive tree: at least one merge (the root must be split)"); return HPS_EINVAL; }
  if (!unbalanced(dfs).empty()) {
    set_error("adaptive tree: level restriction violated (face neighbours more than one level apart)");
    return HPS_EINVAL;
  }
  hps_op* op = new hps_op();
  op->ad = new AdaptivePlan();
  AdaptivePlan& A = *op->ad;
  A.lo = tree->lo;
  A.hi = tree->hi;
  A.p = p;
  A.q = p - 2;
  A.q2 = A.q * A.q;
  op->p = p;
  op->d = 3;
  op->nd = 8;
  op->flags = flags;
  op->nl = (long long)dfs.size();
  const LeafOps& o = leaf_ops(3, p);
  op->npts = o.npts;
  op->ni = o.n_i;
  op->ne = o.n_e;
  op->nb = o.n_b;
  op->stream = (hipStream_t)stream;
  int rc = build_structure(A, dfs);
  if (rc == HPS_OK && A.max_m > 16384) {
    set_error("adaptive tree: a merge matrix D exceeds the Gauss-Jordan limit (m = 16384)");
    rc = HPS_EUNSUPPORTED;
  }
  if (rc == HPS_OK) rc = plan_adaptive(op, A);
  if (rc == HPS_OK) rc = run_adaptive_build(op, A, coeffs, (hipStream_t)stream);
  if (rc == HPS_OK) {
    int flag = 0;
    if (hipMemcpyAsync(&flag, op->flag, sizeof(int), hipMemcpyDeviceToHost, (hipStream_t)stream) != hipSuccess ||
        hipStreamSynchronize((hipStream_t)stream) != hipSuccess) {
      set_error("device error during the adaptive build");
      rc = HPS_EDEVICE;
    } else if (flag) {
      set_error("adaptive build: zero or non-finite pivot in a leaf or merge inverse");
      rc = HPS_ESINGULAR;
    }
  }
  if (rc != HPS_OK) {
    hps_free(op);
    return rc;
  }
  *out = op;
  return HPS_OK;
}

long long hps_adaptive_root_size(const hps_op_t* op, long long* d_size) {
  if (!op || !op->ad) { set_error("not an adaptive operator"); return -HPS_EINVAL; }
  if (d_size) *d_size = op->ad->nodes[0].m;
  return op->ad->root_n;
}

int hps_adaptive_points(const hps_atree_t* tree, int p, int which, double* out) {
  if (!tree || !tree->leaves || tree->n_leaves < 1 || !out) { set_error("bad arguments"); return HPS_EINVAL; }
  if (p < 4 || p > 16 || which < 0 || which > 2) { set_error("p in [4, 16], which in 0..2"); return HPS_EINVAL; }
  std::set<Key> leaves;
  HPS_TRY(read_leaves(tree->leaves, tree->n_leaves, leaves));
  std::vector<Key> dfs;
  if (!dfs_order(leaves, dfs)) { set_error("adaptive tree: the leaves do not tile the cube"); return HPS_EINVAL; }
  const LeafOps& o = leaf_ops(3, p);
  const int np = o.npts;
  const double L = tree->hi - tree->lo;
  auto box_points = [&](const Key& k, double* dst) {
    const double r = L / 2.0 / (double)(1LL << k[0]);
    for (int j = 0; j < np; ++j) {
      const int c[3] = {j % p, (j / p) % p, j / (p * p)};
      for (int a = 0; a < 3; ++a) dst[3 * j + a] = tree->lo + 2.0 * r * k[1 + a] + (o.cheb[c[a]] + 1.0) * r;
    }
  };
  if (which == 0) {
    for (size_t i = 0; i < dfs.size(); ++i) box_points(dfs[i], out + i * 3 * np);
    return HPS_OK;
  }
  if (which == 1) {
    const MergeGeom& G = merge_geom(3);
    for (size_t i = 0; i < dfs.size(); ++i)
      for (int c = 0; c < 8; ++c) box_points(child_key(dfs[i], c, G), out + (i * 8 + c) * 3 * np);
    return HPS_OK;
  }
  if (dfs.size() == 1) { set_error("adaptive tree: at least one merge"); return HPS_EINVAL; }
  if (!unbalanced(dfs).empty()) { set_error("adaptive tree: level restriction violated"); return HPS_EINVAL; }
  AdaptivePlan A;
  A.lo = tree->lo;
  A.hi = tree->hi;
  A.p = p;
  A.q = p - 2;
  A.q2 = A.q * A.q;
  HPS_TRY(build_structure(A, dfs));
  const double h = L / (double)(1LL << A.maxl);
  const int q = A.q;
  long long k = 0;
  for (const Panel& pn : A.nodes[0].bdry) {
    const FaceDesc& fd = merge_geom(3).faces[pn.face];
    for (int b = 0; b < q; ++b)
      for (int a = 0; a < q; ++a, ++k) {
        out[3 * k + pn.axis] = tree->lo + h * (double)pn.plane;
        out[3 * k + fd.tang[0]] = tree->lo + h * (pn.a0 + (o.gl[a] + 1.0) * pn.s / 2.0);
        out[3 * k + fd.tang[1]] = tree->lo + h * (pn.b0 + (o.gl[b] + 1.0) * pn.s / 2.0);
      }
  }
  return HPS_OK;
}

long long hps_adaptive_root_points(const hps_atree_t* tree, int p) {
  if (!tree || !tree->leaves || tree->n_leaves < 2) { set_error("bad arguments"); return -HPS_EINVAL; }
  std::set<Key> leaves;
  if (read_leaves(tree->leaves, tree->n_leaves, leaves) != HPS_OK) return -HPS_EINVAL;
  std::vector<Key> dfs;
  if (!dfs_order(leaves, dfs)) { set_error("adaptive tree: the leaves do not tile the cube"); return -HPS_EINVAL; }
  if (!unbalanced(dfs).empty()) { set_error("adaptive tree: level restriction violated"); return -HPS_EINVAL; }
  AdaptivePlan A;
  A.lo = tree->lo;
  A.hi = tree->hi;
  A.p = p;
  A.q = p - 2;
  A.q2 = A.q * A.q;
  if (build_structure(A, dfs) != HPS_OK) return -HPS_EINVAL;
  return A.root_n;
}

long long hps_adaptive_split(const int* leaves, long long n, const int* split, int* out, long long cap) {
  if (!leaves || !split || n < 1) { set_error("bad arguments"); return -HPS_EINVAL; }
  std::set<Key> ls;
  if (read_leaves(leaves, n, ls) != HPS_OK) return -HPS_EINVAL;
  const MergeGeom& G = merge_geom(3);
  for (long long i = 0; i < n; ++i)
    if (split[i]) {
      const Key k = {leaves[4 * i], leaves[4 * i + 1], leaves[4 * i + 2], leaves[4 * i + 3]};
      ls.erase(k);
      for (int c = 0; c < 8; ++c) ls.insert(child_key(k, c, G));
    }
  std::vector<Key> dfs;
  if (!dfs_order(ls, dfs)) { set_error("adaptive tree: the leaves do not tile the cube"); return -HPS_EINVAL; }
  return write_leaves(dfs, out, cap);
}

long long hps_adaptive_union(const int* a, long long na, const int* b, long long nb, int* out, long long cap) {
  if (!a || !b || na < 1 || nb < 1) { set_error("bad arguments"); return -HPS_EINVAL; }
  std::set<Key> la, lb;
  if (read_leaves(a, na, la) != HPS_OK || read_leaves(b, nb, lb) != HPS_OK) return -HPS_EINVAL;
  std::vector<Key> da, db;
  std::set<Key> ia, ib;
  if (!dfs_order(la, da, &ia) || !dfs_order(lb, db, &ib)) {
    set_error("adaptive tree: the leaves do not tile the cube");
    return -HPS_EINVAL;
  }
  std::set<Key> internal = ia;
  internal.insert(ib.begin(), ib.end());
  std::set<Key> u;
  const MergeGeom& G = merge_geom(3);
  for (const Key& k : internal)
    for (int c = 0; c < 8; ++c) {
      const Key ck = child_key(k, c, G);
      if (!internal.count(ck)) u.insert(ck);
    }
  if (internal.empty()) u.insert(Key{0, 0, 0, 0});
  std::vector<Key> dfs;
  if (!dfs_order(u, dfs)) { set_error("adaptive tree: union failed"); return -HPS_EINVAL; }
  return write_leaves(dfs, out, cap);
}

long long hps_adaptive_balance(const int* leaves, long long n, int* out, long long cap) {
  if (!leaves || n < 1) { set_error("bad arguments"); return -HPS_EINVAL; }
  std::set<Key> ls;
  if (read_leaves(leaves, n, ls) != HPS_OK) return -HPS_EINVAL;
  const MergeGeom& G = merge_geom(3);
  std::vector<Key> dfs;
  for (;;) {
    if (!dfs_order(ls, dfs)) { set_error("adaptive tree: the leaves do not tile the cube"); return -HPS_EINVAL; }
    const std::vector<int> sp = unbalanced(dfs);
    if (sp.empty()) break;
    for (int i : sp) {
      ls.erase(dfs[i]);
      for (int c = 0; c < 8; ++c) ls.insert(child_key(dfs[i], c, G));
    }
  }
  return write_leaves(dfs, out, cap);
}

int hps_adaptive_check(int p, long long nl, const double* f0, const double* f1, double eps, int* split,
                       void* stream) {
  if (p < 4 || p > 16 || nl < 1 || !f0 || !f1 || !split || !(eps > 0.0)) {
    set_error("p in [4, 16], nl >= 1, non-NULL arrays, eps > 0");
    return HPS_EINVAL;
  }
  if (nl > 65535) { set_error("at most 65535 leaves per check"); return HPS_EINVAL; }
  const LeafOps& o = leaf_ops(3, p);
  std::vector<double> ylo(p), yhi(p);
  for (int i = 0; i < p; ++i) { ylo[i] = (o.cheb[i] - 1.0) / 2.0; yhi[i] = (o.cheb[i] + 1.0) / 2.0; }
  std::vector<double> E = interp1d(o.cheb, ylo), E1 = interp1d(o.cheb, yhi);
  E.insert(E.end(), E1.begin(), E1.end());  // [2][p][p] row-major
  hipStream_t st = (hipStream_t)stream;
  double *dE = nullptr, *derr = nullptr;
  HPS_HIP_TRY(hipMalloc(&dE, sizeof(double) * (E.size() + 2 * nl)));
  derr = dE + E.size();
  int rc = HPS_OK;
  std::vector<double> res(2 * nl);
  if (hipMemcpyAsync(dE, E.data(), sizeof(double) * E.size(), hipMemcpyHostToDevice, st) != hipSuccess) rc = HPS_EDEVICE;
  if (rc == HPS_OK) rc = adaptive_check_launch(f0, f1, dE, p, nl, derr, derr + nl, st);
  if (rc == HPS_OK && (hipMemcpyAsync(res.data(), derr, sizeof(double) * 2 * nl, hipMemcpyDeviceToHost, st) != hipSuccess ||
                       hipStreamSynchronize(st) != hipSuccess)) {
    set_error("device error in the refinement check");
    rc = HPS_EDEVICE;
  }
  (void)hipFree(dE);
  if (rc != HPS_OK) return rc;
  double fnorm = 0.0;
  for (long long i = 0; i < nl; ++i) fnorm = std::max(fnorm, res[nl + i]);
  for (long long i = 0; i < nl; ++i) split[i] = (fnorm > 0.0 && !(res[i] < eps * fnorm)) ? 1 : 0;
  return HPS_OK;
}

}  // extern "C"
