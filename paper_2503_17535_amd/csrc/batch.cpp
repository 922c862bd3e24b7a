// Batched solve over several resident operators: the solves of every operator
// in a batch run as one sequence of launches, each launch covering the same
// pass stage of all of them (a ragged work list over operator, tree level,
// node and right-hand side).
//
// Stage order (S = deepest tree in the batch):
//   root boundary data            one gather launch
//   leaf particular solutions      one leaf_src launch, one GEMM (h = Q_i v)
//   upward source pass, step s     gather h_int, GEMM g~ = -Z h_int, GEMM h_parent
//     (s = 0..S-1; an operator of depth L takes part with tree level L-1-s)
//   downward pass, step s          GEMM g_int = S g + g~, gather children's g
//     (s = 0..S-1; tree level s of every operator deeper than s)
//   leaf output                    one leaf_out launch
// so a batch costs 5S + 4 launches whatever the number of operators and
// requests.  The descriptors of one batch are packed into one pinned host
// block and uploaded with a single copy; two such blocks alternate so that
// the host prepares the next batch while the device runs the current one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <set>
#include <string>
#include <vector>

#include "op.hpp"

namespace hps {
int block_copy_multi_launch(const CopyJob* dev_jobs, int njobs, long long nblocks, hipStream_t st);
int root_gather_multi_launch(const LeafJob* dev_jobs, int njobs, int max_nb0, hipStream_t st);
int leaf_src_multi_launch(const LeafJob* dev_jobs, int njobs, long long nblocks, int max_ni, hipStream_t st);
int leaf_out_multi_launch(const LeafJob* dev_jobs, int njobs, long long nblocks, int max_nb, hipStream_t st);
}  // namespace hps

struct hps_batcher {
  hipEvent_t done[2] = {nullptr, nullptr};
  bool used[2] = {false, false};
  char* host[2] = {nullptr, nullptr};
  char* dev[2] = {nullptr, nullptr};
  size_t cap[2] = {0, 0};
  int slot = 0;
};

namespace hps {
namespace {

enum class Kind { Root, LeafSrc, LeafOut, Gemm, Copy, Zero };

struct Launch {
  Kind kind;
  size_t off = 0;          // byte offset of the descriptor array in the block
  int count = 0;           // number of descriptors
  long long nblocks = 0;   // grid size
  long long nrblocks = 0;  // split-K reduction grid (GEMM)
  int aux = 0;             // max n_i / n_b / root size
  double* zdst = nullptr;  // Zero: memset target
  size_t zbytes = 0;
};

struct Packer {
  std::vector<char> buf;
  template <class T>
  size_t put(const std::vector<T>& v) {
    const size_t off = (buf.size() + 255) & ~(size_t)255;
    buf.resize(off + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(buf.data() + off, v.data(), v.size() * sizeof(T));
    return off;
  }
};

CopyJob copy_job(const hps_op* op, const CopyCall& c, int ncols, long long batch, double* dst, long long dst_stride,
                 const double* s0, long long s0_stride, const double* s1, long long s1_stride) {
  CopyJob j;
  std::memset(&j, 0, sizeof(j));
  j.ops = op->dops;
  j.items = op->ditems;
  j.tasks = op->dtasks + c.first_task;
  j.ntasks = c.ntasks;
  j.ncols_rt = ncols;
  j.batch = batch;
  j.dst = dst;
  j.dst_stride = dst_stride;
  j.src0 = s0;
  j.s0_stride = s0_stride;
  j.src1 = s1;
  j.s1_stride = s1_stride;
  return j;
}

void add_copy_launch(Packer& pk, std::vector<Launch>& out, std::vector<CopyJob>& jobs) {
  long long nb = 0;
  std::vector<CopyJob> keep;
  for (auto& j : jobs) {
    if (j.ntasks <= 0 || j.batch <= 0) continue;
    j.first_block = nb;
    nb += (long long)j.ntasks * j.batch;
    keep.push_back(j);
  }
  if (keep.empty()) return;
  Launch l{Kind::Copy};
  l.off = pk.put(keep);
  l.count = (int)keep.size();
  l.nblocks = nb;
  out.push_back(l);
}

void add_gemm_launch(Packer& pk, std::vector<Launch>& out, std::vector<GemmGroup>& groups) {
  if (groups.empty()) return;
  const long long nb = gemm_prepare(groups);
  if (nb <= 0) return;
  Launch l{Kind::Gemm};
  l.off = pk.put(groups);
  l.count = (int)groups.size();
  l.nblocks = nb;
  l.nrblocks = gemm_rblocks(groups);
  out.push_back(l);
}

void append_groups(const hps_op* op, const GemmCall& c, int nrhs, std::vector<GemmGroup>& dst) {
  for (int i = 0; i < c.count; ++i) {
    GemmGroup g = op->hgroups[c.first + i];
    g.N = nrhs;
    dst.push_back(g);
  }
}

int grow(hps_batcher* b, int s, size_t bytes) {
  if (bytes <= b->cap[s]) return HPS_OK;
  size_t cap = std::max(bytes, 2 * b->cap[s]);
  cap = (cap + 65535) & ~(size_t)65535;
  if (b->host[s]) (void)hipHostFree(b->host[s]);
  if (b->dev[s]) (void)hipFree(b->dev[s]);
  b->host[s] = nullptr;
  b->dev[s] = nullptr;
  b->cap[s] = 0;
  HPS_HIP_TRY(hipHostMalloc((void**)&b->host[s], cap, hipHostMallocDefault));
  HPS_HIP_TRY(hipMalloc((void**)&b->dev[s], cap));
  b->cap[s] = cap;
  return HPS_OK;
}

}  // namespace
}  // namespace hps

extern "C" {

int hps_batcher_create(hps_batcher_t** out) {
  if (!out) {
    hps::set_error("out must be non-NULL");
    return HPS_EINVAL;
  }
  *out = nullptr;
  hps_batcher* b = new hps_batcher();
  for (int s = 0; s < 2; ++s) {
    if (hipEventCreateWithFlags(&b->done[s], hipEventDisableTiming) != hipSuccess) {
      hps::set_error("hipEventCreate failed");
      hps_batcher_free(b);
      return HPS_EDEVICE;
    }
  }
  *out = b;
  return HPS_OK;
}

void hps_batcher_free(hps_batcher_t* b) {
  if (!b) return;
  for (int s = 0; s < 2; ++s) {
    if (b->done[s]) {
      if (b->used[s]) (void)hipEventSynchronize(b->done[s]);
      (void)hipEventDestroy(b->done[s]);
    }
    if (b->host[s]) (void)hipHostFree(b->host[s]);
    if (b->dev[s]) (void)hipFree(b->dev[s]);
  }
  delete b;
}

int hps_solve_batch(hps_batcher_t* b, const hps_batch_item_t* items, int nitems, void* stream) {
  using namespace hps;
  if (!b || (nitems > 0 && !items) || nitems < 0) {
    set_error("batcher and items must be non-NULL, nitems >= 0");
    return HPS_EINVAL;
  }
  if (nitems == 0) return HPS_OK;
  hipError_t pending = hipGetLastError();
  if (pending != hipSuccess) {
    set_error(std::string("earlier device error: ") + hipGetErrorString(pending));
    return HPS_EDEVICE;
  }
  hipStream_t st = (hipStream_t)stream;
  // validate
  std::set<const hps_op*> seen;
  int S = 0;
  for (int i = 0; i < nitems; ++i) {
    const hps_batch_item_t& it = items[i];
    const hps_op* op = it.op;
    if (!op) { set_error("batch item " + std::to_string(i) + ": op is NULL"); return HPS_EINVAL; }
    if (op->d != 2) { set_error("batched solve supports 2D operators"); return HPS_EUNSUPPORTED; }
    if (op->sub) { set_error("batched solve needs every leaf operator resident (not subtree recomputation)"); return HPS_EUNSUPPORTED; }
    if (op->iti || op->fp64_dropped || op->ad) { set_error("batched solve serves fp64 DtN operators"); return HPS_EUNSUPPORTED; }
    if (it.nrhs < 1 || it.nrhs > std::min(op->NR, kBatchMaxRhs)) {
      set_error("batch item " + std::to_string(i) + ": nrhs must be in 1..16");
      return HPS_EINVAL;
    }
    if (!seen.insert(op).second) {
      set_error("batch item " + std::to_string(i) + ": an operator may appear once per batch (merge its rhs)");
      return HPS_EINVAL;
    }
    for (int j = 0; j < it.nrhs; ++j)
      if (!it.bdry[j] || !it.u[j]) {
        set_error("batch item " + std::to_string(i) + ": bdry and u must be non-NULL for every rhs");
        return HPS_EINVAL;
      }
    S = std::max(S, op->tree.depth);
  }

  Packer pk;
  std::vector<Launch> plan;
  // jobs of the leaf kernels
  std::vector<LeafJob> all, withsrc;
  std::vector<char> has_src(nitems, 0);
  int max_nb0 = 0, max_ni = 0, max_nb = 0;
  for (int i = 0; i < nitems; ++i) {
    const hps_batch_item_t& it = items[i];
    hps_op* op = it.op;
    LeafJob J;
    std::memset(&J, 0, sizeof(J));
    J.LU = op->LU; J.Y = op->Y; J.P = op->cst->P; J.g = op->g[op->tree.depth];
    J.perm = op->perm; J.pos = op->pos; J.Ii = op->cst->Ii; J.Ie = op->cst->Ie;
    J.v = op->v; J.g0 = op->g[0];
    J.NI = op->ni; J.NE = op->ne; J.NB = op->nb; J.npts = op->npts; J.nrhs = it.nrhs; J.NRcap = op->NR;
    J.nb0 = op->nbl[0]; J.nl = op->nl;
    for (int j = 0; j < it.nrhs; ++j) {
      J.bdry[j] = it.bdry[j];
      J.src[j] = it.src[j];
      J.u[j] = it.u[j];
      if (J.src[j]) has_src[i] = 1;
    }
    max_nb0 = std::max(max_nb0, J.nb0);
    max_ni = std::max(max_ni, J.NI);
    max_nb = std::max(max_nb, J.NB);
    if (has_src[i]) withsrc.push_back(J);
    if (!has_src[i]) J.v = nullptr;
    all.push_back(J);
  }
  {
    Launch l{Kind::Root};
    l.off = pk.put(all);
    l.count = (int)all.size();
    l.aux = max_nb0;
    plan.push_back(l);
  }
  if (!withsrc.empty()) {
    long long nb = 0;
    for (auto& J : withsrc) { J.first_block = nb; nb += J.nl; }
    Launch l{Kind::LeafSrc};
    l.off = pk.put(withsrc);
    l.count = (int)withsrc.size();
    l.nblocks = nb;
    l.aux = max_ni;
    plan.push_back(l);
    std::vector<GemmGroup> gs;
    for (int i = 0; i < nitems; ++i)
      if (has_src[i]) append_groups(items[i].op, items[i].op->gemmHleaf, items[i].nrhs, gs);
    add_gemm_launch(pk, plan, gs);
  }
  // operators without a source: g~ = 0 on every level
  for (int i = 0; i < nitems; ++i) {
    if (has_src[i]) continue;
    hps_op* op = items[i].op;
    for (auto& P : op->levels) {
      Launch l{Kind::Zero};
      l.zdst = P.gt;
      l.zbytes = sizeof(double) * P.nm * op->NR * P.m;
      plan.push_back(l);
    }
  }
  // upward source pass, aligned at the leaves
  for (int s = 0; s < S; ++s) {
    std::vector<CopyJob> cj;
    std::vector<GemmGroup> gt, hp;
    for (int i = 0; i < nitems; ++i) {
      hps_op* op = items[i].op;
      const int L = op->tree.depth;
      if (!has_src[i] || L <= s) continue;
      const int lev = L - 1 - s;
      LevelPlan& P = op->levels[lev];
      cj.push_back(copy_job(op, P.copyHint, items[i].nrhs, P.nm, P.hint, (long long)op->NR * P.m, op->h[lev + 1],
                            (long long)op->nd * op->NR * P.nbc, nullptr, 0));
      append_groups(op, P.gemmGt, items[i].nrhs, gt);
      if (lev > 0) append_groups(op, P.gemmHp, items[i].nrhs, hp);
    }
    add_copy_launch(pk, plan, cj);
    add_gemm_launch(pk, plan, gt);
    add_gemm_launch(pk, plan, hp);
  }
  // downward pass, aligned at the root
  for (int s = 0; s < S; ++s) {
    std::vector<GemmGroup> dn;
    std::vector<CopyJob> cj;
    for (int i = 0; i < nitems; ++i) {
      hps_op* op = items[i].op;
      if (op->tree.depth <= s) continue;
      LevelPlan& P = op->levels[s];
      append_groups(op, P.gemmDown, items[i].nrhs, dn);
      cj.push_back(copy_job(op, P.copyGchild, items[i].nrhs, P.nm, op->g[s + 1], (long long)op->nd * op->NR * P.nbc,
                            op->g[s], (long long)op->NR * P.nbp, P.gint, (long long)op->NR * P.m));
    }
    add_gemm_launch(pk, plan, dn);
    add_copy_launch(pk, plan, cj);
  }
  {
    long long nb = 0;
    for (auto& J : all) { J.first_block = nb; nb += J.nl; }
    Launch l{Kind::LeafOut};
    l.off = pk.put(all);
    l.count = (int)all.size();
    l.nblocks = nb;
    l.aux = max_nb;
    plan.push_back(l);
  }

  // upload the descriptors of this batch into the next free block
  const int s = b->slot;
  if (b->used[s]) HPS_HIP_TRY(hipEventSynchronize(b->done[s]));
  HPS_TRY(grow(b, s, pk.buf.size()));
  std::memcpy(b->host[s], pk.buf.data(), pk.buf.size());
  HPS_HIP_TRY(hipMemcpyAsync(b->dev[s], b->host[s], pk.buf.size(), hipMemcpyHostToDevice, st));
  char* base = b->dev[s];
  for (const Launch& l : plan) {
    switch (l.kind) {
      case Kind::Root:
        HPS_TRY(root_gather_multi_launch((const LeafJob*)(base + l.off), l.count, l.aux, st));
        break;
      case Kind::LeafSrc:
        HPS_TRY(leaf_src_multi_launch((const LeafJob*)(base + l.off), l.count, l.nblocks, l.aux, st));
        break;
      case Kind::LeafOut:
        HPS_TRY(leaf_out_multi_launch((const LeafJob*)(base + l.off), l.count, l.nblocks, l.aux, st));
        break;
      case Kind::Gemm:
        HPS_TRY(gemm_launch((const GemmGroup*)(base + l.off), l.count, l.nblocks, l.nrblocks, false, false, st, 0));
        break;
      case Kind::Copy:
        HPS_TRY(block_copy_multi_launch((const CopyJob*)(base + l.off), l.count, l.nblocks, st));
        break;
      case Kind::Zero:
        HPS_HIP_TRY(hipMemsetAsync(l.zdst, 0, l.zbytes, st));
        break;
    }
  }
  HPS_HIP_TRY(hipEventRecord(b->done[s], st));
  b->used[s] = true;
  b->slot ^= 1;
  return HPS_OK;
}

}  // extern "C"
