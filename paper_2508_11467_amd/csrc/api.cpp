// C ABI of the bidiagonal divide-and-conquer SVD: argument checks, the merge
// tree plan, the workspace, and the level-by-level launch sequence.
//
// The host only builds the plan (the recursive split of Section 4.2.1 at
// k = floor(m/2) down to leaves of at most leaf_size rows) and enqueues
// kernels: every size that depends on the data (how many values survive
// deflation, how many roots, how many rotations) is written and read on the
// device, so a whole solve is one stream of launches with no host
// synchronisation and no matrix traffic between host and device.  Nodes of
// equal height in the tree -- across all problems of a batch -- form one
// level and run in the same launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "bdc.h"
#include "bdc_internal.h"
#include "backtr.h"
#include "plan.h"
#include "crt.h"
#include "qr.h"
#include "gebrd.h"

using namespace bdc;

namespace {

constexpr uint32_t kMagic = 0xBDC05EEDu;
constexpr int kQrDefaultBlock = 32;  // panel width of bdc_geqrf when block = 0
constexpr int kQrMaxGrid = 2048;     // workgroups of a QR panel, at most

enum Kind {
  kReset = 0, kLeaf, kPrep, kRotate, kGather, kStart, kSecular, kLowner, kVectors, kOrder, kUpdate, kUpdateOz,
  kUpdateCrt, kFinal, kKinds
};
const char* kKindNames[kKinds] = {"reset", "leaf", "deflate", "rotate", "gather", "start", "secular",
                                  "lowner", "vectors", "order", "update_gemm", "update_ozaki", "update_crt",
                                  "final"};

struct Level {
  int nnodes = 0;
  int max_m = 0;
  NodeDesc* dev = nullptr;
};

struct Plan {
  std::vector<int64_t> sizes;
  int leaf = 0;
  int64_t total_n = 0, total_n2 = 0;
  int nleaves = 0;
  LeafDesc* dev_leaves = nullptr;
  std::vector<Level> levels;
  std::vector<NodeDesc> host_nodes;
  int nnodes = 0;
  int nprob = 0;
  int64_t* dev_prob = nullptr;  // n, vec, mat, uitem_off, vitem_off (nprob each)
  int32_t* dev_uprob = nullptr;  // final-pass work item -> problem (U, V^T)
  int32_t* dev_vprob = nullptr;
  int64_t total_cols = 0, total_tiles = 0;  // final-pass work items of U and of V^T
  int root_id0 = -1;  // node id of the first problem's root merge
  void* block = nullptr;
};

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct bdc_handle_s {
  uint32_t magic = kMagic;
  int device = 0;
  bdc_options_t opt{};
  void* arena = nullptr;
  size_t arena_bytes = 0;
  int64_t cap_n = -1, cap_n2 = -1;
  int cap_nodes = -1;
  Work w{};
  Plan plan;
  bool plan_valid = false;
  hipStream_t last_stream = nullptr;
  bool have_call = false;
  // captured launch sequence of the current plan and buffers
  hipStream_t cap_stream = nullptr;
  // second stream of the captured sequence (each level's rotations and
  // gather beside its secular solve, Löwner z and vectors) and its fork and
  // join events
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipGraphExec_t gexec = nullptr;
  const void* gkey[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
  // learned start: FP32 parameters and Adam moments (one allocation), the
  // per-workgroup gradient partials of a training step, and harvest buffers
  void* oz_arena = nullptr;  // split-precision slice planes (single-problem solves)
  size_t oz_bytes = 0;
  void* bt_arena = nullptr;   // back-transformation scratch (grown on demand)
  size_t bt_bytes = 0;
  void* bt_fixed = nullptr;   // this device's fixed scratch (allocation-free back-transformation)
  void* qr_sync = nullptr;    // QR panel: grid-barrier state and partial sums
  size_t qr_sync_size = 0;
  void* brd_work = nullptr;   // bidiagonal reduction: panel buffers, barrier state, partial sums
  size_t brd_bytes = 0;
  void* crt_arena = nullptr;  // int8 residue planes (single-problem solves)
  size_t crt_bytes = 0;
  int64_t crt_n = -1;         // problem size the residue planes are laid out for
  int last_split_min_n = INT32_MAX;  // split threshold of the last solve (statistics)
  float* mlp = nullptr;  // params | m | v
  unsigned short* mlp_pk = nullptr;  // inference layout, repacked at each learned solve
  int adam_t = 0;
  float* part = nullptr;  // parts x params | parts losses
  int part_cap = 0;
  Harvest hv{};
  bool harvest = false;
  Tuning tune{96, 0, 1024, 512, kSecLanesMaxN};
};

namespace {

struct DeviceGuard {
  int old = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&old) != hipSuccess) old = -1;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (old >= 0) (void)hipSetDevice(old);
  }
};

bool valid(bdc_handle_t h) { return h != nullptr && h->magic == kMagic; }

void drop_graph(bdc_handle_t h) {
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  h->gexec = nullptr;
  for (auto& k : h->gkey) k = nullptr;
}

void free_plan(Plan& p) {
  if (p.block) (void)hipFree(p.block);
  p = Plan();
}

int make_plan(bdc_handle_t h, const int64_t* sizes, int64_t batch) {
  const int leaf = h->opt.leaf_size;
  if (h->plan_valid && h->plan.leaf == leaf && (int64_t)h->plan.sizes.size() == batch &&
      std::equal(h->plan.sizes.begin(), h->plan.sizes.end(), sizes))
    return BDC_OK;
  if (h->have_call) (void)hipStreamSynchronize(h->last_stream);
  drop_graph(h);
  free_plan(h->plan);
  h->plan_valid = false;
  Plan p;
  p.sizes.assign(sizes, sizes + batch);
  p.leaf = leaf;
  p.nprob = (int)batch;
  HostPlan hp = build_host_plan(sizes, batch, leaf);
  p.total_n = hp.total_n;
  p.total_n2 = hp.total_n2;
  p.total_cols = hp.total_cols;
  p.total_tiles = hp.total_tiles;
  p.nleaves = (int)hp.leaves.size();
  p.root_id0 = hp.root_id0;
  p.host_nodes = hp.nodes;
  const int id = (int)hp.nodes.size();
  p.nnodes = id;
  const int64_t co = hp.total_cols, to = hp.total_tiles;
  size_t bytes = align_up(sizeof(LeafDesc) * std::max<size_t>(1, hp.leaves.size())) +
                 align_up(sizeof(NodeDesc) * std::max(1, id)) +
                 align_up(sizeof(int64_t) * 5 * std::max<int64_t>(1, batch)) +
                 align_up(sizeof(int32_t) * std::max<int64_t>(1, co)) + align_up(sizeof(int32_t) * std::max<int64_t>(1, to));
  if (hipMalloc(&p.block, bytes) != hipSuccess) return BDC_ERR_NOMEM;
  char* b = (char*)p.block;
  p.dev_leaves = (LeafDesc*)b;
  b += align_up(sizeof(LeafDesc) * std::max<size_t>(1, hp.leaves.size()));
  NodeDesc* nodes_dev = (NodeDesc*)b;
  b += align_up(sizeof(NodeDesc) * std::max(1, id));
  p.dev_prob = (int64_t*)b;
  b += align_up(sizeof(int64_t) * 5 * std::max<int64_t>(1, batch));
  p.dev_uprob = (int32_t*)b;
  b += align_up(sizeof(int32_t) * std::max<int64_t>(1, co));
  p.dev_vprob = (int32_t*)b;
  if ((co > 0 && hipMemcpy(p.dev_uprob, hp.uprob.data(), sizeof(int32_t) * co, hipMemcpyHostToDevice) != hipSuccess) ||
      (to > 0 && hipMemcpy(p.dev_vprob, hp.vprob.data(), sizeof(int32_t) * to, hipMemcpyHostToDevice) != hipSuccess))
    return free_plan(p), BDC_ERR_HIP;
  if (!hp.leaves.empty() && hipMemcpy(p.dev_leaves, hp.leaves.data(), sizeof(LeafDesc) * hp.leaves.size(),
                                      hipMemcpyHostToDevice) != hipSuccess)
    return free_plan(p), BDC_ERR_HIP;
  if (id > 0 && hipMemcpy(nodes_dev, hp.nodes.data(), sizeof(NodeDesc) * id, hipMemcpyHostToDevice) != hipSuccess)
    return free_plan(p), BDC_ERR_HIP;
  if (batch > 0 &&
      hipMemcpy(p.dev_prob, hp.prob.data(), sizeof(int64_t) * 5 * batch, hipMemcpyHostToDevice) != hipSuccess)
    return free_plan(p), BDC_ERR_HIP;
  int off = 0;
  for (size_t hh = 0; hh < hp.level_count.size(); ++hh) {
    Level L;
    L.nnodes = hp.level_count[hh];
    L.max_m = hp.level_max_m[hh];
    L.dev = nodes_dev + off;
    off += L.nnodes;
    p.levels.push_back(L);
  }
  h->plan = std::move(p);
  h->plan_valid = true;
  return BDC_OK;
}

}  // namespace

// Workspace layout: four n x n matrices per problem (Uwork, Vwork, UM, VM),
// the per-position arrays and the node states, carved from `base` in this
// order.  Returns the bytes; with w != NULL the pointers are set.
size_t bdc::work_layout(Work* w, char* base, int64_t tn, int64_t tn2, int nnodes) {
  const size_t N1 = (size_t)std::max<int64_t>(tn, 1), N2 = (size_t)std::max<int64_t>(tn2, 1);
  const size_t nd_ = (size_t)std::max(nnodes, 1);
  size_t off = 0;
  auto take = [&](size_t nbytes) {
    char* r = base + off;
    off += align_up(nbytes);
    return (void*)r;
  };
  Work t{};
  t.Uw = (double*)take(N2 * 8);
  t.Vw = (double*)take(N2 * 8);
  t.UM = (double*)take(N2 * 8);
  t.VM = (double*)take(N2 * 8);
  t.sig = (double*)take(N1 * 8);
  t.ps_d = (double*)take(N1 * 8);
  t.ps_z = (double*)take(N1 * 8);
  t.sd = (double*)take(N1 * 8);
  t.sz = (double*)take(N1 * 8);
  t.dval = (double*)take(N1 * 8);
  t.tau = (double*)take(N1 * 8);
  t.zt = (double*)take(N1 * 8);
  t.rot_cs = (double*)take(2 * N1 * 8);
  t.col = (int32_t*)take(N1 * 4);
  t.ulo = (int32_t*)take(N1 * 4);
  t.uhi = (int32_t*)take(N1 * 4);
  t.vlo = (int32_t*)take(N1 * 4);
  t.vhi = (int32_t*)take(N1 * 4);
  t.ps_c = (int32_t*)take(N1 * 4);
  t.ps_col = (int32_t*)take(N1 * 4);
  t.ps_sup = (int32_t*)take(N1 * 4);
  t.status = (int32_t*)take(N1 * 4);
  t.ps_rot = (int32_t*)take(N1 * 4);
  t.cand = (int32_t*)take(N1 * 4);
  t.scol = (int32_t*)take(N1 * 4);
  t.srot = (int32_t*)take(N1 * 4);
  t.sgrp = (int32_t*)take(N1 * 4);
  t.gsurv = (int32_t*)take(N1 * 4);
  t.dcol = (int32_t*)take(N1 * 4);
  t.drot = (int32_t*)take(N1 * 4);
  t.o = (int32_t*)take(N1 * 4);
  t.iters = (int32_t*)take(N1 * 4);
  t.rot_pos = (int32_t*)take(2 * N1 * 4);
  t.rot_col = (int32_t*)take(2 * N1 * 4);
  t.xs = (float*)take(N1 * 4);
  t.tile_off64 = (int*)take((nd_ + 1) * 4);
  t.tile_off128 = (int*)take((nd_ + 1) * 4);
  t.st = (NodeState*)take(nd_ * sizeof(NodeState));
  t.ctl = (Ctl*)take(sizeof(Ctl));
  t.fin = (int4*)take(2 * N1 * sizeof(int4));
  t.leaf_fl = (unsigned long long*)take(N1 * 8);
  t.sec = (SecCount*)take(nd_ * sizeof(SecCount));
  if (w) {
    w->Uw = t.Uw; w->Vw = t.Vw; w->UM = t.UM; w->VM = t.VM;
    w->sig = t.sig; w->ps_d = t.ps_d; w->ps_z = t.ps_z; w->sd = t.sd; w->sz = t.sz; w->dval = t.dval;
    w->tau = t.tau; w->zt = t.zt; w->rot_cs = t.rot_cs;
    w->col = t.col; w->ulo = t.ulo; w->uhi = t.uhi; w->vlo = t.vlo; w->vhi = t.vhi;
    w->ps_c = t.ps_c; w->ps_col = t.ps_col; w->ps_sup = t.ps_sup; w->status = t.status; w->ps_rot = t.ps_rot;
    w->cand = t.cand; w->scol = t.scol; w->srot = t.srot; w->sgrp = t.sgrp; w->gsurv = t.gsurv;
    w->dcol = t.dcol; w->drot = t.drot; w->o = t.o; w->iters = t.iters; w->rot_pos = t.rot_pos;
    w->rot_col = t.rot_col; w->xs = t.xs; w->tile_off64 = t.tile_off64; w->tile_off128 = t.tile_off128;
    w->st = t.st; w->ctl = t.ctl; w->fin = t.fin; w->leaf_fl = t.leaf_fl; w->sec = t.sec;
  }
  return off;
}

namespace {

int ensure_workspace(bdc_handle_t h, int64_t tn, int64_t tn2, int nnodes) {
  if (tn <= h->cap_n && tn2 <= h->cap_n2 && nnodes <= h->cap_nodes && h->arena) return BDC_OK;
  tn = std::max<int64_t>(tn, h->cap_n);
  tn2 = std::max<int64_t>(tn2, h->cap_n2);
  nnodes = std::max(nnodes, h->cap_nodes);
  const size_t bytes = work_layout(nullptr, nullptr, tn, tn2, nnodes);
  if (h->opt.workspace_cap_bytes && bytes > h->opt.workspace_cap_bytes) return BDC_ERR_NOMEM;
  if (h->arena) {
    if (h->have_call) (void)hipStreamSynchronize(h->last_stream);
    drop_graph(h);
    (void)hipFree(h->arena);
    h->arena = nullptr;
    h->arena_bytes = 0;
  }
  if (hipMalloc(&h->arena, bytes) != hipSuccess) {
    h->arena = nullptr;
    h->cap_n = h->cap_n2 = -1;
    h->cap_nodes = -1;
    return BDC_ERR_NOMEM;
  }
  h->arena_bytes = bytes;
  work_layout(&h->w, (char*)h->arena, tn, tn2, nnodes);
  h->cap_n = tn;
  h->cap_n2 = tn2;
  h->cap_nodes = nnodes;
  return BDC_OK;
}

// Slice planes of the split-precision products for one problem of size n:
// per side (U, V) the row-split left operands and the column-split right
// operands of the top and bottom halves, each `slices` bfloat16 planes of
// n rows x P (P >= n + 32, a multiple of 8), and an exponent per plane row.
int64_t ozaki_stride(int64_t n) { return ((n + 32 + 7) / 8) * 8; }

int ensure_ozaki(bdc_handle_t h, int64_t n) {
  const int S = h->opt.ozaki_slices;
  const int64_t P = ozaki_stride(n);
  const size_t plane = (size_t)n * P;
  const size_t bytes = 6 * align_up((size_t)S * plane * 2) + 6 * align_up((size_t)n * 4);
  if (h->oz_arena && h->oz_bytes >= bytes && h->w.oz.P == P && h->w.oz.S == S) return BDC_OK;
  if (h->have_call) (void)hipStreamSynchronize(h->last_stream);
  drop_graph(h);
  if (h->oz_arena) (void)hipFree(h->oz_arena);
  h->oz_arena = nullptr;
  h->oz_bytes = 0;
  if (h->opt.workspace_cap_bytes && h->arena_bytes + bytes > h->opt.workspace_cap_bytes) return BDC_ERR_NOMEM;
  if (hipMalloc(&h->oz_arena, bytes) != hipSuccess) {
    h->oz_arena = nullptr;
    return BDC_ERR_NOMEM;
  }
  h->oz_bytes = bytes;
  char* b = (char*)h->oz_arena;
  auto take = [&](size_t nbytes) {
    char* r = b;
    b += align_up(nbytes);
    return (void*)r;
  };
  OzWork& oz = h->w.oz;
  for (int side = 0; side < 2; ++side) {
    oz.A[side] = (unsigned short*)take((size_t)S * plane * 2);
    oz.Bt[side] = (unsigned short*)take((size_t)S * plane * 2);
    oz.Bb[side] = (unsigned short*)take((size_t)S * plane * 2);
  }
  for (int side = 0; side < 2; ++side) {
    oz.Ea[side] = (int*)take((size_t)n * 4);
    oz.Ebt[side] = (int*)take((size_t)n * 4);
    oz.Ebb[side] = (int*)take((size_t)n * 4);
  }
  oz.plane = (int64_t)plane;
  oz.P = P;
  oz.S = S;
  return BDC_OK;
}

// Residue planes of the int8 split products for one problem of size n: per
// side (U, V) L planes each of the left operands ((n + 257) rows), of the
// right operands of the top and bottom halves ((n + 256) rows), all with row
// stride P = n rounded up to 64 bytes (the extra rows absorb the over-read of
// the last 256-row tile), of the products ((n + 1) x (n + 1), column-major,
// column stride n + 1 rounded up to 16 bytes), and the per-row maxima and
// exponents.
int ensure_crt(bdc_handle_t h, int64_t n) {
  const int L = h->opt.crt_moduli;
  const int64_t P = crt_kpad((int)n);
  const int64_t planeA = (n + 257) * P, planeB = (n + 256) * P, ldr = (n + 1 + 15) / 16 * 16,
                planeC = ldr * (n + 1);
  const size_t bytes = 2 * (align_up((size_t)L * planeA) + 2 * align_up((size_t)L * planeB) +
                            align_up((size_t)L * planeC) + 3 * align_up((size_t)(n + 1) * 8) +
                            3 * align_up((size_t)(n + 1) * 4));
  if (h->crt_arena && h->crt_n == n && h->crt_bytes == bytes && h->w.crt.L == L) return BDC_OK;
  if (h->have_call) (void)hipStreamSynchronize(h->last_stream);
  drop_graph(h);
  if (h->crt_arena) (void)hipFree(h->crt_arena);
  h->crt_arena = nullptr;
  h->crt_bytes = 0;
  h->crt_n = -1;
  if (h->opt.workspace_cap_bytes && h->arena_bytes + bytes > h->opt.workspace_cap_bytes) return BDC_ERR_NOMEM;
  if (hipMalloc(&h->crt_arena, bytes) != hipSuccess) {
    h->crt_arena = nullptr;
    return BDC_ERR_NOMEM;
  }
  h->crt_bytes = bytes;
  h->crt_n = n;
  char* b = (char*)h->crt_arena;
  auto take = [&](size_t nbytes) {
    char* r = b;
    b += align_up(nbytes);
    return (void*)r;
  };
  CrtWork& c = h->w.crt;
  for (int side = 0; side < 2; ++side) {
    c.A[side] = (int8_t*)take((size_t)L * planeA);
    c.Bt[side] = (int8_t*)take((size_t)L * planeB);
    c.Bb[side] = (int8_t*)take((size_t)L * planeB);
    c.C[side] = (int8_t*)take((size_t)L * planeC);
    c.amax[side] = (unsigned long long*)take((size_t)(n + 1) * 8);
    c.btmax[side] = (unsigned long long*)take((size_t)(n + 1) * 8);
    c.bbmax[side] = (unsigned long long*)take((size_t)(n + 1) * 8);
    c.Ea[side] = (int*)take((size_t)(n + 1) * 4);
    c.Ebt[side] = (int*)take((size_t)(n + 1) * 4);
    c.Ebb[side] = (int*)take((size_t)(n + 1) * 4);
  }
  c.planeA = planeA;
  c.planeB = planeB;
  c.planeC = planeC;
  c.P = (int)P;
  c.ldr = (int)ldr;
  c.L = L;
  return BDC_OK;
}

hipEvent_t next_event(bdc_handle_t h) {
  if (h->pool_used == h->pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->pool.push_back(e);
  }
  return h->pool[h->pool_used++];
}

struct Timer {
  bdc_handle_t h;
  hipStream_t st;
  int kind;
  hipEvent_t a = nullptr;
  Timer(bdc_handle_t h_, hipStream_t st_, int kind_) : h(h_), st(st_), kind(kind_) {
    if (h->opt.timing) {
      a = next_event(h);
      if (a) (void)hipEventRecord(a, st);
    }
  }
  ~Timer() {
    if (h->opt.timing && a) {
      hipEvent_t b = next_event(h);
      if (b) {
        (void)hipEventRecord(b, st);
        h->recs.push_back({kind, a, b});
      }
    }
  }
};

// side: a second stream for each level's rotations and gather, or null to
// run every launch on st
int run_plan(bdc_handle_t h, const double* d, const double* e, double* sigma, double* U, double* VT,
             hipStream_t st, hipStream_t side = nullptr) {
  const Plan& p = h->plan;
  Work w = h->w;
  w.d = d;
  w.e = e;
  w.GU = U;
  w.GV = VT;
  w.max_secular_iters = h->opt.max_secular_iters;
  w.max_leaf_sweeps = h->opt.max_leaf_sweeps;
  w.learned_min_n = h->opt.learned_min_n;
  const bool learned = h->opt.start == BDC_START_LEARNED;
  w.xs = nullptr;
  w.mlp_pk = learned ? h->mlp_pk : nullptr;
  // split products only with slice planes laid out for this problem's size
  // (a buffer left by an earlier, larger solve has another row stride)
  const bool ozaki = h->opt.gemm == BDC_GEMM_OZAKI && p.nprob == 1 && h->oz_arena &&
                     h->w.oz.P == ozaki_stride(p.sizes[0]);
  const bool crt = h->opt.gemm == BDC_GEMM_CRT && p.nprob == 1 && h->crt_arena && h->crt_n == p.sizes[0];
  w.oz.min_n = (ozaki || crt) ? h->opt.ozaki_min_n : INT32_MAX;
  h->last_split_min_n = w.oz.min_n;
  w.small_n = h->tune.small_n;
  w.sec_small_n = h->tune.sec_small_n;
  {
    Timer t(h, st, kReset);
    launch_reset(w.ctl, w.st, w.sec, p.nnodes, st);
  }
  if (learned) {
    Timer t(h, st, kStart);
    launch_mlp_pack(h->mlp, h->mlp_pk, st);
  }
  {
    Timer t(h, st, kLeaf);
    launch_leaf(p.dev_leaves, p.nleaves, p.leaf, w, st);
  }
  for (const Level& L : p.levels) {
    { Timer t(h, st, kPrep); launch_prep(L.dev, L.nnodes, L.max_m, w, st); }
    // The rotations of the deflated pairs and the gather of the kept columns
    // (the U and V data) need only the deflation's lists; the secular solve,
    // the Löwner z and the vectors of M~ (the small matrices) need only the
    // deflated values and z.  Neither chain reads what the other writes, so
    // with a second stream they run side by side, joined before the update
    // products, which need both.
    hipStream_t sr = side ? side : st;
    if (side && (hipEventRecord(h->ev_fork, st) != hipSuccess || hipStreamWaitEvent(side, h->ev_fork, 0) != hipSuccess))
      return BDC_ERR_HIP;
    { Timer t(h, sr, kRotate); launch_rotate(L.dev, L.nnodes, L.max_m, w, sr); }
    { Timer t(h, sr, kGather); launch_gather(L.dev, L.nnodes, L.max_m, w, sr); }
    if (side && hipEventRecord(h->ev_join, side) != hipSuccess) return BDC_ERR_HIP;
    { Timer t(h, st, kSecular); launch_secular(L.dev, L.nnodes, L.max_m, w, st); }
    if (h->harvest) launch_harvest(L.dev, L.nnodes, L.max_m, w, h->hv, st);
    { Timer t(h, st, kLowner); launch_lowner(L.dev, L.nnodes, L.max_m, w, st); }
    { Timer t(h, st, kVectors); launch_vectors(L.dev, L.nnodes, L.max_m, w, st); }
    if (side && hipStreamWaitEvent(st, h->ev_join, 0) != hipSuccess) return BDC_ERR_HIP;
    // the update launches carry the merge of roots and deflated values
    // (k_order) as well
    { Timer t(h, st, kUpdate); launch_update(L.dev, L.nnodes, L.max_m, w, h->tune, st); }
    if (ozaki && L.max_m >= w.oz.min_n) {
      Timer t(h, st, kUpdateOz);
      launch_update_ozaki(L.dev, L.nnodes, L.max_m, w, st);
    }
    if (crt && L.max_m >= w.oz.min_n) {
      Timer t(h, st, kUpdateCrt);
      launch_update_crt(L.dev, L.nnodes, L.max_m, w, st);
    }
  }
  {
    Timer t(h, st, kFinal);
    const int64_t np = p.nprob;
    // a single problem whose size is a multiple of 8 chunks (4096) takes the
    // XCD-aligned 4 KB-chunk form
    if (np == 1 && p.sizes[0] % (8 * kFinalChunk) == 0)
      launch_final_single(p.sizes[0], w, sigma, U, VT, st);
    else
      launch_final(p.dev_prob, p.dev_prob + np, p.dev_prob + 2 * np, p.dev_prob + 3 * np, p.dev_prob + 4 * np,
                   p.dev_uprob, p.dev_vprob, p.total_cols, p.total_tiles, w, sigma, U, VT, st);
  }
  if (hipGetLastError() != hipSuccess) return BDC_ERR_HIP;
  h->last_stream = st;
  h->have_call = true;
  return BDC_OK;
}

int solve(bdc_handle_t h, int64_t batch, const int64_t* sizes, const double* d, const double* e,
          double* sigma, double* U, double* VT, hipStream_t st) {
  DeviceGuard g(h->device);
  if (!g.ok) return BDC_ERR_HIP;
  if (h->opt.start == BDC_START_LEARNED && (!h->mlp || !h->mlp_pk)) return BDC_ERR_NO_MODEL;
  int rc = make_plan(h, sizes, batch);
  if (rc != BDC_OK) return rc;
  rc = ensure_workspace(h, h->plan.total_n, h->plan.total_n2, h->plan.nnodes);
  if (rc != BDC_OK) return rc;
  if (h->opt.gemm == BDC_GEMM_OZAKI && batch == 1 && sizes[0] >= h->opt.ozaki_min_n) {
    rc = ensure_ozaki(h, sizes[0]);
    if (rc != BDC_OK) return rc;
  }
  if (h->opt.gemm == BDC_GEMM_CRT && batch == 1 && sizes[0] >= h->opt.ozaki_min_n) {
    rc = ensure_crt(h, sizes[0]);
    if (rc != BDC_OK) return rc;
  }
  if (h->plan.total_n == 0) {
    h->last_stream = st;
    h->have_call = true;
    launch_reset(h->w.ctl, h->w.st, h->w.sec, 0, st);
    return hipGetLastError() == hipSuccess ? BDC_OK : BDC_ERR_HIP;
  }
  if (h->opt.timing || !h->opt.use_graph || h->harvest) return run_plan(h, d, e, sigma, U, VT, st);
  // replay the captured sequence when the plan and the buffers are the same
  const void* key[5] = {d, e, sigma, U, VT};
  bool same = h->gexec != nullptr;
  for (int i = 0; i < 5 && same; ++i) same = key[i] == h->gkey[i];
  if (!same) {
    if (h->have_call) (void)hipStreamSynchronize(h->last_stream);
    drop_graph(h);
    if (!h->cap_stream && hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess)
      return BDC_ERR_HIP;
    if (!h->side_stream && hipStreamCreateWithFlags(&h->side_stream, hipStreamNonBlocking) != hipSuccess)
      return BDC_ERR_HIP;
    if (!h->ev_fork && hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) != hipSuccess) return BDC_ERR_HIP;
    if (!h->ev_join && hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming) != hipSuccess) return BDC_ERR_HIP;
    if (hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return BDC_ERR_HIP;
    const int rc = run_plan(h, d, e, sigma, U, VT, h->cap_stream, h->tune.streams == 2 ? h->side_stream : nullptr);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(h->cap_stream, &g);
    if (rc != BDC_OK || ec != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return rc != BDC_OK ? rc : BDC_ERR_HIP;
    }
    const hipError_t ei = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      h->gexec = nullptr;
      return BDC_ERR_HIP;
    }
    for (int i = 0; i < 5; ++i) h->gkey[i] = key[i];
  }
  if (hipGraphLaunch(h->gexec, st) != hipSuccess) return BDC_ERR_HIP;
  h->last_stream = st;
  h->have_call = true;
  return BDC_OK;
}

}  // namespace

int bdc::handle_sec_small(bdc_handle_t h) { return valid(h) ? h->tune.sec_small_n : 0; }
int bdc::handle_tile128(bdc_handle_t h) { return valid(h) ? h->tune.tile128 : 0; }

int bdc::handle_info(bdc_handle_t h, int* device, int* max_secular_iters, int* max_leaf_sweeps) {
  if (!valid(h)) return BDC_ERR_INVALID_HANDLE;
  *device = h->device;
  *max_secular_iters = h->opt.max_secular_iters;
  *max_leaf_sweeps = h->opt.max_leaf_sweeps;
  return BDC_OK;
}

extern "C" {

void bdc_default_options(bdc_options_t* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->leaf_size = 32;
  opt->max_secular_iters = 64;
  opt->max_leaf_sweeps = 40;
  opt->workspace_cap_bytes = 0;
  opt->timing = 0;
  opt->use_graph = 1;
  opt->start = BDC_START_PLAIN;
  opt->gemm = BDC_GEMM_FP64;
  opt->ozaki_slices = 7;
  opt->ozaki_min_n = 256;
  opt->crt_moduli = 16;
  opt->learned_min_n = BDC_LEARNED_MIN_N;
}

int bdc_create(bdc_handle_t* handle, int device, const bdc_options_t* opt) {
  if (!handle) return -1;
  *handle = nullptr;
  bdc_options_t o;
  bdc_default_options(&o);
  if (opt) o = *opt;
  if (o.leaf_size < 4 || o.leaf_size > kMaxLeaf) return -3;
  if (o.max_secular_iters < 2 || o.max_secular_iters > 64) return -3;
  if (o.max_leaf_sweeps < 1 || o.max_leaf_sweeps > 1000) return -3;
  if (o.start != BDC_START_PLAIN && o.start != BDC_START_LEARNED) return -3;
  if (o.gemm != BDC_GEMM_FP64 && o.gemm != BDC_GEMM_OZAKI && o.gemm != BDC_GEMM_CRT) return -3;
  if (!oz_supported(o.ozaki_slices) || o.ozaki_min_n < 128) return -3;
  if (!crt_supported(o.crt_moduli)) return -3;
  if (o.learned_min_n < 0) return -3;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return BDC_ERR_NO_DEVICE;
  if (device < 0 || device >= count) return BDC_ERR_NO_DEVICE;
  bdc_handle_s* h = new (std::nothrow) bdc_handle_s();
  if (!h) return BDC_ERR_NOMEM;
  h->device = device;
  h->opt = o;
  {
    // the fixed scratch's address on this device, looked up once per device
    DeviceGuard g(device);
    if (g.ok) h->bt_fixed = backtr_fixed_scratch(device);
  }
  *handle = h;
  return BDC_OK;
}

int bdc_destroy(bdc_handle_t h) {
  if (!valid(h)) return BDC_ERR_INVALID_HANDLE;
  {
    DeviceGuard g(h->device);
    if (h->have_call) (void)hipStreamSynchronize(h->last_stream);
    drop_graph(h);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->side_stream) (void)hipStreamDestroy(h->side_stream);
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    free_plan(h->plan);
    if (h->arena) (void)hipFree(h->arena);
    if (h->oz_arena) (void)hipFree(h->oz_arena);
    if (h->crt_arena) (void)hipFree(h->crt_arena);
    if (h->bt_arena) (void)hipFree(h->bt_arena);
    if (h->qr_sync) (void)hipFree(h->qr_sync);
    if (h->brd_work) (void)hipFree(h->brd_work);
    if (h->mlp) (void)hipFree(h->mlp);
    if (h->mlp_pk) (void)hipFree(h->mlp_pk);
    if (h->part) (void)hipFree(h->part);
    for (hipEvent_t e : h->pool) (void)hipEventDestroy(e);
  }
  h->magic = 0;
  delete h;
  return BDC_OK;
}

int bdc_svd(bdc_handle_t h, int64_t n, const double* d, const double* e, double* sigma, double* U,
            double* VT, bdc_stream_t stream) {
  if (!valid(h)) return BDC_ERR_INVALID_HANDLE;
  if (n < 0 || n > (int64_t)INT32_MAX / 2) return -2;
  if (n > 0 && !d) return -3;
  if (n > 1 && !e) return -4;
  if (n > 0 && !sigma) return -5;
  if (n > 0 && !U) return -6;
  if (n > 0 && !VT) return -7;
  if (n > 0 && U == VT) return -7;
  return solve(h, 1, &n, d, e, sigma, U, VT, (hipStream_t)stream);
}

int bdc_svd_batched(bdc_handle_t h, int64_t batch, const int64_t* sizes, const double* d,
                    const double* e, double* sigma, double* U, double* VT, bdc_stream_t stream) {
  if (!valid(h)) return BDC_ERR_INVALID_HANDLE;
  if (batch < 0 || batch > (int64_t)INT32_MAX) return -2;
  if (batch > 0 && !sizes) return -3;
  int64_t total = 0, maxn = 0;
  for (int64_t i = 0; i < batch; ++i) {
    if (sizes[i] < 0 || sizes[i] > (int64_t)INT32_MAX / 2) return -3;
    total += sizes[i];
    maxn = std::max(maxn, sizes[i]);
  }
  if (total > (int64_t)INT32_MAX) return -3;
  if (total > 0 && !d) return -4;
  if (maxn > 1 && !e) return -5;
  if (total > 0 && !sigma) return -6;
  if (total > 0 && !U) return -7;
  if (total > 0 && (!VT || VT == U)) return -8;
  return solve(h, batch, sizes, d, e, sigma, U, VT, (hipStream_t)stream);
}

int bdc_get_info(bdc_handle_t h, int64_t* info, bdc_stats_t* stats) {
  if (!valid(h)) return BDC_ERR_INVALID_HANDLE;
  if (info) *info = 0;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (!h->have_call || !h->arena) return BDC_OK;
  DeviceGuard g(h->device);
  if (hipStreamSynchronize(h->last_stream) != hipSuccess) return BDC_ERR_HIP;
  Ctl ctl;
  if (hipMemcpy(&ctl, h->w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost) != hipSuccess) return BDC_ERR_HIP;
  std::vector<NodeState> sts;
  int64_t sec_capped = 0;
  unsigned long long sec_evals = 0, sec_terms = 0;
  if (h->plan_valid && h->plan.nnodes > 0) {
    sts.resize(h->plan.nnodes);
    std::vector<SecCount> sc(h->plan.nnodes);
    if (hipMemcpy(sts.data(), h->w.st, sizeof(NodeState) * h->plan.nnodes, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(sc.data(), h->w.sec, sizeof(SecCount) * h->plan.nnodes, hipMemcpyDeviceToHost) != hipSuccess)
      return BDC_ERR_HIP;
    for (const SecCount& c : sc) {
      sec_capped += (int64_t)c.capped;
      sec_evals += c.evals;
      sec_terms += c.terms;
    }
  }
  if (info) *info = ctl.nonfinite ? (int64_t)BDC_ERR_NONFINITE : (int64_t)ctl.leaf_capped + sec_capped;
  if (stats && h->plan_valid) {
    const Plan& p = h->plan;
    stats->merges = p.nnodes;
    stats->levels = (int64_t)p.levels.size();
    stats->secular_evals = (int64_t)sec_evals;
    double fl = 0.0;
    for (int i = 0; i < p.nnodes; ++i) {
      const NodeState& s = sts[i];
      const NodeDesc& nd = p.host_nodes[i];
      stats->roots += s.N;
      stats->deflated_small_z += s.nsmall_z;
      stats->deflated_zero_d += s.nzero_d;
      stats->deflated_close += s.nclose;
      stats->rotations += s.nrot;
      const double N = s.N, top = s.n1 + 1 + s.n2, bot = 1 + s.n2 + s.n3;
      const double f = 2.0 * N * (nd.k * top + (nd.m - nd.k) * bot) +     // left vectors
                       2.0 * N * (nd.k * top + (nd.m + nd.s - nd.k) * bot);  // right vectors
      fl += f;
      if (s.N >= h->last_split_min_n) {
        stats->split_merges += 1;
        stats->split_flops += f;
      }
    }
    stats->update_flops = fl;
    if (p.root_id0 >= 0) stats->root_N = sts[p.root_id0].N;
    stats->secular_terms = (int64_t)sec_terms;
    {
      std::vector<unsigned long long> lf(std::max(p.nleaves, 1));
      if (p.nleaves > 0 &&
          hipMemcpy(lf.data(), h->w.leaf_fl, sizeof(unsigned long long) * p.nleaves, hipMemcpyDeviceToHost) !=
              hipSuccess)
        return BDC_ERR_HIP;
      double lfl = 0.0;
      for (int i = 0; i < p.nleaves; ++i) lfl += (double)lf[i];
      stats->leaf_flops = lfl;
    }
    double gb = 0.0;
    for (int i = 0; i < p.nnodes; ++i) {
      const NodeDesc& nd = p.host_nodes[i];
      gb += 16.0 * sts[i].N * (2.0 * nd.m + nd.s);  // read + write, U and V columns
    }
    stats->gather_bytes = gb;
    // supports read by the final pass
    const size_t tn = (size_t)p.total_n;
    std::vector<int32_t> lo(tn), hi(tn), vl(tn), vh(tn), col(tn);
    if (tn > 0 &&
        (hipMemcpy(lo.data(), h->w.ulo, 4 * tn, hipMemcpyDeviceToHost) != hipSuccess ||
         hipMemcpy(hi.data(), h->w.uhi, 4 * tn, hipMemcpyDeviceToHost) != hipSuccess ||
         hipMemcpy(vl.data(), h->w.vlo, 4 * tn, hipMemcpyDeviceToHost) != hipSuccess ||
         hipMemcpy(vh.data(), h->w.vhi, 4 * tn, hipMemcpyDeviceToHost) != hipSuccess))
      return BDC_ERR_HIP;
    int64_t fr = 0;
    for (size_t c = 0; c < tn; ++c) fr += (int64_t)(hi[c] - lo[c]) + (int64_t)(vh[c] - vl[c]);
    stats->final_read_elems = fr;
  }
  return BDC_OK;
}

int bdc_get_timing(bdc_handle_t h, int cap, const char** names, double* ms, int64_t* launches) {
  if (!valid(h)) return BDC_ERR_INVALID_HANDLE;
  double tot[kKinds] = {0};
  int64_t cnt[kKinds] = {0};
  if (h->have_call) {
    DeviceGuard g(h->device);
    if (hipStreamSynchronize(h->last_stream) != hipSuccess) return BDC_ERR_HIP;
    for (auto& r : h->recs) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) tot[r.kind] += t;
      cnt[r.kind] += 1;
    }
  }
  for (int i = 0; i < kKinds && i < cap; ++i) {
    if (names) names[i] = kKindNames[i];
    if (ms) ms[i] = tot[i];
    if (launches) launches[i] = cnt[i];
  }
  return kKinds;
}

int bdc_clear_timing(bdc_handle_t h) {
  if (!valid(h)) return BDC_ERR_INVALID_HANDLE;
  h->recs.clear();
  h->pool_used = 0;
  return BDC_OK;
}

// ---- back-transformation -----------------------------------------------------

namespace {
// argument checks shared by both back-transformation entry points: BDC_OK to
// proceed, 1 for an empty call (nothing to do), or the error status
int reflector_args(bdc_handle_t h, int trans, int m, int p, int k, int offset, const double* Y, int64_t y_rs,
                   int64_t y_cs, const double* tau, double* C, int ldc, int* block) {
  if (!valid(h)) return BDC_ERR_INVALID_HANDLE;
  if (trans != 0 && trans != 1) return -2;
  if (m < 0) return -3;
  if (p < 0) return -4;
  if (k < 0) return -5;
  if (offset < 0) return -6;
  if (m == 0 || p == 0 || k == 0) return 1;
  if (!Y) return -7;
  if (y_rs < 1 && y_cs < 1) return -8;
  if (!tau) return -10;
  if (!C) return -11;
  if (ldc < m) return -12;
  if (*block == 0) *block = kBtMaxBlock;
  if (*block < 1 || *block > kBtMaxBlock) return -13;
  return BDC_OK;
}
}  // namespace

namespace {
// the handle's back-transformation scratch, grown to at least `bytes`
int ensure_bt(bdc_handle_t h, size_t bytes) {
  if (h->bt_bytes >= bytes) return BDC_OK;
  if (h->have_call) (void)hipStreamSynchronize(h->last_stream);
  if (h->bt_arena) (void)hipFree(h->bt_arena);
  h->bt_arena = nullptr;
  h->bt_bytes = 0;
  if (h->opt.workspace_cap_bytes && h->arena_bytes + bytes > h->opt.workspace_cap_bytes) return BDC_ERR_NOMEM;
  if (hipMalloc(&h->bt_arena, bytes) != hipSuccess) {
    h->bt_arena = nullptr;
    return BDC_ERR_NOMEM;
  }
  h->bt_bytes = bytes;
  return BDC_OK;
}
}  // namespace

int bdc_apply_reflectors(bdc_handle_t h, int trans, int m, int p, int k, int offset, const double* Y, int64_t y_rs,
                         int64_t y_cs, const double* tau, double* C, int ldc, int block, bdc_stream_t stream) {
  const int a = reflector_args(h, trans, m, p, k, offset, Y, y_rs, y_cs, tau, C, ldc, &block);
  if (a != BDC_OK) return a == 1 ? BDC_OK : a;
  DeviceGuard g(h->device);
  if (!g.ok) return BDC_ERR_HIP;
  const int rc = ensure_bt(h, backtr_bytes(m, p, block));
  if (rc != BDC_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  launch_backtr(trans, m, p, k, offset, Y, y_rs, y_cs, tau, C, ldc, block, h->bt_arena, p, st);
  if (hipGetLastError() != hipSuccess) return BDC_ERR_HIP;
  h->last_stream = st;
  h->have_call = true;
  return BDC_OK;
}

int bdc_apply_reflectors_noalloc(bdc_handle_t h, int trans, int m, int p, int k, int offset, const double* Y,
                                 int64_t y_rs, int64_t y_cs, const double* tau, double* C, int ldc, int block,
                                 bdc_stream_t stream) {
  const int a = reflector_args(h, trans, m, p, k, offset, Y, y_rs, y_cs, tau, C, ldc, &block);
  if (a != BDC_OK) return a == 1 ? BDC_OK : a;
  const int panel = std::min(p, kBtFixedPanel);
  if (backtr_bytes(m, panel, block) > kBtFixedScratchBytes) return BDC_ERR_TOO_LARGE;
  if (!h->bt_fixed) return BDC_ERR_HIP;  // the scratch address was not found at bdc_create
  DeviceGuard g(h->device);
  if (!g.ok) return BDC_ERR_HIP;
  hipStream_t st = (hipStream_t)stream;
  launch_backtr(trans, m, p, k, offset, Y, y_rs, y_cs, tau, C, ldc, block, h->bt_fixed, panel, st);
  if (hipGetLastError() != hipSuccess) return BDC_ERR_HIP;
  h->last_stream = st;
  h->have_call = true;
  return BDC_OK;
}

// ---- tall-and-skinny QR ---------------------------------------------------------

int bdc_geqrf(bdc_handle_t h, int m, int n, double* A, int lda, double* tau, int block, bdc_stream_t stream) {
  if (!valid(h)) return BDC_ERR_INVALID_HANDLE;
  if (m < 0) return -2;
  if (n < 0 || n > m) return -3;
  if (m == 0 || n == 0) return BDC_OK;
  if (!A) return -4;
  if (lda < m) return -5;
  if (!tau) return -6;
  if (block == 0) block = kQrDefaultBlock;
  if (block < 1 || block > qr_max_block()) return -7;
  DeviceGuard g(h->device);
  if (!g.ok) return BDC_ERR_HIP;
  int rc = ensure_bt(h, backtr_bytes(m, n, block));
  if (rc != BDC_OK) return rc;
  const size_t sb = qr_sync_bytes(kQrMaxGrid);
  if (h->qr_sync_size < sb) {
    if (h->have_call) (void)hipStreamSynchronize(h->last_stream);
    if (h->qr_sync) (void)hipFree(h->qr_sync);
    h->qr_sync = nullptr;
    h->qr_sync_size = 0;
    if (hipMalloc(&h->qr_sync, sb) != hipSuccess) {
      h->qr_sync = nullptr;
      return BDC_ERR_NOMEM;
    }
    h->qr_sync_size = sb;
  }
  hipStream_t st = (hipStream_t)stream;
  rc = launch_geqrf(h->device, m, n, A, lda, tau, block, h->qr_sync, h->qr_sync_size, h->bt_arena, st);
  if (rc != BDC_OK) return rc;
  if (hipGetLastError() != hipSuccess) return BDC_ERR_HIP;
  h->last_stream = st;
  h->have_call = true;
  return BDC_OK;
}

int bdc_orgqr(bdc_handle_t h, int m, int ncols, int k, const double* A, int lda, const double* tau, double* Q, int ldq,
              int block, bdc_stream_t stream) {
  if (!valid(h)) return BDC_ERR_INVALID_HANDLE;
  if (m < 0) return -2;
  if (ncols < 0 || ncols > m) return -3;
  if (k < 0 || k > ncols) return -4;
  if (m == 0 || ncols == 0) return BDC_OK;
  if (k > 0 && !A) return -5;
  if (lda < m) return -6;
  if (k > 0 && !tau) return -7;
  if (!Q) return -8;
  if (ldq < m) return -9;
  if (block == 0) block = kBtMaxBlock;
  if (block < 1 || block > kBtMaxBlock) return -10;
  DeviceGuard g(h->device);
  if (!g.ok) return BDC_ERR_HIP;
  const int rc = ensure_bt(h, backtr_bytes(m, ncols, block));
  if (rc != BDC_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  launch_orgqr(m, ncols, k, A, lda, tau, Q, ldq, block, h->bt_arena, st);
  if (hipGetLastError() != hipSuccess) return BDC_ERR_HIP;
  h->last_stream = st;
  h->have_call = true;
  return BDC_OK;
}

// ---- bidiagonal reduction -------------------------------------------------------

int bdc_gebrd(bdc_handle_t h, int m, int n, double* A, int lda, double* d, double* e, double* tauq, double* taup,
              int block, bdc_stream_t stream) {
  if (!valid(h)) return BDC_ERR_INVALID_HANDLE;
  if (m < 0) return -2;
  if (n < 0 || n > m) return -3;
  if (m == 0 || n == 0) return BDC_OK;
  if (!A) return -4;
  if (lda < m) return -5;
  if (!d) return -6;
  if (!e && n > 1) return -7;
  if (!tauq) return -8;
  if (!taup) return -9;
  if (block == 0) block = gebrd_max_block();
  if (block < 1 || block > gebrd_max_block()) return -10;
  DeviceGuard g(h->device);
  if (!g.ok) return BDC_ERR_HIP;
  const size_t bytes = gebrd_work_bytes(m, n, block, kQrMaxGrid);
  if (h->brd_bytes < bytes) {
    if (h->have_call) (void)hipStreamSynchronize(h->last_stream);
    if (h->brd_work) (void)hipFree(h->brd_work);
    h->brd_work = nullptr;
    h->brd_bytes = 0;
    if (h->opt.workspace_cap_bytes && h->arena_bytes + bytes > h->opt.workspace_cap_bytes) return BDC_ERR_NOMEM;
    if (hipMalloc(&h->brd_work, bytes) != hipSuccess) {
      h->brd_work = nullptr;
      return BDC_ERR_NOMEM;
    }
    h->brd_bytes = bytes;
  }
  hipStream_t st = (hipStream_t)stream;
  const int rc = launch_gebrd(h->device, m, n, A, lda, tauq, taup, d, e, block, h->brd_work, h->brd_bytes,
                              kQrMaxGrid, st);
  if (rc != BDC_OK) return rc;
  if (hipGetLastError() != hipSuccess) return BDC_ERR_HIP;
  h->last_stream = st;
  h->have_call = true;
  return BDC_OK;
}

// ---- launch tuning -----------------------------------------------------------

namespace {
// small_n at or above every merge size: all merges take the 64 x 64 tiles
// and the 128 x 128 launch is left out of every level
constexpr int kSmallNAll = 1 << 20;

bool tuning_valid(const bdc_tuning_t* t) {
  return t->small_n >= 32 && t->small_n <= kSmallNAll && (t->flat == 0 || t->flat == 1) && t->grid64 >= 1 &&
         t->grid64 <= 65535 && t->grid128 >= 1 && t->grid128 <= 65535 && t->sec_small_n >= 0 &&
         t->sec_small_n <= kSecLanesMaxN && (t->leaf_size == 0 || (t->leaf_size >= 4 && t->leaf_size <= kMaxLeaf)) &&
         (t->tile128 == 0 || t->tile128 == 1) && (t->streams == 1 || t->streams == 2);
}
}  // namespace

int bdc_get_tuning(bdc_handle_t h, bdc_tuning_t* t) {
  if (!valid(h)) return BDC_ERR_INVALID_HANDLE;
  if (!t) return -2;
  t->small_n = h->tune.small_n;
  t->flat = h->tune.flat;
  t->grid64 = h->tune.grid64;
  t->grid128 = h->tune.grid128;
  t->sec_small_n = h->tune.sec_small_n;
  t->leaf_size = h->opt.leaf_size;
  t->tile128 = h->tune.tile128;
  t->streams = h->tune.streams;
  return BDC_OK;
}

int bdc_set_tuning(bdc_handle_t h, const bdc_tuning_t* t) {
  if (!valid(h)) return BDC_ERR_INVALID_HANDLE;
  if (!t || !tuning_valid(t)) return -2;
  DeviceGuard g(h->device);
  if (h->have_call) (void)hipStreamSynchronize(h->last_stream);
  drop_graph(h);  // launch shapes are part of a captured sequence
  h->tune = Tuning{t->small_n, t->flat, t->grid64, t->grid128, t->sec_small_n, t->tile128, t->streams};
  if (t->leaf_size) h->opt.leaf_size = t->leaf_size;  // the plan is rebuilt on the next solve
  return BDC_OK;
}

int bdc_autotune(bdc_handle_t h, int64_t batch, const int64_t* sizes, const double* d, const double* e,
                 double* sigma, double* U, double* VT, bdc_stream_t stream, int repeats, bdc_tuning_t* best) {
  if (!valid(h)) return BDC_ERR_INVALID_HANDLE;
  if (repeats < 1 || repeats > 100) return -10;
  if (!best) return -11;
  DeviceGuard g(h->device);
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    return BDC_ERR_HIP;
  }
  const Tuning keep = h->tune;
  const int keep_leaf = h->opt.leaf_size;
  int rc = BDC_OK;
  // time of one candidate (leaf size, launch shapes): a warm-up solve (plan,
  // workspace, graph capture), then `repeats` timed ones
  auto time_one = [&](int leaf, const Tuning& c, float& ms) {
    if (h->have_call) (void)hipStreamSynchronize(h->last_stream);
    drop_graph(h);
    h->opt.leaf_size = leaf;
    h->tune = c;
    int r = bdc_svd_batched(h, batch, sizes, d, e, sigma, U, VT, stream);
    if (r != BDC_OK) return r;
    (void)hipEventRecord(a, st);
    for (int q = 0; q < repeats && r == BDC_OK; ++q) r = bdc_svd_batched(h, batch, sizes, d, e, sigma, U, VT, stream);
    (void)hipEventRecord(b, st);
    if (r != BDC_OK) return r;
    if (hipEventSynchronize(b) != hipSuccess) return (int)BDC_ERR_HIP;
    ms = 0.0f;
    (void)hipEventElapsedTime(&ms, a, b);
    ms /= repeats;
    return (int)BDC_OK;
  };
  // 1. the tree: leaf size, with the current launch shapes
  float best_ms = -1.0f;
  int best_leaf = keep_leaf;
  Tuning best_t = keep;
  for (int leaf : {8, 12, 16, 20, 24, 32}) {
    float ms = 0.0f;
    rc = time_one(leaf, keep, ms);
    if (rc != BDC_OK) break;
    if (best_ms < 0.0f || ms < best_ms) {
      best_ms = ms;
      best_leaf = leaf;
    }
  }
  // 2. launch shapes with that tree
  if (rc == BDC_OK) {
    std::vector<Tuning> cand;
    for (int ss : {0, 256})
      for (int sn : {64, 96, 192, kSmallNAll}) {
        cand.push_back(Tuning{sn, 0, 1024, 512, ss});
        for (int gm : {256, 512, 1024}) cand.push_back(Tuning{sn, 1, 2 * gm, gm, ss});
      }
    for (const Tuning& c : cand) {
      float ms = 0.0f;
      rc = time_one(best_leaf, c, ms);
      if (rc != BDC_OK) break;
      if (ms < best_ms) {
        best_ms = ms;
        best_t = c;
      }
    }
  }
  // 3. the other form of the 128 x 128 tile with those shapes
  if (rc == BDC_OK && !best_t.flat) {
    Tuning c = best_t;
    c.tile128 = 1 - c.tile128;
    float ms = 0.0f;
    rc = time_one(best_leaf, c, ms);
    if (rc == BDC_OK && ms < best_ms) {
      best_ms = ms;
      best_t = c;
    }
  }
  // 4. the rotations and gathers on a second stream (captured solves only)
  if (rc == BDC_OK && h->opt.use_graph) {
    Tuning c = best_t;
    c.streams = 3 - c.streams;
    float ms = 0.0f;
    rc = time_one(best_leaf, c, ms);
    if (rc == BDC_OK && ms < best_ms) {
      best_ms = ms;
      best_t = c;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (h->have_call) (void)hipStreamSynchronize(h->last_stream);
  drop_graph(h);
  h->tune = rc == BDC_OK ? best_t : keep;
  h->opt.leaf_size = rc == BDC_OK ? best_leaf : keep_leaf;
  best->small_n = h->tune.small_n;
  best->flat = h->tune.flat;
  best->grid64 = h->tune.grid64;
  best->grid128 = h->tune.grid128;
  best->sec_small_n = h->tune.sec_small_n;
  best->leaf_size = h->opt.leaf_size;
  best->tile128 = h->tune.tile128;
  best->streams = h->tune.streams;
  best->ms = rc == BDC_OK ? best_ms : 0.0f;
  return rc;
}

// ---- learned start ---------------------------------------------------------

int bdc_mlp_set(bdc_handle_t h, const float* params, int64_t count) {
  if (!valid(h)) return BDC_ERR_INVALID_HANDLE;
  if (!params) return -2;
  if (count != BDC_MLP_PARAMS) return -3;
  DeviceGuard g(h->device);
  if (h->have_call) (void)hipStreamSynchronize(h->last_stream);
  if (!h->mlp && hipMalloc(&h->mlp, sizeof(float) * 3 * BDC_MLP_PARAMS) != hipSuccess) {
    h->mlp = nullptr;
    return BDC_ERR_NOMEM;
  }
  if (!h->mlp_pk && hipMalloc(&h->mlp_pk, mlp_pack_bytes()) != hipSuccess) {
    h->mlp_pk = nullptr;
    return BDC_ERR_NOMEM;
  }
  if (hipMemcpy(h->mlp, params, sizeof(float) * BDC_MLP_PARAMS, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(h->mlp + BDC_MLP_PARAMS, 0, sizeof(float) * 2 * BDC_MLP_PARAMS) != hipSuccess)
    return BDC_ERR_HIP;
  h->adam_t = 0;
  return BDC_OK;
}

int bdc_mlp_get(bdc_handle_t h, float* params, int64_t count) {
  if (!valid(h)) return BDC_ERR_INVALID_HANDLE;
  if (!params) return -2;
  if (count != BDC_MLP_PARAMS) return -3;
  if (!h->mlp) return BDC_ERR_NO_MODEL;
  DeviceGuard g(h->device);
  if (h->have_call && hipStreamSynchronize(h->last_stream) != hipSuccess) return BDC_ERR_HIP;
  if (hipMemcpy(params, h->mlp, sizeof(float) * BDC_MLP_PARAMS, hipMemcpyDeviceToHost) != hipSuccess)
    return BDC_ERR_HIP;
  return BDC_OK;
}

int bdc_mlp_forward(bdc_handle_t h, const float* X, int64_t rows, float* xhat, bdc_stream_t stream) {
  if (!valid(h)) return BDC_ERR_INVALID_HANDLE;
  if (rows < 0 || rows > (int64_t)INT32_MAX - 64) return -3;
  if (rows > 0 && !X) return -2;
  if (rows > 0 && !xhat) return -4;
  if (!h->mlp) return BDC_ERR_NO_MODEL;
  DeviceGuard g(h->device);
  launch_mlp_forward(h->mlp, X, (int)rows, xhat, (hipStream_t)stream);
  if (hipGetLastError() != hipSuccess) return BDC_ERR_HIP;
  h->last_stream = (hipStream_t)stream;
  h->have_call = true;
  return BDC_OK;
}

namespace {
int ensure_parts(bdc_handle_t h, int rows) {
  const int parts = mlp_parts(rows);
  if (parts <= h->part_cap) return BDC_OK;
  if (h->have_call) (void)hipStreamSynchronize(h->last_stream);
  if (h->part) (void)hipFree(h->part);
  h->part = nullptr;
  h->part_cap = 0;
  if (hipMalloc(&h->part, sizeof(float) * (size_t)parts * (BDC_MLP_PARAMS + 1)) != hipSuccess) {
    h->part = nullptr;
    return BDC_ERR_NOMEM;
  }
  h->part_cap = parts;
  return BDC_OK;
}
}  // namespace

int bdc_mlp_grad(bdc_handle_t h, const float* X, const float* y, int64_t rows, float* grad, float* loss,
                 bdc_stream_t stream) {
  if (!valid(h)) return BDC_ERR_INVALID_HANDLE;
  if (!X) return -2;
  if (!y) return -3;
  if (rows < 1 || rows > (int64_t)1 << 24) return -4;
  if (!grad) return -5;
  if (!h->mlp) return BDC_ERR_NO_MODEL;
  DeviceGuard g(h->device);
  int rc = ensure_parts(h, (int)rows);
  if (rc != BDC_OK) return rc;
  const int parts = mlp_parts((int)rows);
  float* part_loss = h->part + (size_t)h->part_cap * BDC_MLP_PARAMS;
  hipStream_t st = (hipStream_t)stream;
  launch_mlp_grad(h->mlp, X, y, nullptr, (int)rows, h->part, part_loss, st);
  launch_adam(h->mlp, h->mlp + BDC_MLP_PARAMS, h->mlp + 2 * BDC_MLP_PARAMS, h->part, parts, part_loss, grad, loss,
              0, 0.0f, 1.0f / (float)rows, st);
  if (hipGetLastError() != hipSuccess) return BDC_ERR_HIP;
  h->last_stream = st;
  h->have_call = true;
  return BDC_OK;
}

int bdc_mlp_train(bdc_handle_t h, const float* X, const float* y, const int32_t* idx, int64_t batch,
                  int64_t steps, float lr, float* loss_hist, bdc_stream_t stream) {
  if (!valid(h)) return BDC_ERR_INVALID_HANDLE;
  if (!X) return -2;
  if (!y) return -3;
  if (!idx) return -4;
  if (batch < 1 || batch > (int64_t)1 << 24) return -5;
  if (steps < 0 || steps > (int64_t)1 << 30) return -6;
  if (!(lr > 0.0f) || !(lr < 1.0f)) return -7;
  if (!h->mlp) return BDC_ERR_NO_MODEL;
  DeviceGuard g(h->device);
  int rc = ensure_parts(h, (int)batch);
  if (rc != BDC_OK) return rc;
  const int parts = mlp_parts((int)batch);
  float* part_loss = h->part + (size_t)h->part_cap * BDC_MLP_PARAMS;
  hipStream_t st = (hipStream_t)stream;
  for (int64_t s = 0; s < steps; ++s) {
    launch_mlp_grad(h->mlp, X, y, idx + s * batch, (int)batch, h->part, part_loss, st);
    launch_adam(h->mlp, h->mlp + BDC_MLP_PARAMS, h->mlp + 2 * BDC_MLP_PARAMS, h->part, parts, part_loss, nullptr,
                loss_hist ? loss_hist + s : nullptr, ++h->adam_t, lr, 1.0f / (float)batch, st);
  }
  if (hipGetLastError() != hipSuccess) return BDC_ERR_HIP;
  h->last_stream = st;
  h->have_call = true;
  return BDC_OK;
}

int bdc_set_harvest(bdc_handle_t h, float* X, float* y, int32_t* tag, int64_t capacity,
                    unsigned long long* count) {
  if (!valid(h)) return BDC_ERR_INVALID_HANDLE;
  if (!X) {
    h->harvest = false;
    h->hv = Harvest{};
    return BDC_OK;
  }
  if (!y) return -3;
  if (!tag) return -4;
  if (capacity < 0) return -5;
  if (!count) return -6;
  h->hv = Harvest{X, y, tag, capacity, count};
  h->harvest = true;
  return BDC_OK;
}

const char* bdc_status_string(int status) {
  switch (status) {
    case BDC_OK: return "ok";
    case BDC_ERR_INVALID_HANDLE: return "invalid handle";
    case BDC_ERR_NO_DEVICE: return "no such HIP device";
    case BDC_ERR_NOMEM: return "out of device memory or over the workspace cap";
    case BDC_ERR_HIP: return "HIP runtime error";
    case BDC_ERR_NONFINITE: return "input holds Inf or NaN";
    case BDC_ERR_UNSUPPORTED: return "unsupported option";
    case BDC_ERR_NO_MODEL: return "learned start selected but no network parameters were set";
    case BDC_ERR_TOO_LARGE: return "problem larger than the fixed scratch of the allocation-free entry point";
    default: return status < 0 ? "invalid argument" : "iteration caps reached";
  }
}

}  // extern "C"
