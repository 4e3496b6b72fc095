// Internal structures of the bidiagonal divide-and-conquer solver (device
// descriptors, per-call workspace pointers, kernel launchers).
//
// Layout in HBM (per problem p of size n, offsets mat_off = sum n_j^2 and
// vec_off = sum n_j over the problems before it):
//   Uwork, Vwork   n x n column-major working left / right singular vectors.
//                  A node (r0, m, s) owns rows and columns [r0, r0+m) of Uwork
//                  and [r0, r0+m+s) of Vwork.  Columns are never moved when a
//                  merge deflates them: the node's sorted order is kept as an
//                  index (col[]), and each physical column records the row
//                  range outside which it is zero (ulo/uhi, vlo/vhi), so the
//                  rows outside are never read or written.
//   GU, GV         gathered non-deflated columns of a merge (m x N and
//                  (m+s) x N at the node's diagonal block).  These live in the
//                  caller's U and VT buffers, which are free until the end.
//   UM, VM         N x N singular vectors of the deflated M at the node's
//                  diagonal block of an n x n workspace matrix.
//   per-position   arrays of length n indexed vec_off + r0 + i for a node.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bdc.h"

namespace bdc {

constexpr int kMaxLeaf = 32;
// Batched final pass of V^T: bands of kVtBand output rows (singular
// vectors) by tiles of kVtTile output columns, kVtTilesPerGroup tiles per
// work item (one workgroup); work items of a problem of size n
// One tile per work item: short-lived workgroups stream the non-temporal
// stores best (the 2000-problem batch's final kernels 4.0-4.1 ms against
// 4.6-4.8 with 16 tiles per item and 4.4-4.5 with 4).
constexpr int kVtTilesPerGroup = 1;
constexpr int kVtBand = 256, kVtTile = 16;
__host__ __device__ inline int64_t vt_bands(int64_t n) { return (n + kVtBand - 1) / kVtBand; }
__host__ __device__ inline int64_t vt_groups(int64_t n) {
  return ((n + kVtTile - 1) / kVtTile + kVtTilesPerGroup - 1) / kVtTilesPerGroup;
}
// largest secular problem the lanes-per-root kernel takes
constexpr int kSecLanesMaxN = 256;
// doubles per 4 KB output chunk of the single-problem final pass
constexpr int kFinalChunk = 512;
// Columns of U written by one final-pass workgroup of a problem of size n
// (at least 16384 contiguous doubles per workgroup for small problems).
__host__ __device__ inline int final_u_cols(int64_t n) {
  // about 32 KB of output per work item (the 2000-problem batch's final
  // kernels 3.75 against 4.13 ms with 128 KB items)
  return n >= 4096 ? 1 : (int)(4096 / n < 64 ? 4096 / n : 64);
}
// flags of a column touched by a deflation rotation
constexpr int kRotV = 1;  // its right vector (both deflation rotations)
constexpr int kRotU = 2;  // its left vector (close-pair rotations only)

struct LeafDesc {
  int64_t mat_off;
  int64_t vec_off;
  int32_t ld;  // problem size n
  int32_t r0, m, s;
};

struct NodeDesc {
  int64_t mat_off;
  int64_t vec_off;
  int32_t ld;
  int32_t r0, m, s, k;
  int32_t id;  // index into the node-state array
};

// Written on the device by the deflation kernel of a merge.
struct NodeState {
  int32_t N;         // non-deflated size (secular roots)
  int32_t n1, n2, n3;  // kept columns supported on the left child, both, right child
  int32_t nrot;      // deflation rotations
  int32_t nsmall_z, nzero_d, nclose;
  double scale;      // power of two the merge was scaled by
  double tol;        // deflation tolerance (scaled units)
  double c0, s0;     // rotation combining the children's null vectors
  double rho;        // sum of the kept z_j^2
  unsigned long long zmax_bits;  // max(d, |z|) of the merge, as bits (atomic max)
};

// Secular statistics of one merge (atomics on the node's own counters, so the
// many merges of a level do not contend for one address).
struct SecCount {
  unsigned long long evals, terms;
  unsigned long long capped;
};

// Per-call device counters (rare events only; the statistics are per node
// and per leaf).
struct Ctl {
  int32_t nonfinite;
  int32_t leaf_capped;
};

// Split-precision update products: bfloat16 slice planes per side (0 U,
// 1 V) of the row-split left operands (A) and the column-split right operands
// of the top and bottom halves (Bt, Bb), with their power-of-two exponents.
struct OzWork {
  unsigned short* A[2];
  unsigned short* Bt[2];
  unsigned short* Bb[2];
  int* Ea[2];
  int* Ebt[2];
  int* Ebb[2];
  int64_t plane;  // elements per slice plane
  int64_t P;      // row stride of a plane
  int S;          // slices per operand
  int min_n;      // merges with at least this many kept values use it (INT32_MAX: off)
};

// Split-precision update products on the int8 matrix cores (k_crt.hip): per
// side (0 U, 1 V) the L residue planes of the row-scaled left operands (A,
// plane row = the node's row), of the column-scaled right operands of the top
// and bottom halves (Bt, Bb, plane row = the node's first column + the kept
// value's index), both k contiguous from 0 with row stride P, and of the
// products (C, column-major with ld ldr at the node's diagonal block); the
// largest |entry| per plane row (bits) and the scale exponents.
struct CrtWork {
  int8_t* A[2];
  int8_t* Bt[2];
  int8_t* Bb[2];
  int8_t* C[2];
  unsigned long long* amax[2];
  unsigned long long* btmax[2];
  unsigned long long* bbmax[2];
  int* Ea[2];
  int* Ebt[2];
  int* Ebb[2];
  int64_t planeA, planeB, planeC;  // bytes per modulus plane
  int P;                           // row stride (bytes) of the A and B planes
  int ldr;                         // leading dimension of the C planes
  int L;                           // moduli
};

// Device pointers of one call (passed to every kernel by value).
struct Work {
  const double* d;  // inputs, packed per problem at vec_off
  const double* e;
  double* Uw;  // working vectors, packed per problem at mat_off
  double* Vw;
  double* GU;  // gathered kept columns (caller's U buffer)
  double* GV;  // (caller's VT buffer)
  double* UM;
  double* VM;
  // per node-position arrays (packed at vec_off)
  double* sig;       // values of the node's sorted positions (unscaled)
  int32_t* col;      // physical column of each sorted position
  int32_t* ulo;      // row support of each physical column of Uwork: [ulo, uhi)
  int32_t* uhi;
  int32_t* vlo;      // and of Vwork
  int32_t* vhi;
  double* ps_d;      // merge scratch at sorted positions: value (scaled)
  double* ps_z;      //   z
  int32_t* ps_c;     //   node column (the children's sorted positions)
  int32_t* ps_col;   //   physical column
  int32_t* ps_sup;   //   1 left child, 2 both, 3 right child, 0 the new d = 0
  int32_t* status;   //   deflation status
  int32_t* ps_rot;   //   which side a deflation rotation touched (kRotU | kRotV)
  int32_t* cand;     // positions that pass the small-z test
  double* sd;        // kept values (scaled), ascending
  double* sz;        // kept z
  int32_t* scol;     // physical column of kept value i
  int32_t* srot;     // rotation flags of kept value i
  int32_t* sgrp;     // position of kept value i in the update order
  int32_t* gsurv;    // kept value at update position g
  double* dval;      // deflated values (scaled), ascending
  int32_t* dcol;     // their physical columns
  int32_t* drot;     // their rotation flags
  int32_t* o;        // secular roots: origin pole
  double* tau;       //   offset from it
  int32_t* iters;    //   evaluations
  double* zt;        // recomputed z
  int32_t* rot_pos;  // rotations: sorted positions (2 per rotation)
  int32_t* rot_col;  //   physical columns (2 per rotation)
  double* rot_cs;    //   (c, s)
  float* xs;         // caller-given start of each root in its interval, or nullptr
  unsigned long long* leaf_fl;  // per leaf: rotation flops (a plain store each, summed on the host)
  SecCount* sec;     // per node: secular statistics
  int4* fin;         // final pass of a single problem: per output index, (column, lo, hi) of U then of V
  const unsigned short* mlp_pk;  // packed network for the in-kernel learned start,
                                 // or nullptr
  OzWork oz;         // oz.min_n: merges with at least this many kept values take the
                     // split products (bfloat16 slices or int8 residues)
  CrtWork crt;
  int small_n;        // update products of merges with N <= small_n use 64 x 64 tiles
  int sec_small_n;    // secular problems with N <= sec_small_n use the lanes-per-root kernel
  int* tile_off64;    // flattened tile schedule of a level (nnodes + 1 each)
  int* tile_off128;
  NodeState* st;
  Ctl* ctl;
  int max_secular_iters;
  int max_leaf_sweeps;
  int learned_min_n;  // merges with fewer kept values skip the in-kernel network
};

// Caller buffers that collect training rows of the learned start.
struct Harvest {
  float* X;          // rows x BDC_MLP_FEATURES
  float* y;          // position of the computed root in its interval
  int32_t* tag;      // rows x 3: (problem offset + node r0, node m, root index)
  int64_t capacity;  // rows that fit; later rows are counted, not written
  unsigned long long* count;
};

// Launch configuration picked by the autotuner (see bdc_tuning_t).
struct Tuning {
  int small_n;  // 64 x 64 tiles for merges with N <= small_n, else 128 x 128
  int flat;     // 1: persistent grids over a flattened tile list; 0: grid per node
  int grid64;   // workgroups of the 64-tile update (flat), or twice the per-node cap
  int grid128;
  int sec_small_n;  // secular problems with N <= this (at most kSecLanesMaxN) use 8 or 16 lanes per root
  int tile128 = 1;  // 128 x 128 products (per-merge grids): 0 single-buffered tile, 1 double-buffered (default)
  int streams = 1;  // 2: each level's rotations and gather on a second stream (captured solves)
};

// Workspace layout of tn positions, tn2 matrix entries and nnodes merges
// carved from base (bytes returned; with w != NULL the pointers are set).
size_t work_layout(Work* w, char* base, int64_t tn, int64_t tn2, int nnodes);

// ---- launchers (defined next to their kernels) ----
void launch_reset(Ctl* ctl, NodeState* st, SecCount* sec, int nnodes, hipStream_t st_);
// leaves of at most max_m rows
void launch_leaf(const LeafDesc* leaves, int nleaves, int max_m, const Work& w, hipStream_t st);
void launch_prep(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, hipStream_t st);
void launch_rotate(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, hipStream_t st);
void launch_gather(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, hipStream_t st);
void launch_secular(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, hipStream_t st);
void launch_lowner(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, hipStream_t st);
void launch_vectors(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, hipStream_t st);
void launch_order(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, hipStream_t st);
void launch_update(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, const Tuning& tu,
                   hipStream_t st);
// Final pass: work items of U (groups of final_u_cols columns) and of V^T
// (bands x groups of column tiles, as above), numbered per problem from
// uitem_off / vitem_off, with item -> problem tables uprob / vprob.
void launch_final_single(int64_t n, const Work& w, double* sigma, double* U, double* VT, hipStream_t st);
void launch_final(const int64_t* prob_n, const int64_t* prob_vec, const int64_t* prob_mat,
                  const int64_t* uitem_off, const int64_t* vitem_off, const int32_t* uprob,
                  const int32_t* vprob, int64_t total_uitems, int64_t total_vitems, const Work& w,
                  double* sigma, double* U, double* VT, hipStream_t st);
// device and iteration options of a handle (BDC_OK or BDC_ERR_INVALID_HANDLE)
int handle_info(bdc_handle_t h, int* device, int* max_secular_iters, int* max_leaf_sweeps);
// the handle's secular small-problem threshold (launch tuning)
int handle_sec_small(bdc_handle_t h);

size_t mlp_pack_bytes();
void launch_mlp_pack(const float* params, unsigned short* packed, hipStream_t st);
void launch_harvest(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, const Harvest& hv,
                    hipStream_t st);
void launch_features(const double* d, const double* z, int N, float* X, hipStream_t st);
void launch_mlp_forward(const float* params, const float* X, int rows, float* xhat, hipStream_t st);
int mlp_parts(int rows);
void launch_mlp_grad(const float* params, const float* X, const float* y, const int32_t* idx, int rows,
                     float* part, float* part_loss, hipStream_t st);
void launch_adam(float* params, float* m, float* v, const float* part, int nparts, const float* part_loss,
                 float* grad_out, float* loss_out, int adam_t, float lr, float inv_rows, hipStream_t st);

int oz_supported(int slices);
void launch_update_ozaki(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, hipStream_t st);
void launch_gemm_ozaki_plain(int slices, int M, int N, int K, const double* A, int lda, const double* B, int ldb,
                             double* C, int ldc, unsigned short* sa, unsigned short* sb, int* ea, int* eb, int64_t P,
                             hipStream_t st);

void launch_update_crt(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, hipStream_t st);

void launch_gemm_plain(int M, int N, int K, const double* A, int lda, const double* B, int ldb,
                       double* C, int ldc, int tile128, hipStream_t st);
// the handle's 128 x 128 tile form (launch tuning)
int handle_tile128(bdc_handle_t h);

}  // namespace bdc
