// Vector side of a merge and the final output.
//   k_rotate   applies the deflation rotations (Algorithm 3's rotation step)
//              row-parallel: one thread per row of the node applies the whole
//              list in order.  Columns touched are first zero-filled outside
//              their support so the rotated columns are dense over the node.
//   k_gather   copies the kept columns, in update order [left-only | d = 0 |
//              mixed | right-only], into the compact GU / GV blocks (a node's
//              columns as one flattened element range).  Deflated columns are
//              not moved at all.
//   k_order    merges the roots with the deflated values (Algorithm 2 step
//              (3)'s sort, done per node), records each sorted position's
//              physical column and updates the supports.
//   k_update   the vector update of eq. bdc-Mv2Bv-u-vt as FP64 matrix-core
//              GEMMs.  With the update order above, the rows of the left
//              child's block need only the columns [left-only | d=0 | mixed]
//              and the right child's rows only [d=0 | mixed | right-only]: two
//              contiguous products per side instead of the paper's three.
//              Results are written straight into the kept columns' physical
//              places, scaled to unit length already.
//   k_final_u / k_final_vt  write sigma, U and V^T in descending order
//              (the root's ascending order reversed), expanding each column's
//              support to the full matrix; V^T goes through an LDS transpose.
#include <algorithm>

#include "bdc_internal.h"
#include "block_util.h"

namespace bdc {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

inline int grid_y(int nnodes, int units, int cap_total) {
  int gy = units;
  int cap = cap_total / (nnodes > 0 ? nnodes : 1);
  if (cap < 1) cap = 1;
  if (gy > cap) gy = cap;
  if (gy < 1) gy = 1;
  if (gy > 65535) gy = 65535;
  return gy;
}

// ------------------------------------------------------------------ rotate
__global__ __launch_bounds__(256) void k_rotate(const NodeDesc* __restrict__ nodes, Work w) {
  const NodeDesc nd = nodes[blockIdx.x];
  const int nrot = w.st[nd.id].nrot;
  if (nrot == 0) return;
  const int m = nd.m, s = nd.s, r0 = nd.r0;
  const int64_t ld = nd.ld, pv = nd.vec_off;
  const int64_t rb = 2 * (nd.vec_off + nd.r0);
  double* U = w.Uw + nd.mat_off;
  double* V = w.Vw + nd.mat_off;
  for (int row = blockIdx.y * kBlock + threadIdx.x; row < m + s; row += gridDim.y * kBlock) {
    const int gr = r0 + row;
    const bool inU = row < m;
    // zero-fill the touched columns outside their current support
    for (int q = 0; q < nrot; ++q) {
      const bool both = w.rot_pos[rb + 2 * q] != 0;
      for (int h = 0; h < 2; ++h) {
        const int pc = w.rot_col[rb + 2 * q + h];
        if (both && inU && (gr < w.ulo[pv + pc] || gr >= w.uhi[pv + pc])) U[gr + pc * ld] = 0.0;
        if (gr < w.vlo[pv + pc] || gr >= w.vhi[pv + pc]) V[gr + pc * ld] = 0.0;
      }
    }
    for (int q = 0; q < nrot; ++q) {
      const bool both = w.rot_pos[rb + 2 * q] != 0;
      const int pp = w.rot_col[rb + 2 * q], pj = w.rot_col[rb + 2 * q + 1];
      const double c = w.rot_cs[rb + 2 * q], sn = w.rot_cs[rb + 2 * q + 1];
      if (both && inU) {
        const double a = U[gr + pp * ld], b = U[gr + pj * ld];
        U[gr + pp * ld] = c * a + sn * b;
        U[gr + pj * ld] = -sn * a + c * b;
      }
      const double a = V[gr + pp * ld], b = V[gr + pj * ld];
      V[gr + pp * ld] = c * a + sn * b;
      V[gr + pj * ld] = -sn * a + c * b;
    }
  }
}

// ------------------------------------------------------------------ gather
// The node's kept columns in update order, both sides, as one flattened
// range of N (m + s) elements (column g, row r) -> g (m + s) + r; a workgroup
// takes slabs of kGatherSlab consecutive elements (four per thread, loads
// issued before the stores), so that few long columns and many short ones
// alike fill the workgroups.  U rows run to m, V rows to m + s.
constexpr int kGatherSlab = 4 * kBlock;

__global__ __launch_bounds__(256) void k_gather(const NodeDesc* __restrict__ nodes, Work w) {
  const NodeDesc nd = nodes[blockIdx.x];
  const int N = w.st[nd.id].N;
  const int m = nd.m, s = nd.s, r0 = nd.r0, k = nd.k;
  const int R = m + s;
  const int64_t ld = nd.ld, pv = nd.vec_off, vo = nd.vec_off + nd.r0;
  const double* U = w.Uw + nd.mat_off;
  const double* V = w.Vw + nd.mat_off;
  double* GU = w.GU + nd.mat_off;
  double* GV = w.GV + nd.mat_off;
  const int64_t total = (int64_t)N * R;
  const int64_t units = (total + kGatherSlab - 1) / kGatherSlab;
  const double inv_r = 1.0 / (double)R;
  for (int64_t u = blockIdx.y; u < units; u += gridDim.y) {
    double xu[4], xv[4];
    int gq[4], rq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t e = u * kGatherSlab + q * kBlock + threadIdx.x;
      gq[q] = -1;
      rq[q] = 0;
      xu[q] = xv[q] = 0.0;
      if (e >= total) continue;
      int g = (int)((double)e * inv_r);
      if ((int64_t)g * R > e) --g;
      else if ((int64_t)(g + 1) * R <= e) ++g;
      const int row = (int)(e - (int64_t)g * R);
      gq[q] = g;
      rq[q] = row;
      const int i = w.gsurv[vo + g];
      const int gr = r0 + row;
      if (i == 0) {
        // d = 0 position: left vector e_{k-1} (the middle row), right vector x1
        xu[q] = (row == k - 1) ? 1.0 : 0.0;
        xv[q] = V[gr + (int64_t)(r0 + k - 1) * ld];
      } else {
        const int64_t pc = w.scol[vo + i];
        const int rf = w.srot[vo + i];
        const bool fu = (rf & kRotU) != 0, fv = (rf & kRotV) != 0;
        const int ul = fu ? r0 : w.ulo[pv + pc], uh = fu ? r0 + m : w.uhi[pv + pc];
        const int vl = fv ? r0 : w.vlo[pv + pc], vh = fv ? r0 + m + s : w.vhi[pv + pc];
        xu[q] = (row < m && gr >= ul && gr < uh) ? U[gr + pc * ld] : 0.0;
        xv[q] = (gr >= vl && gr < vh) ? V[gr + pc * ld] : 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (gq[q] < 0) continue;
      const int64_t off = r0 + rq[q] + (int64_t)(r0 + gq[q]) * ld;
      if (rq[q] < m) GU[off] = xu[q];
      GV[off] = xv[q];
    }
  }
}

// ------------------------------------------------------------------ order
__device__ inline double root_value(const double* d, const int* o, const double* tau, int i) {
  return d[o[i]] + tau[i];
}

__device__ inline void order_node(const NodeDesc& nd, const Work& w) {
  const NodeState st = w.st[nd.id];
  const int N = st.N, m = nd.m, s = nd.s, r0 = nd.r0, D = nd.m - st.N;
  const int64_t pv = nd.vec_off, vo = nd.vec_off + nd.r0;
  const double* d = w.sd + vo;
  const int* o = w.o + vo;
  const double* tau = w.tau + vo;
  const double* dv = w.dval + vo;
  const double p = st.scale;
  for (int idx = blockIdx.y * kBlock + threadIdx.x; idx < m; idx += gridDim.y * kBlock) {
    if (idx < N) {
      const int i = idx;
      const double wi = root_value(d, o, tau, i);
      int lo = 0, hi = D;  // deflated values strictly below w_i
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (dv[mid] < wi) lo = mid + 1;
        else hi = mid;
      }
      const int dest = i + lo;
      const int pc = w.scol[vo + i];
      w.sig[vo + dest] = wi * p;
      w.col[vo + dest] = pc;
      w.ulo[pv + pc] = r0;
      w.uhi[pv + pc] = r0 + m;
      w.vlo[pv + pc] = r0;
      w.vhi[pv + pc] = r0 + m + s;
    } else {
      const int q = idx - N;
      const double v = dv[q];
      int lo = 0, hi = N;  // roots at or below v (roots first on ties)
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (root_value(d, o, tau, mid) <= v) lo = mid + 1;
        else hi = mid;
      }
      const int dest = q + lo;
      const int pc = w.dcol[vo + q];
      w.sig[vo + dest] = v * p;
      w.col[vo + dest] = pc;
      const int rf = w.drot[vo + q];
      if (rf & kRotU) {  // rotated columns were made dense over the node
        w.ulo[pv + pc] = r0;
        w.uhi[pv + pc] = r0 + m;
      }
      if (rf & kRotV) {
        w.vlo[pv + pc] = r0;
        w.vhi[pv + pc] = r0 + m + s;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_order(const NodeDesc* __restrict__ nodes, Work w) {
  order_node(nodes[blockIdx.x], w);
}

// ------------------------------------------------------------------ GEMM
// TM x TN output tile per 256-thread workgroup: four wavefronts in 2 x 2, each
// owning a (TM/2) x (TN/2) block as (TM/32) x (TN/32) v_mfma_f64_16x16x4f64
// tiles.  A (M x K) and B (K x N) are column-major; 16-deep K slabs are staged
// in LDS, and the next slab is loaded into registers while the current one is
// multiplied.
constexpr int TK = 16;

// the 64 x 64 output tile is turned around in LDS for the stores, half its
// columns at a time (column stride kCt doubles: 16-byte aligned, spreads the
// writes over the banks).  The half-tile buffer is no larger than the two
// K slabs it shares the LDS with: 17 KB per workgroup, so LDS admits eight
// workgroups per CU as the registers do (the whole tile's 34 KB held it to
// four, and the small merges of a batch, a latency chain of K slabs per
// tile, run at the number of tiles in flight).
constexpr int kCt = 66;

template <int TM, int TN>
struct TileSmem {
  union {
    struct {
      double A[TK * TM];
      double B[TK * TN];
    } ab;
    double C[TM <= 64 ? (TN / 2) * kCt : 1];
  };
};

template <int TM, int TN, class Store>
__device__ inline void gemm_tile(TileSmem<TM, TN>& sm, const double* __restrict__ A, int64_t lda,
                                 const double* __restrict__ B, int64_t ldb, int M, int N, int K,
                                 int tm0, int tn0, Store store) {
  constexpr int FA = TM * TK / kBlock;  // A elements per thread per slab
  constexpr int FB = TN * TK / kBlock;
  constexpr int BM = TM / 32, BN = TN / 32;  // 16x16 blocks per wavefront
  // slabs of registers in flight: one ahead of the slab being multiplied
  // (deeper prefetch measured slower here: the registers cost occupancy)
  constexpr int P = 1;
  const int t = threadIdx.x, wv = t >> 6, l = t & 63;
  const int wm = wv & 1, wn = wv >> 1;
  const int li = l & 15, lk = l >> 4;
  v4d acc[BM][BN];
#pragma unroll
  for (int a = 0; a < BM; ++a)
#pragma unroll
    for (int b = 0; b < BN; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  double ra[P][FA], rb[P][FB];
  auto load = [&](double (&xa)[FA], double (&xb)[FB], int k0) {
#pragma unroll
    for (int q = 0; q < FA; ++q) {
      const int e = t + kBlock * q;
      const int r = e % TM, kk = e / TM;
      const int gr = tm0 + r, gk = k0 + kk;
      xa[q] = (gr < M && gk < K) ? A[gr + (int64_t)gk * lda] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < FB; ++q) {
      const int e = t + kBlock * q;
      const int kk = e % TK, c = e / TK;
      const int gk = k0 + kk, gc = tn0 + c;
      xb[q] = (gk < K && gc < N) ? B[gk + (int64_t)gc * ldb] : 0.0;
    }
  };
  const int nslab = (K + TK - 1) / TK;
#pragma unroll
  for (int p = 0; p < P; ++p)
    if (p < nslab) load(ra[p], rb[p], p * TK);
  for (int s0 = 0; s0 < nslab; s0 += P) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int sl = s0 + p;
      if (sl >= nslab) break;
      __syncthreads();
#pragma unroll
      for (int q = 0; q < FA; ++q) {
        const int e = t + kBlock * q;
        sm.ab.A[(e / TM) * TM + e % TM] = ra[p][q];
      }
#pragma unroll
      for (int q = 0; q < FB; ++q) {
        const int e = t + kBlock * q;
        sm.ab.B[(e % TK) * TN + e / TK] = rb[p][q];
      }
      __syncthreads();
      if (sl + P < nslab) load(ra[p], rb[p], (sl + P) * TK);
#pragma unroll
      for (int kk = 0; kk < TK; kk += 4) {
        double af[BM], bf[BN];
#pragma unroll
        for (int a = 0; a < BM; ++a) af[a] = sm.ab.A[(kk + lk) * TM + wm * (TM / 2) + a * 16 + li];
#pragma unroll
        for (int b = 0; b < BN; ++b) bf[b] = sm.ab.B[(kk + lk) * TN + wn * (TN / 2) + b * 16 + li];
#pragma unroll
        for (int a = 0; a < BM; ++a)
#pragma unroll
          for (int b = 0; b < BN; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
      }
    }
  }
  // D[i][j] of a 16x16 block sits in lane j + 16 * (i % 4), register i / 4
  // (checked against a host product)
  if constexpr (TM <= 64) {
    // through LDS, one column half (the two wavefronts that own it) at a
    // time: each output column's 64 rows leave as one 512-byte run (32
    // lanes x 16 bytes), two columns per store instruction
    constexpr int TH = TN / 2;
    const int half = l >> 5, rr = 2 * (l & 31);
    const int grow = tm0 + rr;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      __syncthreads();
      if (wn == h) {
#pragma unroll
        for (int a = 0; a < BM; ++a)
#pragma unroll
          for (int b = 0; b < BN; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              sm.C[(b * 16 + li) * kCt + wm * (TM / 2) + a * 16 + lk + 4 * r] = acc[a][b][r];
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < TH / 8; ++q) {
        const int c = wv * (TH / 4) + 2 * q + half;
        const int colc = tn0 + h * TH + c;
        if (colc >= N) continue;
        double* dst = store.col(colc);
        const double2 v = *reinterpret_cast<const double2*>(&sm.C[c * kCt + rr]);
        if (grow + 1 < M) {
          dst[grow] = v.x;
          dst[grow + 1] = v.y;
        } else if (grow < M) {
          dst[grow] = v.x;
        }
      }
    }
    __syncthreads();
  } else {
#pragma unroll
    for (int a = 0; a < BM; ++a)
#pragma unroll
      for (int b = 0; b < BN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = tm0 + wm * (TM / 2) + a * 16 + lk + 4 * r;
          const int colc = tn0 + wn * (TN / 2) + b * 16 + li;
          if (row < M && colc < N) *(store.col(colc) + row) = acc[a][b][r];
        }
  }
}

// Second form of the 128 x 128 tile: both 16-deep slabs double-buffered in
// LDS (one barrier per slab: the next slab's global loads are issued before
// the current slab's products and land in the other buffer after them), and
// laid out so that neither the stores nor the operand reads conflict on the
// LDS banks: A as [k][m] with a row stride of 144 doubles (the two k rows of
// a half-wavefront's read are 32 banks apart), B as [n][k] with a column
// stride of 17 doubles (k contiguous as in memory; the 16 columns of a read
// fall on distinct banks).  70 KB of LDS; one workgroup per CU (the 64
// accumulators per lane need more registers than two would leave).
constexpr int kSA2 = 144, kSB2 = 17;
struct TileSmem2 {
  double A[2][TK * kSA2];
  double B[2][128 * kSB2];
};

template <class Store>
__device__ inline void gemm_tile2(TileSmem2& sm, const double* __restrict__ A, int64_t lda,
                                  const double* __restrict__ B, int64_t ldb, int M, int N, int K, int tm0, int tn0,
                                  Store store) {
  constexpr int TM = 128, TN = 128;
  constexpr int FA = TM * TK / kBlock, FB = TN * TK / kBlock;
  const int t = threadIdx.x, wv = t >> 6, l = t & 63;
  const int wm = wv & 1, wn = wv >> 1;
  const int li = l & 15, lk = l >> 4;
  v4d acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  double ra[FA], rb[FB];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < FA; ++q) {
      const int e = t + kBlock * q;
      const int r = e % TM, kk = e / TM;
      const int gr = tm0 + r, gk = k0 + kk;
      ra[q] = (gr < M && gk < K) ? A[gr + (int64_t)gk * lda] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < FB; ++q) {
      const int e = t + kBlock * q;
      const int kk = e % TK, c = e / TK;
      const int gk = k0 + kk, gc = tn0 + c;
      rb[q] = (gk < K && gc < N) ? B[gk + (int64_t)gc * ldb] : 0.0;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int q = 0; q < FA; ++q) {
      const int e = t + kBlock * q;
      sm.A[buf][(e / TM) * kSA2 + e % TM] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < FB; ++q) {
      const int e = t + kBlock * q;
      sm.B[buf][(e / TK) * kSB2 + e % TK] = rb[q];
    }
  };
  const int nslab = (K + TK - 1) / TK;
  __syncthreads();  // the previous tile's readers are done with both buffers
  load(0);
  stash(0);
  __syncthreads();
  for (int sl = 0; sl < nslab; ++sl) {
    const int buf = sl & 1;
    if (sl + 1 < nslab) load((sl + 1) * TK);
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      double af[4], bf[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) af[a] = sm.A[buf][(kk + lk) * kSA2 + wm * 64 + a * 16 + li];
#pragma unroll
      for (int b = 0; b < 4; ++b) bf[b] = sm.B[buf][(wn * 64 + b * 16 + li) * kSB2 + kk + lk];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
    if (sl + 1 < nslab) {
      stash(buf ^ 1);
      __syncthreads();
    }
  }
  // D[i][j] of a 16x16 block sits in lane j + 16 * (i % 4), register i / 4
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = tm0 + wm * 64 + a * 16 + lk + 4 * r;
        const int colc = tn0 + wn * 64 + b * 16 + li;
        if (row < M && colc < N) *(store.col(colc) + row) = acc[a][b][r];
      }
}

// destination of output column c (row 0): the kept value's physical column
struct NodeStore {
  double* C;
  const int* scol;
  int64_t ld;
  int rowbase;
  __device__ double* col(int c) const { return C + rowbase + (int64_t)scol[c] * ld; }
};

// Nodes whose kept size N is at most w.small_n use 64 x 64 tiles, larger ones
// 128 x 128 (tunable); each launch skips the nodes of the other class.

// grid: (node, tile slot, side-half).  side-half: 0 U rows [0,k), 1 U rows
// [k,m), 2 V rows [0,k), 3 V rows [k,m+s); the 64-tile launch has a fifth
// slice z = 4 whose workgroups do k_order's work (it touches none of the
// products' data), saving a launch per level.  Tiles are visited with the row
// index fastest, so the workgroups on one XCD (every 8th) share B panels.
// The 64-tile class is held to four wavefronts per SIMD (126 registers, no
// spills; unbounded it takes 168 and three): the small merges of a level are
// thousands of short workgroups, and residency decides their time.
constexpr int update_waves_per_eu(int tm) { return tm <= 64 ? 4 : 1; }

template <int TM, int TN>
__global__ __launch_bounds__(256, update_waves_per_eu(TM)) void k_update(const NodeDesc* __restrict__ nodes,
                                                                          Work w) {
  __shared__ TileSmem<TM, TN> sm;
  const NodeDesc nd = nodes[blockIdx.x];
  if (blockIdx.z == 4) {  // the 64-tile launch also carries the node's k_order work
    order_node(nd, w);
    return;
  }
  const NodeState st = w.st[nd.id];
  const int N = st.N, n1 = st.n1, n2 = st.n2;
  if ((TM <= 64) != (N <= w.small_n)) return;
  if (N >= w.oz.min_n) return;  // done by the split-precision products
  const int m = nd.m, s = nd.s, k = nd.k, r0 = nd.r0;
  const int64_t ld = nd.ld, vo = nd.vec_off + nd.r0;
  const int sub = blockIdx.z;
  const bool isV = sub >= 2, bottom = sub & 1;
  const int rows = bottom ? (isV ? m + s - k : m - k) : k;
  const int kb = bottom ? n1 : 0;
  const int ke = bottom ? N : n1 + 1 + n2;
  const int K = ke - kb;
  const int rowoff = bottom ? k : 0;
  const double* G = (isV ? w.GV : w.GU) + nd.mat_off;
  const double* Mv = (isV ? w.VM : w.UM) + nd.mat_off;
  const double* A = G + (r0 + rowoff) + (int64_t)(r0 + kb) * ld;
  const double* B = Mv + (r0 + kb) + (int64_t)r0 * ld;
  NodeStore store{(isV ? w.Vw : w.Uw) + nd.mat_off, w.scol + vo, ld, r0 + rowoff};
  const int tiles_m = (rows + TM - 1) / TM, tiles_n = (N + TN - 1) / TN;
  const int ntiles = tiles_m * tiles_n;
  for (int tile = blockIdx.y; tile < ntiles; tile += gridDim.y) {
    const int tm = tile % tiles_m, tn = tile / tiles_m;
    gemm_tile<TM, TN>(sm, A, ld, B, ld, rows, N, K, tm * TM, tn * TN, store);
  }
}

// The 128 x 128 class with the double-buffered tile (two workgroups per CU).
__global__ __launch_bounds__(256, 1) void k_update2(const NodeDesc* __restrict__ nodes, Work w) {
  __shared__ TileSmem2 sm;
  const NodeDesc nd = nodes[blockIdx.x];
  const NodeState st = w.st[nd.id];
  const int N = st.N, n1 = st.n1, n2 = st.n2;
  if (N <= w.small_n) return;
  if (N >= w.oz.min_n) return;  // done by the split-precision products
  const int m = nd.m, s = nd.s, k = nd.k, r0 = nd.r0;
  const int64_t ld = nd.ld, vo = nd.vec_off + nd.r0;
  const int sub = blockIdx.z;
  const bool isV = sub >= 2, bottom = sub & 1;
  const int rows = bottom ? (isV ? m + s - k : m - k) : k;
  const int kb = bottom ? n1 : 0;
  const int ke = bottom ? N : n1 + 1 + n2;
  const int K = ke - kb;
  const int rowoff = bottom ? k : 0;
  const double* G = (isV ? w.GV : w.GU) + nd.mat_off;
  const double* Mv = (isV ? w.VM : w.UM) + nd.mat_off;
  const double* A = G + (r0 + rowoff) + (int64_t)(r0 + kb) * ld;
  const double* B = Mv + (r0 + kb) + (int64_t)r0 * ld;
  NodeStore store{(isV ? w.Vw : w.Uw) + nd.mat_off, w.scol + vo, ld, r0 + rowoff};
  const int tiles_m = (rows + 127) / 128, tiles_n = (N + 127) / 128;
  for (int tile = blockIdx.y; tile < tiles_m * tiles_n; tile += gridDim.y) {
    const int tm = tile % tiles_m, tn = tile / tiles_m;
    gemm_tile2(sm, A, ld, B, ld, rows, N, K, tm * 128, tn * 128, store);
  }
}

// Levels whose merges are all at most 16 B values (rows and kept columns of
// every side-half <= 16 B): one workgroup per node, wavefront q the
// side-half q (U rows [0,k), U rows [k,m), V rows [0,k), V rows [k,m+s)) as
// one (16 B) x (16 B) output of B x B v_mfma_f64_16x16x4f64 blocks with its
// operands read straight from the gathered columns, then the node's k_order
// work.  The k-steps run in the order of the 64-tile products (k = 0, 4, 8,
// ...), so the sums are the same.  A level of many tiny merges takes one
// short workgroup per node instead of five 64 x 64 tiles that are mostly
// padding.
template <int B>
__global__ __launch_bounds__(256) void k_update_wave(const NodeDesc* __restrict__ nodes, Work w) {
  constexpr int TW = 16 * B;
  const NodeDesc nd = nodes[blockIdx.x];
  const int sub = threadIdx.x >> 6, l = threadIdx.x & 63;
  const NodeState st = w.st[nd.id];
  const int N = st.N, n1 = st.n1, n2 = st.n2;
  if (N < w.oz.min_n) {  // larger kept sizes are done by the split-precision products
    const int m = nd.m, s = nd.s, k = nd.k, r0 = nd.r0;
    const int64_t ld = nd.ld, vo = nd.vec_off + nd.r0;
    const bool isV = sub >= 2, bottom = sub & 1;
    const int rows = bottom ? (isV ? m + s - k : m - k) : k;
    const int kb = bottom ? n1 : 0;
    const int ke = bottom ? N : n1 + 1 + n2;
    const int K = ke - kb;
    const int rowoff = bottom ? k : 0;
    const double* G = (isV ? w.GV : w.GU) + nd.mat_off;
    const double* Mv = (isV ? w.VM : w.UM) + nd.mat_off;
    const double* __restrict__ A = G + (r0 + rowoff) + (int64_t)(r0 + kb) * ld;
    const double* __restrict__ Bm = Mv + (r0 + kb) + (int64_t)r0 * ld;
    NodeStore store{(isV ? w.Vw : w.Uw) + nd.mat_off, w.scol + vo, ld, r0 + rowoff};
    const int li = l & 15, lk = l >> 4;
    v4d acc[B][B];
#pragma unroll
    for (int a = 0; a < B; ++a)
#pragma unroll
      for (int b = 0; b < B; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int gk = k0 + lk;
      double af[B], bf[B];
#pragma unroll
      for (int a = 0; a < B; ++a) {
        const int row = a * 16 + li;
        af[a] = (row < rows && gk < K) ? A[row + (int64_t)gk * ld] : 0.0;
      }
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int col = b * 16 + li;
        bf[b] = (gk < K && col < N) ? Bm[gk + (int64_t)col * ld] : 0.0;
      }
#pragma unroll
      for (int a = 0; a < B; ++a)
#pragma unroll
        for (int b = 0; b < B; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
    // D[i][j] of a 16x16 block sits in lane j + 16 (i % 4), register i / 4
#pragma unroll
    for (int a = 0; a < B; ++a)
#pragma unroll
      for (int b = 0; b < B; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = a * 16 + lk + 4 * r, col = b * 16 + li;
          if (row < rows && col < N) *(store.col(col) + row) = acc[a][b][r];
        }
    static_assert(TW >= 16, "tile");
  }
  order_node(nd, w);
}

// ---- flattened schedule: all tiles of a level in one list per tile class.
// Tiles of a node, sub-half by sub-half (0 U rows [0,k), 1 U rows [k,m),
// 2 V rows [0,k), 3 V rows [k,m+s)), row index fastest.
__device__ inline int sub_rows(const NodeDesc& nd, int sub) {
  const bool isV = sub >= 2, bottom = sub & 1;
  return bottom ? (isV ? nd.m + nd.s - nd.k : nd.m - nd.k) : nd.k;
}

template <int T>
__device__ inline int node_tiles(const NodeDesc& nd, int N) {
  const int tn = (N + T - 1) / T;
  int c = 0;
  for (int sub = 0; sub < 4; ++sub) c += ((sub_rows(nd, sub) + T - 1) / T) * tn;
  return c;
}

// Tile offsets of the level's nodes in the 64 and 128 classes
// (off64/off128[i] .. [i+1]); one workgroup.
__global__ __launch_bounds__(256) void k_tile_sched(const NodeDesc* __restrict__ nodes, int nnodes, Work w) {
  __shared__ int sh[2 * kBlock];
  const int t = threadIdx.x;
  const int per = (nnodes + kBlock - 1) / kBlock;
  const int i0 = min(nnodes, t * per), i1 = min(nnodes, i0 + per);
  int v[2] = {0, 0};
  for (int i = i0; i < i1; ++i) {
    const NodeDesc nd = nodes[i];
    const int N = w.st[nd.id].N;
    if (N >= w.oz.min_n || N == 0) continue;
    if (N <= w.small_n) v[0] += node_tiles<64>(nd, N);
    else v[1] += node_tiles<128>(nd, N);
  }
  int tot[2];
  block_exscan_w<2, kBlock>(v, tot, sh);
  int o64 = v[0], o128 = v[1];
  for (int i = i0; i < i1; ++i) {
    w.tile_off64[i] = o64;
    w.tile_off128[i] = o128;
    const NodeDesc nd = nodes[i];
    const int N = w.st[nd.id].N;
    if (N >= w.oz.min_n || N == 0) continue;
    if (N <= w.small_n) o64 += node_tiles<64>(nd, N);
    else o128 += node_tiles<128>(nd, N);
  }
  if (t == 0) {
    w.tile_off64[nnodes] = tot[0];
    w.tile_off128[nnodes] = tot[1];
  }
}

// Persistent form of k_update: a fixed grid walks the level's flattened tile
// list of its class.
template <int TM, int TN>
__global__ __launch_bounds__(256, update_waves_per_eu(TM)) void k_update_flat(const NodeDesc* __restrict__ nodes, int nnodes, Work w) {
  __shared__ TileSmem<TM, TN> sm;
  const int* __restrict__ off = TM <= 64 ? w.tile_off64 : w.tile_off128;
  const int total = off[nnodes];
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    // node holding tile t: last i with off[i] <= t
    int lo = 0, hi = nnodes;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (off[mid] <= t) lo = mid;
      else hi = mid;
    }
    const NodeDesc nd = nodes[lo];
    const NodeState st = w.st[nd.id];
    const int N = st.N, n1 = st.n1, n2 = st.n2;
    const int tn_count = (N + TN - 1) / TN;
    int local = t - off[lo];
    int sub = 0, rows = sub_rows(nd, 0);
    for (;;) {
      const int c = ((rows + TM - 1) / TM) * tn_count;
      if (local < c || sub == 3) break;
      local -= c;
      ++sub;
      rows = sub_rows(nd, sub);
    }
    const int tiles_m = (rows + TM - 1) / TM;
    const int tm = local % tiles_m, tn = local / tiles_m;
    const bool isV = sub >= 2, bottom = sub & 1;
    const int kb = bottom ? n1 : 0;
    const int ke = bottom ? N : n1 + 1 + n2;
    const int rowoff = bottom ? nd.k : 0;
    const int64_t ld = nd.ld, vo = nd.vec_off + nd.r0;
    const double* G = (isV ? w.GV : w.GU) + nd.mat_off;
    const double* Mv = (isV ? w.VM : w.UM) + nd.mat_off;
    const double* A = G + (nd.r0 + rowoff) + (int64_t)(nd.r0 + kb) * ld;
    const double* B = Mv + (nd.r0 + kb) + (int64_t)nd.r0 * ld;
    NodeStore store{(isV ? w.Vw : w.Uw) + nd.mat_off, w.scol + vo, ld, nd.r0 + rowoff};
    gemm_tile<TM, TN>(sm, A, ld, B, ld, rows, N, ke - kb, tm * TM, tn * TN, store);
  }
}

struct PlainStore {
  double* C;
  int64_t ldc;
  __device__ double* col(int c) const { return C + (int64_t)c * ldc; }
};

template <int TM, int TN>
__global__ __launch_bounds__(256) void k_gemm_plain(int M, int N, int K, const double* A, int lda,
                                                     const double* B, int ldb, double* C, int ldc) {
  __shared__ TileSmem<TM, TN> sm;
  const int tiles_m = (M + TM - 1) / TM, tiles_n = (N + TN - 1) / TN;
  for (int tile = blockIdx.x; tile < tiles_m * tiles_n; tile += gridDim.x) {
    const int tm = tile % tiles_m, tn = tile / tiles_m;
    gemm_tile<TM, TN>(sm, A, lda, B, ldb, M, N, K, tm * TM, tn * TN, PlainStore{C, ldc});
  }
}

__global__ __launch_bounds__(256, 1) void k_gemm_plain2(int M, int N, int K, const double* A, int lda,
                                                        const double* B, int ldb, double* C, int ldc) {
  __shared__ TileSmem2 sm;
  const int tiles_m = (M + 127) / 128, tiles_n = (N + 127) / 128;
  for (int tile = blockIdx.x; tile < tiles_m * tiles_n; tile += gridDim.x) {
    const int tm = tile % tiles_m, tn = tile / tiles_m;
    gemm_tile2(sm, A, lda, B, ldb, M, N, K, tm * 128, tn * 128, PlainStore{C, ldc});
  }
}

// ------------------------------------------------------------------ final
// U: a work item is a group of final_u_cols(n) output columns (one column
// for n >= 16384, up to 64 short columns otherwise), in descending order.
// Single columns are written in row pairs with 16-byte stores (four in flight
// per thread); a group of short columns as one contiguous range.
__global__ __launch_bounds__(256) void k_final_u(const int64_t* __restrict__ pn,
                                                 const int64_t* __restrict__ pvec,
                                                 const int64_t* __restrict__ pmat,
                                                 const int64_t* __restrict__ uitem_off,
                                                 const int32_t* __restrict__ uprob, Work w, double* sigma,
                                                 double* U) {
  __shared__ int64_t s_pc[64];
  __shared__ int s_ul[64], s_uh[64];
  const int64_t item = blockIdx.x;
  const int prob = uprob[item];
  const int64_t n = pn[prob], pv = pvec[prob], mo = pmat[prob];
  const int G = final_u_cols(n);
  const int64_t c0 = (item - uitem_off[prob]) * G;
  const int cols = (int)min((int64_t)G, n - c0);
  if (cols <= 0) return;
  if (G > 1) {
    const int t = threadIdx.x;
    if (t < cols) {
      const int64_t tcol = c0 + t, src = n - 1 - tcol;
      const int64_t pc = w.col[pv + src];
      s_pc[t] = pc;
      s_ul[t] = w.ulo[pv + pc];
      s_uh[t] = w.uhi[pv + pc];
      sigma[pv + tcol] = w.sig[pv + src];
    }
    __syncthreads();
    double* __restrict__ out = U + mo + c0 * n;
    const double* __restrict__ Uw = w.Uw + mo;
    const int nn = (int)n, tot = cols * nn;
    // four reads in flight per thread before their stores
    for (int e0 = t; e0 < tot; e0 += 4 * kBlock) {
      double v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = e0 + q * kBlock;
        v[q] = 0.0;
        if (e < tot) {
          const int col = e / nn, row = e - col * nn;
          if (row >= s_ul[col] && row < s_uh[col]) v[q] = Uw[s_pc[col] * n + row];
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (e0 + q * kBlock < tot) out[e0 + q * kBlock] = v[q];
    }
    return;
  }
  const int64_t tcol = c0;
  const int64_t src = n - 1 - tcol;
  const int64_t pc = w.col[pv + src];
  const int64_t ul = w.ulo[pv + pc], uh = w.uhi[pv + pc];
  if (threadIdx.x == 0) sigma[pv + tcol] = w.sig[pv + src];
  const double* in = w.Uw + mo + pc * n;
  double* out = U + mo + tcol * n;
  if ((((uintptr_t)out) & 15) == 0 && (((uintptr_t)in) & 15) == 0) {
    const int64_t n2 = n >> 1;
    double2* o2 = reinterpret_cast<double2*>(out);
    const double2* i2 = reinterpret_cast<const double2*>(in);
    // four 16-byte stores in flight per thread
    for (int64_t b2 = threadIdx.x; b2 < n2; b2 += 4 * kBlock) {
      double2 v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r2 = b2 + q * kBlock, r = 2 * r2;
        v[q] = make_double2(0.0, 0.0);
        if (r2 < n2 && r + 1 >= ul && r < uh) {
          if (r >= ul && r + 1 < uh) {
            v[q] = i2[r2];
          } else {
            v[q].x = (r >= ul && r < uh) ? in[r] : 0.0;
            v[q].y = (r + 1 >= ul && r + 1 < uh) ? in[r + 1] : 0.0;
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (b2 + q * kBlock < n2) o2[b2 + q * kBlock] = v[q];
    }
    if ((n & 1) && threadIdx.x == 0) {
      const int64_t r = n - 1;
      out[r] = (r >= ul && r < uh) ? in[r] : 0.0;
    }
  } else {
    for (int64_t r = threadIdx.x; r < n; r += kBlock) out[r] = (r >= ul && r < uh) ? in[r] : 0.0;
  }
}

// V^T: bands of kVtBand output rows (singular vectors); a workgroup takes
// one band and kVtTilesPerGroup tiles of kVtTile output columns.  Each
// vector's kVtTile-entry run of its Vwork column is read inside its support
// only (eight threads per 128-byte run, two entries each; entries outside
// the support are zeros without a read), the tile is turned around in LDS
// and each output column's kVtBand rows leave as one 2 KB run (non-temporal
// stores: written once, they would only displace the reads).  The next
// tile's reads are issued before the current tile's LDS round trip and
// stores.  Measured on the 2000-problem batch, this shape beats 64 x 64
// tiles (512-byte runs), 512 x 8 tiles and one entry per lane.
__global__ __launch_bounds__(256) void k_final_vt(const int64_t* __restrict__ pn,
                                                  const int64_t* __restrict__ pvec,
                                                  const int64_t* __restrict__ pmat,
                                                  const int64_t* __restrict__ vitem_off,
                                                  const int32_t* __restrict__ vprob, Work w, double* VT) {
  static_assert(kVtBand == kBlock && kVtTile == 16, "one vector per thread, eight threads per run");
  constexpr int kPass = kVtBand / (kBlock / 8);  // vectors per thread in the reads
  __shared__ double tileS[kVtTile][kVtBand + 1];
  __shared__ int pcs[kVtBand], lov[kVtBand], hiv[kVtBand];
  const int64_t gt = blockIdx.x;
  const int pr = vprob[gt];
  const int64_t n = pn[pr], pv = pvec[pr], mo = pmat[pr];
  const int64_t nb = vt_bands(n), ng = vt_groups(n);
  const int64_t item = gt - vitem_off[pr];
  if (item >= nb * ng) return;
  const int64_t t0 = (item % nb) * kVtBand;  // first output row (singular vector index)
  const int64_t g0 = (item / nb) * kVtTilesPerGroup;
  const int64_t ntile = (n + kVtTile - 1) / kVtTile;
  const int64_t gend = min(ntile, g0 + kVtTilesPerGroup);
  const int t = threadIdx.x;
  const int64_t tv = t0 + t;  // this thread's vector (meta) and output row (stores)
  if (tv < n) {
    const int pc = w.col[pv + (n - 1 - tv)];
    pcs[t] = pc;
    lov[t] = w.vlo[pv + pc];
    hiv[t] = w.vhi[pv + pc];
  } else {
    pcs[t] = -1;
    lov[t] = 0;
    hiv[t] = 0;
  }
  __syncthreads();
  const double* Vw = w.Vw + mo;
  double* out = VT + mo;
  const int part = t & 7;
  auto fetch = [&](int64_t g, double (&x)[2 * kPass]) {
    const int64_t ja = g * kVtTile + 2 * part, jb = ja + 1;
#pragma unroll
    for (int p = 0; p < kPass; ++p) {
      const int tt = (t >> 3) + p * (kBlock / 8);
      const int pc = pcs[tt];
      const int lo = lov[tt], hi = hiv[tt];
      double a = 0.0, b = 0.0;
      if (pc >= 0) {
        const double* col = Vw + (int64_t)pc * n;
        if (ja < n && ja >= lo && ja < hi) a = col[ja];
        if (jb < n && jb >= lo && jb < hi) b = col[jb];
      }
      x[2 * p] = a;
      x[2 * p + 1] = b;
    }
  };
  auto put = [&](int64_t g, const double (&x)[2 * kPass]) {
    const int jn = (int)min((int64_t)kVtTile, n - g * kVtTile);
#pragma unroll
    for (int p = 0; p < kPass; ++p) {
      const int tt = (t >> 3) + p * (kBlock / 8);
      tileS[2 * part][tt] = x[2 * p];
      tileS[2 * part + 1][tt] = x[2 * p + 1];
    }
    __syncthreads();
    // output column g kVtTile + jj, rows t0 .. t0 + kVtBand - 1, a row per thread
    if (tv < n)
      for (int jj = 0; jj < jn; ++jj) __builtin_nontemporal_store(tileS[jj][t], out + tv + (g * kVtTile + jj) * n);
    __syncthreads();
  };
  double A[2 * kPass], B[2 * kPass];
  fetch(g0, A);
  for (int64_t g = g0;; g += 2) {
    if (g + 1 < gend) fetch(g + 1, B);
    put(g, A);
    if (g + 1 >= gend) return;
    if (g + 2 < gend) fetch(g + 2, A);
    put(g + 1, B);
    if (g + 2 >= gend) return;
  }
}

// ---- single problem: 4 KB chunks, XCD-aligned
// Per output index tv (descending values): the source column of the tv-th
// largest value with its row supports in U and in V; sigma written here.
__global__ __launch_bounds__(256) void k_final_meta(int64_t n, Work w, double* sigma) {
  const int64_t tv = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (tv >= n) return;
  const int64_t src = n - 1 - tv;
  const int pc = w.col[src];
  w.fin[tv] = make_int4(pc, w.ulo[pc], w.uhi[pc], 0);
  w.fin[n + tv] = make_int4(pc, w.vlo[pc], w.vhi[pc], 0);
  sigma[tv] = w.sig[src];
}

// Chunks of kFinalChunk doubles (4 KB) of the column-major output are written
// by one 16-byte store per thread.  Workgroups are dealt to the 8 XCDs in turn
// (XCD = workgroup index mod 8), and workgroup b writes chunks congruent to b
// mod 8 only, so each XCD streams a fixed eighth of the output's 4 KB pages;
// measured on this part, that is the pattern that reaches the fill rate, where
// longer per-workgroup runs fall 10-15% short.  Both passes store
// non-temporally (the 2 x 8n^2 bytes are written once and never read here):
// the stores then leave the caches to the V^T pass's scattered support
// reads, which otherwise cost it about 100 us of its 480 (measured: 0.79
// against 0.87 ms for the two passes; either pass alone non-temporal gains
// little or loses).  Of the batch's final kernels, whose reads are a quarter
// of their traffic, the V^T one stores non-temporally too (4.75 against 4.89
// ms for the two) and the U one keeps plain stores (5.27 with them).
// One chunk per workgroup: with non-temporal stores, measured 0.735 ms for
// the two passes of n = 16384 against 0.764-0.771 with two chunks, 0.79
// with four and 0.773-0.779 with eight (with plain stores four was best).
constexpr int kFinalR = 1;  // chunks per workgroup

__device__ inline int64_t div_n(int64_t e, int64_t n, double inv_n) {
  int64_t q = (int64_t)((double)e * inv_n);
  if (q * n > e) --q;
  else if ((q + 1) * n <= e) ++q;
  return q;
}

// U: chunks c0 + 8q, c0 = (b / 8) 8 kFinalR + b mod 8
__global__ __launch_bounds__(256) void k_final_u_chunks(int64_t n, Work w, double* U) {
  const int64_t total = n * n;
  const double inv_n = 1.0 / (double)n;
  const int64_t c0 = (int64_t)(blockIdx.x >> 3) * (8 * kFinalR) + (blockIdx.x & 7);
  const double* Uw = w.Uw;
  int64_t e[kFinalR], row[kFinalR];
  int4 mt[kFinalR];
#pragma unroll
  for (int q = 0; q < kFinalR; ++q) {
    e[q] = (c0 + 8 * q) * kFinalChunk + 2 * threadIdx.x;
    mt[q] = make_int4(0, 0, 0, 0);
    row[q] = 0;
    if (e[q] < total) {
      const int64_t col = div_n(e[q], n, inv_n);
      row[q] = e[q] - col * n;
      mt[q] = w.fin[col];
    }
  }
  double2 v[kFinalR];
#pragma unroll
  for (int q = 0; q < kFinalR; ++q) {
    const int64_t r = row[q];
    const int lo = mt[q].y, hi = mt[q].z;
    v[q] = make_double2(0.0, 0.0);
    if (e[q] < total && r + 1 >= lo && r < hi) {
      const double* in = Uw + (int64_t)mt[q].x * n;
      if (r >= lo && r + 1 < hi) {
        v[q] = *reinterpret_cast<const double2*>(in + r);
      } else {
        v[q].x = (r >= lo && r < hi) ? in[r] : 0.0;
        v[q].y = (r + 1 >= lo && r + 1 < hi) ? in[r + 1] : 0.0;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kFinalR; ++q)
    if (e[q] < total) __builtin_nontemporal_store(v2d{v[q].x, v[q].y}, reinterpret_cast<v2d*>(U + e[q]));
}

// V^T (n a multiple of 8 chunks): element e = tv + j n holds V[j, column(tv)]
// inside that column's support.  A workgroup owns 512 vectors tv (one 4 KB
// chunk of every output column) and a contiguous range of groups of kVtJ = 8
// output columns j (one group as launched; the chunk row's residue mod 8 is
// the workgroup's XCD).  Lane L of
// a wavefront stores vectors 2L and 2L+1 of its 128: one 16-byte store per
// output column of the group.  It reads a vector's 64-byte run V[j0 .. j0+7,
// column] when that vector's support meets the group, and a fixed cached run
// otherwise (supports are a few hundred rows of n, so most lanes read the
// cached run); no LDS and no barrier.  The next group's reads are issued
// before the current group's stores.
constexpr int kVtJ = 8;

__global__ __launch_bounds__(256) void k_final_vt_chunks(int64_t n, Work w, double* VT) {
  const double* Vw = w.Vw;
  const int4* fv = w.fin + n;
  const int64_t cpc = n / kFinalChunk;  // chunks per output column
  const int64_t b = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t ch = b % cpc, nblk = gridDim.x / cpc, ngroups = n / kVtJ;
  const int64_t gpb = (ngroups + nblk - 1) / nblk;
  const int64_t g0 = (b / cpc) * gpb, gend = min(ngroups, g0 + gpb);
  if (g0 >= gend) return;
  const int64_t tv = ch * kFinalChunk + wv * 128 + 2 * lane;  // this lane's two vectors
  const int4 s0 = fv[tv], s1 = fv[tv + 1];
  const double* p0 = Vw + (int64_t)s0.x * n;
  const double* p1 = Vw + (int64_t)s1.x * n;
  auto fetch = [&](int64_t g, double2 (&x)[4], double2 (&y)[4]) {
    const int64_t j0 = g * kVtJ;
    // every lane issues the same loads (a lane whose vector's support misses
    // the group reads the cached first run of Vw instead), so the wait for a
    // group's data is a fixed count that leaves the next group's loads and
    // the previous group's stores in flight
    const double* q0 = (s0.y < j0 + kVtJ && s0.z > j0) ? p0 + j0 : Vw;
    const double* q1 = (s1.y < j0 + kVtJ && s1.z > j0) ? p1 + j0 : Vw;
#pragma unroll
    for (int q = 0; q < 4; ++q) x[q] = *reinterpret_cast<const double2*>(q0 + 2 * q);
#pragma unroll
    for (int q = 0; q < 4; ++q) y[q] = *reinterpret_cast<const double2*>(q1 + 2 * q);
  };
  auto put = [&](int64_t g, const double2 (&x)[4], const double2 (&y)[4]) {
    const int64_t j0 = g * kVtJ;
    double* out = VT + tv + j0 * n;
#pragma unroll
    for (int q = 0; q < kVtJ; ++q) {
      const int64_t j = j0 + q;
      const double a = (j >= s0.y && j < s0.z) ? ((q & 1) ? x[q >> 1].y : x[q >> 1].x) : 0.0;
      const double c = (j >= s1.y && j < s1.z) ? ((q & 1) ? y[q >> 1].y : y[q >> 1].x) : 0.0;
      __builtin_nontemporal_store(v2d{a, c}, reinterpret_cast<v2d*>(out + q * n));
    }
  };
  // the fetch after the last group reads a valid group again, unused (no
  // branch around a fetch, so the waits stay fixed counts)
  double2 A0[4], B0[4], A1[4], B1[4];
  fetch(g0, A0, B0);
  for (int64_t g = g0;; g += 2) {
    fetch(g + 1 < gend ? g + 1 : gend - 1, A1, B1);
    put(g, A0, B0);
    if (g + 1 >= gend) return;
    fetch(g + 2 < gend ? g + 2 : gend - 1, A0, B0);
    put(g + 1, A1, B1);
    if (g + 2 >= gend) return;
  }
}

}  // namespace

void launch_rotate(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, hipStream_t st) {
  if (nnodes <= 0) return;
  const int gy = grid_y(nnodes, (max_m + 1 + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL(k_rotate, dim3(nnodes, gy), dim3(kBlock), 0, st, nodes, w);
}

void launch_gather(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, hipStream_t st) {
  if (nnodes <= 0) return;
  // up to 65536 workgroups per level (a batch's top level of a few hundred
  // 2048-value merges: 3.0 ms for its gathers against 3.1-3.4 with 8192)
  const int gy = grid_y(nnodes, (int)std::min<int64_t>(65535, ((int64_t)max_m * (max_m + 1) + kGatherSlab - 1) / kGatherSlab), 65536);
  hipLaunchKernelGGL(k_gather, dim3(nnodes, gy), dim3(kBlock), 0, st, nodes, w);
}

void launch_order(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, hipStream_t st) {
  if (nnodes <= 0) return;
  const int gy = grid_y(nnodes, (max_m + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL(k_order, dim3(nnodes, gy), dim3(kBlock), 0, st, nodes, w);
}

void launch_update(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, const Tuning& tu,
                   hipStream_t st) {
  if (nnodes <= 0) return;
  // every side-half at most 16 B x 16 B (rows <= m + 1 - k, N <= m): one
  // workgroup per node, carrying the k_order work too.  The 64-wide form
  // (two wavefronts per SIMD) wins only on levels of thousands of merges
  // (batches); a single problem's level of a few hundred merges of about 64
  // values runs faster as 64 x 64 tiles (measured 19 vs 27 us).
  if (max_m <= 48 || (max_m <= 64 && nnodes >= 2048)) {
    if (max_m <= 32) hipLaunchKernelGGL((k_update_wave<2>), dim3(nnodes), dim3(kBlock), 0, st, nodes, w);
    else if (max_m <= 48) hipLaunchKernelGGL((k_update_wave<3>), dim3(nnodes), dim3(kBlock), 0, st, nodes, w);
    else hipLaunchKernelGGL((k_update_wave<4>), dim3(nnodes), dim3(kBlock), 0, st, nodes, w);
    return;
  }
  if (tu.flat) {
    launch_order(nodes, nnodes, max_m, w, st);
    hipLaunchKernelGGL(k_tile_sched, dim3(1), dim3(kBlock), 0, st, nodes, nnodes, w);
    hipLaunchKernelGGL((k_update_flat<64, 64>), dim3(tu.grid64), dim3(kBlock), 0, st, nodes, nnodes, w);
    if (max_m > w.small_n)
      hipLaunchKernelGGL((k_update_flat<128, 128>), dim3(tu.grid128), dim3(kBlock), 0, st, nodes, nnodes, w);
    return;
  }
  {
    const int tiles = ((max_m + 1 + 63) / 64) * ((std::min(max_m, w.small_n) + 63) / 64);
    const int gy = grid_y(nnodes, tiles, tu.grid64 * 2);
    hipLaunchKernelGGL((k_update<64, 64>), dim3(nnodes, gy, 5), dim3(kBlock), 0, st, nodes, w);
  }
  if (max_m > w.small_n) {
    const int tiles = ((max_m + 1 + 127) / 128) * ((max_m + 127) / 128);
    const int gy = grid_y(nnodes, tiles, tu.grid128 * 2);
    if (tu.tile128)
      hipLaunchKernelGGL(k_update2, dim3(nnodes, gy, 4), dim3(kBlock), 0, st, nodes, w);
    else
      hipLaunchKernelGGL((k_update<128, 128>), dim3(nnodes, gy, 4), dim3(kBlock), 0, st, nodes, w);
  }
}

void launch_gemm_plain(int M, int N, int K, const double* A, int lda, const double* B, int ldb,
                       double* C, int ldc, int tile128, hipStream_t st) {
  if (M <= 0 || N <= 0) return;
  if (N <= 96) {
    int tiles = ((M + 63) / 64) * ((N + 63) / 64);
    if (tiles > 4096) tiles = 4096;
    hipLaunchKernelGGL((k_gemm_plain<64, 64>), dim3(tiles), dim3(kBlock), 0, st, M, N, K, A, lda, B, ldb, C, ldc);
  } else {
    int tiles = ((M + 127) / 128) * ((N + 127) / 128);
    if (tiles > 4096) tiles = 4096;
    if (tile128)
      hipLaunchKernelGGL(k_gemm_plain2, dim3(tiles), dim3(kBlock), 0, st, M, N, K, A, lda, B, ldb, C, ldc);
    else
      hipLaunchKernelGGL((k_gemm_plain<128, 128>), dim3(tiles), dim3(kBlock), 0, st, M, N, K, A, lda, B, ldb, C,
                         ldc);
  }
}

void launch_final(const int64_t* prob_n, const int64_t* prob_vec, const int64_t* prob_mat,
                  const int64_t* uitem_off, const int64_t* vitem_off, const int32_t* uprob,
                  const int32_t* vprob, int64_t total_uitems, int64_t total_vitems, const Work& w,
                  double* sigma, double* U, double* VT, hipStream_t st) {
  if (total_uitems <= 0) return;
  hipLaunchKernelGGL(k_final_u, dim3((unsigned)total_uitems), dim3(kBlock), 0, st, prob_n, prob_vec, prob_mat,
                     uitem_off, uprob, w, sigma, U);
  hipLaunchKernelGGL(k_final_vt, dim3((unsigned)total_vitems), dim3(kBlock), 0, st, prob_n, prob_vec, prob_mat,
                     vitem_off, vprob, w, VT);
}

void launch_final_single(int64_t n, const Work& w, double* sigma, double* U, double* VT, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_final_meta, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, n, w, sigma);
  const int64_t chunks = (n * n + kFinalChunk - 1) / kFinalChunk;
  const int64_t groups = (chunks + 8 * kFinalR - 1) / (8 * kFinalR);
  hipLaunchKernelGGL(k_final_u_chunks, dim3((unsigned)(groups * 8)), dim3(kBlock), 0, st, n, w, U);
  // V^T: one workgroup per (chunk row, group of kVtJ columns), a multiple of
  // the chunks per output column and so of 8.  With non-temporal stores,
  // short-lived workgroups stream best: 0.677 ms for the two passes of n =
  // 16384 against 0.73-0.74 with persistent grids of 768 to 8192 workgroups
  // walking column ranges (with plain stores three workgroups per CU were).
  const int64_t cpc = n / kFinalChunk;
  const int64_t gv = cpc * (n / kVtJ);
  hipLaunchKernelGGL(k_final_vt_chunks, dim3((unsigned)gv), dim3(kBlock), 0, st, n, w, VT);
}

}  // namespace bdc
