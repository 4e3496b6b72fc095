// Split-precision (Ozaki-style) form of the vector-update products: FP64
// operands are cut into bfloat16 "digit" slices, the slice products run on the
// bfloat16 matrix cores (v_mfma_f32_16x16x32_bf16) with FP32 accumulation, and
// the partial sums are combined in FP64.  The paper computes these products
// in FP64 (eq. bdc-Mv2Bv-u-vt); this is an optional replacement.
//
// Splitting.  Each row of A (over the product's K range) and each column of B
// gets a power of two 2^E with every |entry| < 2^E; x = entry * 2^-E lies in
// (-1, 1) and is written exactly as x = v_0 + v_1 + ... + v_{S-1} + r with
// v_p = rint(r_p 2^(7+8p)) 2^-(7+8p), r_0 = x, r_{p+1} = r_p - v_p (each
// digit has |digit| <= 128, so v_p is exact in bfloat16, and |r| <= 2^-(8S)).
// The remainder r is dropped.
//
// Products.  C = 2^(E_row + E_col) sum_{p+q <= S-1} A_p B_q: the pairs with
// p + q >= S are dropped (their terms are below (S+1) 2^-8S relative to
// |A_row| |B_col|).  Pair sums go to five FP32 accumulators by weight
// g = min(p+q, 4).  With at most 128-magnitude digits the terms of weight t
// are multiples of 2^-(14+8t) of size at most (t+1) 2^-8t, so groups 0..3 are
// exact in FP32 over 128 values of k (14 + log2(4 * 128) <= 23 bits); group 4
// holds terms below 5 * 2^-32 per k whose FP32 rounding stays below 2^-48
// relative to |A_row| |B_col| per 128 values of k.  Every 128 values of k the
// five accumulators are added into an FP64 one.
//
// Layout.  Slices are bfloat16 planes with K contiguous: A slice p of the
// element (row, k) at A + p * plane + row * P + k, B slice p of (k, col) at
// B + p * plane + col * P + k; K is padded with zeros to a multiple of 32.
#include "bdc_internal.h"
#include "block_util.h"

namespace bdc {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int OTM = 128, OTN = 64, OTK = 32;  // output tile, K slab
constexpr int kFlushSlabs = 4;                   // 128 values of k between FP64 flushes
constexpr int kGroups = 5;                       // FP32 accumulators by digit weight

__device__ inline unsigned short bf16_exact(double v) {
  // v has at most 8 significant bits: the float's top half is exact
  return (unsigned short)(__float_as_uint((float)v) >> 16);
}

__device__ inline int exponent_above(double mx) {
  if (!(mx > 0.0)) return 0;
  int e;
  (void)frexp(mx, &e);  // mx = f 2^e, f in [0.5, 1): every |x| <= mx < 2^e
  return e;
}

// Digits of 8 consecutive values, packed 8 bf16 per slice.
template <int S>
__device__ inline void split8(const double v[8], int E, uint4 out[S]) {
  unsigned short b[S][8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    double r = ldexp(v[j], -E);
#pragma unroll
    for (int p = 0; p < S; ++p) {
      const double sc = ldexp(1.0, 7 + 8 * p);
      const double dg = rint(r * sc);
      const double vp = dg / sc;
      r -= vp;
      b[p][j] = bf16_exact(vp);
    }
  }
#pragma unroll
  for (int p = 0; p < S; ++p) {
    out[p].x = (unsigned)b[p][0] | ((unsigned)b[p][1] << 16);
    out[p].y = (unsigned)b[p][2] | ((unsigned)b[p][3] << 16);
    out[p].z = (unsigned)b[p][4] | ((unsigned)b[p][5] << 16);
    out[p].w = (unsigned)b[p][6] | ((unsigned)b[p][7] << 16);
  }
}

// Row split, one thread per row: element (row, k) = src[row + k * lda],
// k in [0, K); writes Kpad = K rounded up to 32 columns of every slice.
template <int S>
__device__ void split_row(const double* __restrict__ src, int64_t lda, int K, unsigned short* __restrict__ dst,
                          int64_t plane, int* __restrict__ Eout) {
  double mx = 0.0;
  for (int k = 0; k < K; ++k) mx = fmax(mx, fabs(src[(int64_t)k * lda]));
  const int E = exponent_above(mx);
  *Eout = E;
  const int Kpad = (K + OTK - 1) / OTK * OTK;
  for (int k8 = 0; k8 < Kpad; k8 += 8) {
    double v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (k8 + j < K) ? src[(int64_t)(k8 + j) * lda] : 0.0;
    uint4 o[S];
    split8<S>(v, E, o);
#pragma unroll
    for (int p = 0; p < S; ++p) *(uint4*)(dst + p * plane + k8) = o[p];
  }
}

// Column split, one wavefront per column: element k = src[k], k in [0, K).
template <int S>
__device__ void split_col(const double* __restrict__ src, int K, unsigned short* __restrict__ dst, int64_t plane,
                          int* __restrict__ Eout) {
  const int lane = threadIdx.x & 63;
  double mx = 0.0;
  for (int k = lane; k < K; k += 64) mx = fmax(mx, fabs(src[k]));
  mx = wave_maxd(mx);
  const int E = exponent_above(mx);
  if (lane == 0) *Eout = E;
  const int Kpad = (K + OTK - 1) / OTK * OTK;
  for (int k8 = 8 * lane; k8 < Kpad; k8 += 512) {
    double v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (k8 + j < K) ? src[k8 + j] : 0.0;
    uint4 o[S];
    split8<S>(v, E, o);
#pragma unroll
    for (int p = 0; p < S; ++p) *(uint4*)(dst + p * plane + k8) = o[p];
  }
}

template <int S>
struct OzSmem {
  uint4 A[S][OTM * OTK / 8];
  uint4 B[S][OTN * OTK / 8];
};

// One 128 x 64 tile of C = 2^(Ea + Eb) sum A_p B_q: four wavefronts in 2 x 2,
// each 64 x 32 as 4 x 2 blocks of 16 x 16.
template <int S, class Store>
__device__ void oz_tile(OzSmem<S>& sm, const unsigned short* __restrict__ A, int64_t planeA, int64_t PA,
                        const int* __restrict__ Ea, const unsigned short* __restrict__ B, int64_t planeB,
                        int64_t PB, const int* __restrict__ Eb, int M, int N, int K, int tm0, int tn0, Store store) {
  constexpr int BA = 4, BB = 2;  // 16 x 16 blocks per wavefront
  const int t = threadIdx.x, wv = t >> 6, l = t & 63;
  const int wm = wv & 1, wn = wv >> 1;
  const int li = l & 15, kq = l >> 4;
  const int Kpad = (K + OTK - 1) / OTK * OTK;
  f32x4 acc[kGroups][BA][BB];
  double acc64[BA][BB][4];
#pragma unroll
  for (int g = 0; g < kGroups; ++g)
#pragma unroll
    for (int a = 0; a < BA; ++a)
#pragma unroll
      for (int b = 0; b < BB; ++b) acc[g][a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int a = 0; a < BA; ++a)
#pragma unroll
    for (int b = 0; b < BB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[a][b][r] = 0.0;
  int slab = 0;
  for (int k0 = 0; k0 < Kpad; k0 += OTK, ++slab) {
    __syncthreads();
#pragma unroll
    for (int p = 0; p < S; ++p) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int c = t + 256 * h;  // 512 chunks of 8 values per A slice tile
        const int rr = c >> 2, kc = c & 3;
        const int gr = tm0 + rr;
        uint4 va = {0u, 0u, 0u, 0u};
        if (gr < M) va = *(const uint4*)(A + p * planeA + (int64_t)gr * PA + k0 + kc * 8);
        sm.A[p][c] = va;
      }
      {
        const int c = t;  // 256 chunks per B slice tile
        const int cc = c >> 2, kc = c & 3;
        const int gc = tn0 + cc;
        uint4 vb = {0u, 0u, 0u, 0u};
        if (gc < N) vb = *(const uint4*)(B + p * planeB + (int64_t)gc * PB + k0 + kc * 8);
        sm.B[p][c] = vb;
      }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < S; ++p) {
      bf16x8 af[BA];
#pragma unroll
      for (int a = 0; a < BA; ++a)
        af[a] = __builtin_bit_cast(bf16x8, sm.A[p][(wm * 64 + a * 16 + li) * 4 + kq]);
#pragma unroll
      for (int q = 0; q + p < S; ++q) {
        const int g = (p + q) < kGroups - 1 ? (p + q) : kGroups - 1;
#pragma unroll
        for (int b = 0; b < BB; ++b) {
          const bf16x8 bf = __builtin_bit_cast(bf16x8, sm.B[q][(wn * 32 + b * 16 + li) * 4 + kq]);
#pragma unroll
          for (int a = 0; a < BA; ++a)
            acc[g][a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bf, acc[g][a][b], 0, 0, 0);
        }
      }
    }
    if ((slab + 1) % kFlushSlabs == 0 || k0 + OTK >= Kpad) {
#pragma unroll
      for (int a = 0; a < BA; ++a)
#pragma unroll
        for (int b = 0; b < BB; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const double lowp = ((double)acc[4][a][b][r] + (double)acc[3][a][b][r]) + (double)acc[2][a][b][r];
            acc64[a][b][r] += ((double)acc[0][a][b][r] + (double)acc[1][a][b][r]) + lowp;
          }
#pragma unroll
      for (int g = 0; g < kGroups; ++g)
#pragma unroll
        for (int a = 0; a < BA; ++a)
#pragma unroll
          for (int b = 0; b < BB; ++b) acc[g][a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  }
  // block (a, b): lane l, register r holds row 4 (l / 16) + r, column l % 16
#pragma unroll
  for (int a = 0; a < BA; ++a)
#pragma unroll
    for (int b = 0; b < BB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = tm0 + wm * 64 + a * 16 + kq * 4 + r;
        const int col = tn0 + wn * 32 + b * 16 + li;
        if (row < M && col < N) store(row, col, ldexp(acc64[a][b][r], Ea[row] + Eb[col]));
      }
}

struct OzNodeStore {
  double* C;
  const int* scol;
  int64_t ld;
  int rowbase;
  __device__ void operator()(int row, int c, double v) const { C[(rowbase + row) + (int64_t)scol[c] * ld] = v; }
};

struct OzPlainStore {
  double* C;
  int64_t ldc;
  __device__ void operator()(int row, int c, double v) const { C[row + (int64_t)c * ldc] = v; }
};

// Geometry of one half-side of a merge's update (sub: 0 U rows [0,k), 1 U
// rows [k,m), 2 V rows [0,k), 3 V rows [k,m+s)).
struct Half {
  int rows, kb, K, rowoff, isV, bottom;
};
__device__ inline Half half_of(const NodeDesc& nd, const NodeState& st, int sub) {
  Half h;
  h.isV = sub >= 2;
  h.bottom = sub & 1;
  h.rows = h.bottom ? (h.isV ? nd.m + nd.s - nd.k : nd.m - nd.k) : nd.k;
  h.kb = h.bottom ? st.n1 : 0;
  const int ke = h.bottom ? st.N : st.n1 + 1 + st.n2;
  h.K = ke - h.kb;
  h.rowoff = h.bottom ? nd.k : 0;
  return h;
}

// Plane rows of a node start at its first row r0; plane columns (k) at the
// multiple of 8 at or below r0, so every 8-value chunk is 16-byte aligned.
__device__ inline int64_t kcol0(int r0) { return (int64_t)(r0 & ~7); }

// Row splits of the gathered columns: grid (node, row block of 64, sub).
template <int S>
__global__ __launch_bounds__(64) void k_oz_rows(const NodeDesc* __restrict__ nodes, Work w) {
  const NodeDesc nd = nodes[blockIdx.x];
  const NodeState st = w.st[nd.id];
  if (st.N < w.oz.min_n) return;
  const Half h = half_of(nd, st, blockIdx.z);
  const int row = blockIdx.y * 64 + threadIdx.x;
  if (row >= h.rows) return;
  const int64_t ld = nd.ld;
  const double* G = (h.isV ? w.GV : w.GU) + nd.mat_off;
  const double* src = G + (nd.r0 + h.rowoff + row) + (int64_t)(nd.r0 + h.kb) * ld;
  const int side = h.isV;
  const int64_t prow = nd.r0 + h.rowoff + row;
  unsigned short* dst = w.oz.A[side] + prow * w.oz.P + kcol0(nd.r0);
  split_row<S>(src, ld, h.K, dst, w.oz.plane, w.oz.Ea[side] + prow);
}

// Column splits of the merge's singular-vector blocks: grid (node, column
// block of 4, sub); one wavefront per column.
template <int S>
__global__ __launch_bounds__(256) void k_oz_cols(const NodeDesc* __restrict__ nodes, Work w) {
  const NodeDesc nd = nodes[blockIdx.x];
  const NodeState st = w.st[nd.id];
  if (st.N < w.oz.min_n) return;
  const int sub = blockIdx.z;  // 0 U top, 1 U bottom, 2 V top, 3 V bottom
  const Half h = half_of(nd, st, sub);
  const int c = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (c >= st.N) return;
  const int64_t ld = nd.ld;
  const double* Mv = (h.isV ? w.VM : w.UM) + nd.mat_off;
  const double* src = Mv + (nd.r0 + h.kb) + (int64_t)(nd.r0 + c) * ld;
  const int side = h.isV;
  unsigned short* planeB = h.bottom ? w.oz.Bb[side] : w.oz.Bt[side];
  int* E = h.bottom ? w.oz.Ebb[side] : w.oz.Ebt[side];
  const int64_t pcol = nd.r0 + c;
  split_col<S>(src, h.K, planeB + pcol * w.oz.P + kcol0(nd.r0), w.oz.plane, E + pcol);
}

template <int S>
__global__ __launch_bounds__(256) void k_update_oz(const NodeDesc* __restrict__ nodes, Work w) {
  __shared__ OzSmem<S> sm;
  const NodeDesc nd = nodes[blockIdx.x];
  const NodeState st = w.st[nd.id];
  if (st.N < w.oz.min_n) return;
  const Half h = half_of(nd, st, blockIdx.z);
  const int side = h.isV;
  const int64_t vo = nd.vec_off + nd.r0;
  const int64_t k0c = kcol0(nd.r0);
  const unsigned short* A = w.oz.A[side] + (int64_t)(nd.r0 + h.rowoff) * w.oz.P + k0c;
  const int* Ea = w.oz.Ea[side] + nd.r0 + h.rowoff;
  const unsigned short* B = (h.bottom ? w.oz.Bb[side] : w.oz.Bt[side]) + (int64_t)nd.r0 * w.oz.P + k0c;
  const int* Eb = (h.bottom ? w.oz.Ebb[side] : w.oz.Ebt[side]) + nd.r0;
  OzNodeStore store{(h.isV ? w.Vw : w.Uw) + nd.mat_off, w.scol + vo, nd.ld, nd.r0 + h.rowoff};
  const int N = st.N;
  const int tiles_m = (h.rows + OTM - 1) / OTM, tiles_n = (N + OTN - 1) / OTN;
  for (int tile = blockIdx.y; tile < tiles_m * tiles_n; tile += gridDim.y) {
    const int tm = tile % tiles_m, tn = tile / tiles_m;
    oz_tile<S>(sm, A, w.oz.plane, w.oz.P, Ea, B, w.oz.plane, w.oz.P, Eb, h.rows, N, h.K, tm * OTM, tn * OTN, store);
  }
}

// ---- a plain product (for checking the kernels on caller data)
template <int S>
__global__ __launch_bounds__(64) void k_oz_rows_plain(const double* A, int64_t lda, int M, int K,
                                                      unsigned short* dst, int64_t plane, int64_t P, int* E) {
  const int row = blockIdx.x * 64 + threadIdx.x;
  if (row >= M) return;
  split_row<S>(A + row, lda, K, dst + (int64_t)row * P, plane, E + row);
}

template <int S>
__global__ __launch_bounds__(256) void k_oz_cols_plain(const double* B, int64_t ldb, int N, int K,
                                                       unsigned short* dst, int64_t plane, int64_t P, int* E) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= N) return;
  split_col<S>(B + (int64_t)c * ldb, K, dst + (int64_t)c * P, plane, E + c);
}

template <int S>
__global__ __launch_bounds__(256) void k_gemm_oz_plain(const unsigned short* A, int64_t planeA, const int* Ea,
                                                       const unsigned short* B, int64_t planeB, const int* Eb,
                                                       int64_t P, int M, int N, int K, double* C, int64_t ldc) {
  __shared__ OzSmem<S> sm;
  const int tiles_m = (M + OTM - 1) / OTM, tiles_n = (N + OTN - 1) / OTN;
  for (int tile = blockIdx.x; tile < tiles_m * tiles_n; tile += gridDim.x) {
    const int tm = tile % tiles_m, tn = tile / tiles_m;
    oz_tile<S>(sm, A, planeA, P, Ea, B, planeB, P, Eb, M, N, K, tm * OTM, tn * OTN, OzPlainStore{C, ldc});
  }
}

inline int grid_y(int nnodes, int units, int cap_total) {
  int gy = units;
  int cap = cap_total / (nnodes > 0 ? nnodes : 1);
  if (cap < 1) cap = 1;
  if (gy > cap) gy = cap;
  if (gy < 1) gy = 1;
  if (gy > 65535) gy = 65535;
  return gy;
}

template <int S>
void launch_oz_level(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, hipStream_t st) {
  const int rb = (max_m + 1 + 63) / 64;
  hipLaunchKernelGGL(k_oz_rows<S>, dim3(nnodes, rb, 4), dim3(64), 0, st, nodes, w);
  const int cb = (max_m + 3) / 4;
  hipLaunchKernelGGL(k_oz_cols<S>, dim3(nnodes, cb, 4), dim3(256), 0, st, nodes, w);
  const int tiles = ((max_m + 1 + OTM - 1) / OTM) * ((max_m + OTN - 1) / OTN);
  const int gy = grid_y(nnodes, tiles, 1024);
  hipLaunchKernelGGL(k_update_oz<S>, dim3(nnodes, gy, 4), dim3(256), 0, st, nodes, w);
}

template <int S>
void launch_oz_plain(int M, int N, int K, const double* A, int lda, const double* B, int ldb, double* C, int ldc,
                     unsigned short* sa, unsigned short* sb, int* ea, int* eb, int64_t P, hipStream_t st) {
  const int64_t planeA = (int64_t)M * P, planeB = (int64_t)N * P;
  hipLaunchKernelGGL(k_oz_rows_plain<S>, dim3((M + 63) / 64), dim3(64), 0, st, A, (int64_t)lda, M, K, sa, planeA, P,
                     ea);
  hipLaunchKernelGGL(k_oz_cols_plain<S>, dim3((N + 3) / 4), dim3(256), 0, st, B, (int64_t)ldb, N, K, sb, planeB, P,
                     eb);
  int tiles = ((M + OTM - 1) / OTM) * ((N + OTN - 1) / OTN);
  if (tiles > 4096) tiles = 4096;
  hipLaunchKernelGGL(k_gemm_oz_plain<S>, dim3(tiles), dim3(256), 0, st, sa, planeA, ea, sb, planeB, eb, P, M, N, K,
                     C, (int64_t)ldc);
}

}  // namespace

int oz_supported(int slices) { return slices >= 5 && slices <= 7; }

void launch_update_ozaki(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, hipStream_t st) {
  if (nnodes <= 0 || max_m < w.oz.min_n) return;
  switch (w.oz.S) {
    case 5: launch_oz_level<5>(nodes, nnodes, max_m, w, st); break;
    case 6: launch_oz_level<6>(nodes, nnodes, max_m, w, st); break;
    case 7: launch_oz_level<7>(nodes, nnodes, max_m, w, st); break;
    default: break;
  }
}

void launch_gemm_ozaki_plain(int slices, int M, int N, int K, const double* A, int lda, const double* B, int ldb,
                             double* C, int ldc, unsigned short* sa, unsigned short* sb, int* ea, int* eb, int64_t P,
                             hipStream_t st) {
  if (M <= 0 || N <= 0) return;
  switch (slices) {
    case 5: launch_oz_plain<5>(M, N, K, A, lda, B, ldb, C, ldc, sa, sb, ea, eb, P, st); break;
    case 6: launch_oz_plain<6>(M, N, K, A, lda, B, ldb, C, ldc, sa, sb, ea, eb, P, st); break;
    case 7: launch_oz_plain<7>(M, N, K, A, lda, B, ldb, C, ldc, sa, sb, ea, eb, P, st); break;
    default: break;
  }
}

}  // namespace bdc
