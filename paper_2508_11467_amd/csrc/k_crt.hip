// Split-precision FP64 products on the int8 matrix cores through the Chinese
// remainder theorem (the integer-modular emulation of Ozaki, Uchino and
// Imamura, "Ozaki Scheme II", 2025), for the vector-update products of eq.
// bdc-Mv2Bv-u-vt:
//
//   1. every row r of the left operand and every column of the right one is
//      scaled by a power of two 2^E_r so that its largest entry lies below
//      2^beta, and rounded to an integer (A', B');
//   2. for each of L pairwise coprime odd moduli m_l <= 255 the residues
//      A' mod m_l and B' mod m_l are taken in the balanced range
//      [-(m_l-1)/2, (m_l-1)/2] (they fit int8);
//   3. the residue matrices are multiplied on v_mfma_i32_16x16x64_i8 with
//      exact int32 accumulation, and each sum is reduced mod m_l again;
//   4. the integer A'B' is rebuilt from its L residues by Garner's
//      mixed-radix algorithm with balanced digits (every step exact in FP32)
//      and an exact Horner sum of the digits in 128-bit integers, then
//      scaled back by 2^-(E_r + E_c) with a single rounding to FP64.
//
// beta is chosen so that K 2^(2 beta) <= (M - 1)/2, M = prod m_l, hence
// |A'B'| lies inside the balanced range and step 4 recovers it exactly; it is
// capped at 55 so that |A'| <= 2^55 fits the seven bytes step 2 splits it into.  The
// only roundings are those of A and B to integers (at most half a unit of
// 2^-beta times the row's / column's largest entry) and the final conversion
// to FP64.  Residue planes are int8, k contiguous, rows padded to kCrtRowPad
// and k to kCrtKStep with zeros.
#include <algorithm>
#include <cmath>

#include "bdc_internal.h"
#include "crt.h"

namespace bdc {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// ------------------------------------------------------------ moduli tables
// moduli in descending order; Garner constants inv(m_j) mod m_l (balanced)
// and 2^(8b) mod m_l, all computed at compile time
constexpr int kMod[kCrtMaxMod] = {255, 253, 251, 247, 241, 239, 233, 229,
                                  227, 223, 217, 211, 199, 197, 193, 191};

constexpr int mod_pos(long long a, int m) {
  const long long r = a % m;
  return (int)(r < 0 ? r + m : r);
}
constexpr int mod_inv(int a, int m) {
  // extended Euclid on (a mod m, m)
  long long r0 = m, r1 = mod_pos(a, m), t0 = 0, t1 = 1;
  while (r1 != 0) {
    const long long q = r0 / r1;
    const long long r2 = r0 - q * r1, t2 = t0 - q * t1;
    r0 = r1;
    r1 = r2;
    t0 = t1;
    t1 = t2;
  }
  return mod_pos(t0, m);
}
constexpr int balanced(int r, int m) { return r > (m - 1) / 2 ? r - m : r; }

struct CrtTables {
  float inv[kCrtMaxMod][kCrtMaxMod];  // [j][l]: inverse of m_j mod m_l (balanced), j < l
  float pw[8][kCrtMaxMod];            // [b][l]: 2^(8 b) mod m_l
};
constexpr CrtTables make_tables() {
  CrtTables t{};
  for (int j = 0; j < kCrtMaxMod; ++j)
    for (int l = 0; l < kCrtMaxMod; ++l)
      t.inv[j][l] = j < l ? (float)balanced(mod_inv(kMod[j], kMod[l]), kMod[l]) : 0.0f;
  for (int l = 0; l < kCrtMaxMod; ++l) {
    long long p = 1;
    for (int b = 0; b < 8; ++b) {
      t.pw[b][l] = (float)mod_pos(p, kMod[l]);
      p = (p * 256) % kMod[l];
    }
  }
  return t;
}
constexpr CrtTables kTab = make_tables();

// x (an integer-valued float, |x| < 2^24) mod m in the balanced range.  For
// odd m, x/m is never within 1/(2m) of a half-integer, so the rounded
// quotient is exact despite the rounding of x * (1/m), and the remainder
// fma(-q, m, x) is exact.
__device__ __forceinline__ float bal_mod(float x, int l) {
  const float m = (float)kMod[l];
  const float q = rintf(x * (1.0f / m));
  return fmaf(-q, m, x);
}

// ------------------------------------------------------------ 1. max |x| per row
// X(r, k) = X[r * sr + k * sk]; rmax[r] = bits of max_k |X(r, k)| (atomic max
// on the bit pattern of a non-negative double orders like the value, so the
// result does not depend on the order of the workgroups).
__global__ __launch_bounds__(256) void k_crt_rowmax(const double* __restrict__ X, int64_t sr, int64_t sk, int R,
                                                    int K, unsigned long long* __restrict__ rmax) {
  const int t = threadIdx.x;
  const int k0 = blockIdx.y * 256;
  double mx = 0.0;
  int r;
  if (sr == 1) {  // rows contiguous: thread = row, loop over k
    r = blockIdx.x * 256 + t;
    if (r < R)
      for (int k = k0; k < min(K, k0 + 256); ++k) mx = fmax(mx, fabs(X[r + (int64_t)k * sk]));
    if (r < R && mx > 0.0) atomicMax(&rmax[r], (unsigned long long)__double_as_longlong(mx));
  } else {  // k contiguous: a wavefront per row
    const int w = t >> 6, l = t & 63;
    for (int q = 0; q < 64; ++q) {
      r = blockIdx.x * 256 + w * 64 + q;
      if (r >= R) break;
      mx = 0.0;
      for (int k = k0 + l; k < min(K, k0 + 256); k += 64) mx = fmax(mx, fabs(X[(int64_t)r * sr + k]));
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
      if (l == 0 && mx > 0.0) atomicMax(&rmax[r], (unsigned long long)__double_as_longlong(mx));
    }
  }
}

// scale exponent of a row: max * 2^E < 2^beta (0 for an all-zero row)
__device__ __forceinline__ int row_exp(unsigned long long bits, int beta) {
  if (bits == 0ull) return 0;
  return beta - 1 - ilogb(__longlong_as_double((long long)bits));
}

// ------------------------------------------------------------ 2. residues
// 16 consecutive k of one row: rounds the scaled entries to integers, splits
// |A'| into its 7 low bytes, and for every modulus writes the 16 balanced
// residues as one 16-byte store at out + l * plane.  Entries outside
// (r < R, k < K) are zeros.
template <int L>
__device__ __forceinline__ void split16(const double* __restrict__ X, int64_t sr, int64_t sk, int R, int K, int r,
                                        int k0, int E, int8_t* __restrict__ out, int64_t plane) {
  float by[16][7];
  float sg[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int k = k0 + e;
    double x = 0.0;
    if (r < R && k < K) x = X[(int64_t)r * sr + (int64_t)k * sk];
    const double a = rint(ldexp(x, E));
    sg[e] = a < 0.0 ? -1.0f : 1.0f;
    const unsigned long long u = (unsigned long long)fabs(a);
    const unsigned int lo = (unsigned int)u, hi = (unsigned int)(u >> 32);
    by[e][0] = (float)(lo & 255u);
    by[e][1] = (float)((lo >> 8) & 255u);
    by[e][2] = (float)((lo >> 16) & 255u);
    by[e][3] = (float)(lo >> 24);
    by[e][4] = (float)(hi & 255u);
    by[e][5] = (float)((hi >> 8) & 255u);
    by[e][6] = (float)((hi >> 16) & 255u);
  }
#pragma unroll
  for (int l = 0; l < L; ++l) {
    unsigned int wd[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      unsigned int v = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int e = 4 * q + b;
        float s = by[e][0];
#pragma unroll
        for (int j = 1; j < 7; ++j) s = fmaf(by[e][j], kTab.pw[j][l], s);
        const int res = (int)(sg[e] * bal_mod(s, l));
        v |= ((unsigned int)res & 255u) << (8 * b);
      }
      wd[q] = v;
    }
    *reinterpret_cast<uint4*>(out + l * plane + k0) = make_uint4(wd[0], wd[1], wd[2], wd[3]);
  }
}

// Thread mapping of a 64-row x 64-k block: with rows contiguous in memory
// (sr == 1) lanes run over rows, else over the four 16-k groups of a row.
__device__ __forceinline__ void split_lane(int64_t sr, int& r, int& kq) {
  const int t = threadIdx.x;
  if (sr == 1) {
    r = t & 63;
    kq = t >> 6;
  } else {
    r = t >> 2;
    kq = t & 3;
  }
}

template <int L>
__global__ __launch_bounds__(256) void k_crt_split(const double* __restrict__ X, int64_t sr, int64_t sk, int R,
                                                   int K, const unsigned long long* __restrict__ rmax, int beta,
                                                   int8_t* __restrict__ out, int64_t plane, int P, int Rpad,
                                                   int* __restrict__ rexp) {
  int r, kq;
  split_lane(sr, r, kq);
  r += blockIdx.x * 64;
  const int k0 = (blockIdx.y * 4 + kq) * 16;
  if (r >= Rpad || k0 >= P) return;
  const int E = r < R ? row_exp(rmax[r], beta) : 0;
  if (r < R && k0 == 0 && rexp) rexp[r] = E;
  split16<L>(X, sr, sk, R, K, r, k0, E, out + (int64_t)r * P, plane);
}

// ------------------------------------------------------------ 3. residue products
// 256 x 128 output tile per 256-thread workgroup: four wavefronts in 2 x 2,
// each 128 x 64 as 4 x 2 blocks of v_mfma_i32_32x32x32_i8 (the int32 sums
// of a block stay in 16 accumulation registers per lane).  k advances in
// 64-byte stages: the residue tiles of a stage (256 and 128 rows of 64 bytes)
// are copied from global memory straight into LDS by the memory unit
// (global_load_lds_dwordx4: lane i of an instruction lands at the
// instruction's LDS base + 16 i), into a ring of four stage buffers, three
// stages ahead of the one being multiplied; a stage is waited for by the
// vector-memory counter and one barrier.  In LDS the four 16-byte chunks of
// row r are stored in the order c ^ f(r), f(r) = ((r >> 1) ^ (r >> 3)) & 3
// (each lane loads the chunk that belongs at its slot), so the operand reads
// of 8 or 16 consecutive lanes, which read the same chunk of consecutive
// rows, fall on distinct banks.  Each lane feeds the matrix cores the 16
// bytes of chunk 2 kk + (lane >> 5) of row (lane & 31) of its A and B blocks:
// the products sum over all 32 k of a step whichever lanes hold which k, as
// long as A and B agree.  The int32 sums are reduced mod m_l and stored as
// balanced int8, column-major (ldr rows).
constexpr int kTile = 256, kTileN = 128, kKs = 64, kRing = 4;
constexpr int kStageA = kTile * kKs, kStageB = kTileN * kKs;  // bytes

struct CrtSmem {
  int8_t A[kRing][kStageA];
  int8_t B[kRing][kStageB];
};

__device__ __forceinline__ int crt_swz(int r) { return ((r >> 1) ^ (r >> 3)) & 3; }

// s_waitcnt with only the vector-memory count set (gfx9 encoding: vmcnt in
// bits 3:0 and 15:14, expcnt 6:4 and lgkmcnt 11:8 at their maxima)
template <int N>
__device__ __forceinline__ void wait_vm() {
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// One 256 x 128 tile: A rows row0.., B^T rows col0.. (both k contiguous,
// stride P, nk stages; the rows up to 255 (A) and 127 (B) past the tile's
// first ones must be readable), output (i, j) mod m_l at C[j ldr + i] for
// i < M, j < N (tile-relative bounds).
__device__ __forceinline__ void crt_tile(CrtSmem& sm, const int8_t* __restrict__ A, const int8_t* __restrict__ B,
                                         int P, int nk, int M, int N, int l, int8_t* __restrict__ C, int64_t ldr) {
  const int t = threadIdx.x, wv = t >> 6, ln = t & 63;
  const int wm = wv & 1, wn = wv >> 1;
  // slot q * 256 + t of a stage (q = 0..3 for A, 0..1 for B): row slot / 4,
  // position slot % 4, holding chunk position ^ f(row) of that row
  const int8_t* ga[4];
  const int8_t* gb[2];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int slot = q * 256 + t, row = slot >> 2, c = (slot & 3) ^ crt_swz(row);
    ga[q] = A + (int64_t)row * P + 16 * c;
    if (q < 2) gb[q] = B + (int64_t)row * P + 16 * c;
  }
  // the six copies of stage s into ring buffer s % kRing; the LDS base of an
  // instruction is uniform over the wavefront
  auto issue = [&](int s) {
    const int buf = s & (kRing - 1), k0 = s * kKs;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      __builtin_amdgcn_global_load_lds(ga[q] + k0, &sm.A[buf][16 * (q * 256 + wv * 64)], 16, 0, 0);
#pragma unroll
    for (int q = 0; q < 2; ++q)
      __builtin_amdgcn_global_load_lds(gb[q] + k0, &sm.B[buf][16 * (q * 256 + wv * 64)], 16, 0, 0);
  };
  v16i acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0;
  const int lr = ln & 31, lh = ln >> 5;
  // the previous tile's readers are done with every ring buffer
  __syncthreads();
#pragma unroll
  for (int s = 0; s < kRing - 1; ++s)
    if (s < nk) issue(s);
  for (int s = 0; s < nk; ++s) {
    // stage s has landed (the copies of the stages after it may still fly)
    if (s + 2 < nk) wait_vm<12>();
    else if (s + 1 < nk) wait_vm<6>();
    else wait_vm<0>();
    // every wavefront's copies of stage s are in, and every wavefront is done
    // reading the buffer that stage s + 3 reuses (stage s - 1's)
    __builtin_amdgcn_s_barrier();
    if (s + kRing - 1 < nk) issue(s + kRing - 1);
    const int buf = s & (kRing - 1);
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      v4i af[4], bf[2];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int row = wm * 128 + a * 32 + lr;
        af[a] = *reinterpret_cast<const v4i*>(&sm.A[buf][row * kKs + 16 * ((2 * kk + lh) ^ crt_swz(row))]);
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int row = wn * 64 + b * 32 + lr;
        bf[b] = *reinterpret_cast<const v4i*>(&sm.B[buf][row * kKs + 16 * ((2 * kk + lh) ^ crt_swz(row))]);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
  }
  // D[i][j] of a 32 x 32 block: lane j + 32 h, register r holds row
  // 8 (r / 4) + 4 h + r % 4: four consecutive rows per register quad
  const double m = (double)kMod[l], im = 1.0 / m;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int col = wn * 64 + b * 32 + lr;
      if (col >= N) continue;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int row = wm * 128 + a * 32 + 8 * g + 4 * lh;
        unsigned int word = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double x = (double)acc[a][b][4 * g + q];
          const int v = (int)fma(-rint(x * im), m, x);
          word |= ((unsigned int)v & 255u) << (8 * q);
        }
        int8_t* dst = C + (int64_t)col * ldr + row;
        if (row + 3 < M && (reinterpret_cast<uintptr_t>(dst) & 3) == 0) {
          *reinterpret_cast<unsigned int*>(dst) = word;
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (row + q < M) dst[q] = (int8_t)(word >> (8 * q));
        }
      }
    }
}

// Grid: x = output tiles (row tile fastest), z = modulus.  Residues of the
// products, column-major (ldr rows).
template <int L>
__global__ __launch_bounds__(256, 1) void k_crt_gemm(const int8_t* __restrict__ RA, const int8_t* __restrict__ RB,
                                                     int64_t planeA, int64_t planeB, int P, int M, int N,
                                                     int8_t* __restrict__ RC, int64_t planeC, int ldr) {
  __shared__ __attribute__((aligned(16))) CrtSmem sm;
  const int l = blockIdx.z;
  const int tiles_m = (M + kTile - 1) / kTile;
  const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
  const int row0 = tm * kTile, col0 = tn * kTileN;
  crt_tile(sm, RA + l * planeA + (int64_t)row0 * P, RB + l * planeB + (int64_t)col0 * P, P, P / kKs, M - row0,
           N - col0, l, RC + l * planeC + (int64_t)col0 * ldr + row0, ldr);
}

// ------------------------------------------------------------ 4. rebuild
// Garner with balanced digits: v_0 = r_0; t_l <- (t_l - v_j) inv(m_j) mod m_l
// for j < l (every step exact in FP32); then the integer
// x = v_0 + m_0 (v_1 + m_1 (v_2 + ...)) exactly, in 128-bit two's complement
// (|x| <= (M - 1) / 2 < 2^127), and x 2^e rounded once to FP64 (to nearest,
// ties to even): an exact product of integers comes out bit for bit.
__device__ __forceinline__ double round_i128(long long hi, unsigned long long lo, int e) {
  const bool neg = hi < 0;
  unsigned long long uh = (unsigned long long)hi, ul = lo;
  if (neg) {  // magnitude
    ul = ~ul + 1ull;
    uh = ~uh + (ul == 0ull ? 1ull : 0ull);
  }
  if (uh == 0ull && ul == 0ull) return 0.0;
  unsigned long long t;
  bool sticky;
  if (uh != 0ull) {
    const int lz = __clzll((long long)uh);
    t = lz ? (uh << lz) | (ul >> (64 - lz)) : uh;
    sticky = lz ? (ul << lz) != 0ull : ul != 0ull;
    e += 64 - lz;
  } else {
    const int lz = __clzll((long long)ul);
    t = ul << lz;
    sticky = false;
    e -= lz;
  }
  // |x| 2^e = (t + a fraction below its last bit) 2^e; keep the top 53 bits of t
  unsigned long long mant = t >> 11;
  const unsigned int rem = (unsigned int)(t & 0x7FFull);
  if (rem > 0x400u || (rem == 0x400u && (sticky || (mant & 1ull)))) ++mant;
  const double v = ldexp((double)mant, e + 11);
  return neg ? -v : v;
}

template <int L>
__device__ __forceinline__ double garner(const int8_t* __restrict__ rc, int64_t planeC, int e) {
  float tt[L];
#pragma unroll
  for (int l = 0; l < L; ++l) tt[l] = (float)rc[l * planeC];
#pragma unroll
  for (int j = 0; j < L - 1; ++j)
#pragma unroll
    for (int l = j + 1; l < L; ++l) tt[l] = bal_mod((tt[l] - tt[j]) * kTab.inv[j][l], l);
  // Horner: x <- x m_l + v_l on (hi, lo) = hi 2^64 + lo
  long long v = (long long)(int)tt[L - 1];
  long long hi = v < 0 ? -1ll : 0ll;
  unsigned long long lo = (unsigned long long)v;
#pragma unroll
  for (int l = L - 2; l >= 0; --l) {
    const unsigned long long m = (unsigned long long)kMod[l];
    const unsigned long long plo = lo * m;
    hi = hi * (long long)m + (long long)__umul64hi(lo, m);
    v = (long long)(int)tt[l];
    lo = plo + (unsigned long long)v;
    hi += (v < 0 ? -1ll : 0ll) + (lo < plo ? 1ll : 0ll);
  }
  return round_i128(hi, lo, e);
}

// Thread: one output element, scaled by 2^-(E_r + E_c).
template <int L>
__global__ __launch_bounds__(256) void k_crt_combine(const int8_t* __restrict__ RC, int64_t planeC, int ldr, int M,
                                                     int N, const int* __restrict__ ea, const int* __restrict__ eb,
                                                     double* __restrict__ C, int64_t ldc) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= (int64_t)M * N) return;
  const int col = (int)(g / M), row = (int)(g % M);
  C[row + (int64_t)col * ldc] = garner<L>(RC + (int64_t)col * ldr + row, planeC, -(ea[row] + eb[col]));
}

// ------------------------------------------------------------ vector update of a merge level
// Geometry of one half-side of a merge's update (sub: 0 U rows [0,k), 1 U
// rows [k,m), 2 V rows [0,k), 3 V rows [k,m+s)): left operand = gathered
// kept columns [kb, kb+K) of those rows, right operand = rows [kb, kb+K) of
// the N x N vectors of M.
struct CrtHalf {
  int rows, kb, K, rowoff, isV, bottom;
};
__device__ inline CrtHalf crt_half(const NodeDesc& nd, const NodeState& st, int sub) {
  CrtHalf h;
  h.isV = sub >= 2;
  h.bottom = sub & 1;
  h.rows = h.bottom ? (h.isV ? nd.m + nd.s - nd.k : nd.m - nd.k) : nd.k;
  h.kb = h.bottom ? st.n1 : 0;
  const int ke = h.bottom ? st.N : st.n1 + 1 + st.n2;
  h.K = ke - h.kb;
  h.rowoff = h.bottom ? nd.k : 0;
  return h;
}

// Zero the maxima of the merges that take the split products.  Grid (node, 1, sub).
__global__ __launch_bounds__(256) void k_crt_lvl_clear(const NodeDesc* __restrict__ nodes, Work w) {
  const NodeDesc nd = nodes[blockIdx.x];
  const NodeState st = w.st[nd.id];
  if (st.N < w.oz.min_n) return;
  const CrtHalf h = crt_half(nd, st, blockIdx.z);
  unsigned long long* am = w.crt.amax[h.isV] + nd.r0 + h.rowoff;
  for (int i = threadIdx.x; i < h.rows; i += 256) am[i] = 0ull;
  unsigned long long* bm = (h.bottom ? w.crt.bbmax[h.isV] : w.crt.btmax[h.isV]) + nd.r0;
  for (int c = threadIdx.x; c < st.N; c += 256) bm[c] = 0ull;
}

// Largest |entry| per row of the left operands: grid (node, row block of 256
// x k chunk of 256, sub), a thread per row.
__global__ __launch_bounds__(256) void k_crt_lvl_amax(const NodeDesc* __restrict__ nodes, int kchunks, Work w) {
  const NodeDesc nd = nodes[blockIdx.x];
  const NodeState st = w.st[nd.id];
  if (st.N < w.oz.min_n) return;
  const CrtHalf h = crt_half(nd, st, blockIdx.z);
  const int rb = blockIdx.y / kchunks, kc = blockIdx.y % kchunks;
  const int row = rb * 256 + threadIdx.x, k0 = kc * 256;
  if (row >= h.rows || k0 >= h.K) return;
  const int64_t ld = nd.ld;
  const double* G = (h.isV ? w.GV : w.GU) + nd.mat_off + (nd.r0 + h.rowoff + row) + (int64_t)(nd.r0 + h.kb) * ld;
  double mx = 0.0;
  const int ke = min(h.K, k0 + 256);
  for (int k = k0; k < ke; ++k) mx = fmax(mx, fabs(G[(int64_t)k * ld]));
  if (mx > 0.0) atomicMax(&w.crt.amax[h.isV][nd.r0 + h.rowoff + row], (unsigned long long)__double_as_longlong(mx));
}

// Largest |entry| per column of the right operands: grid (node, column block
// of 64 x k chunk of 256, sub); a wavefront per column.
__global__ __launch_bounds__(256) void k_crt_lvl_bmax(const NodeDesc* __restrict__ nodes, int kchunks, Work w) {
  const NodeDesc nd = nodes[blockIdx.x];
  const NodeState st = w.st[nd.id];
  if (st.N < w.oz.min_n) return;
  const CrtHalf h = crt_half(nd, st, blockIdx.z);
  const int cb = blockIdx.y / kchunks, kc = blockIdx.y % kchunks;
  const int k0 = kc * 256;
  if (k0 >= h.K) return;
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  const int64_t ld = nd.ld;
  const double* Mv = (h.isV ? w.VM : w.UM) + nd.mat_off + (nd.r0 + h.kb);
  unsigned long long* bm = (h.bottom ? w.crt.bbmax[h.isV] : w.crt.btmax[h.isV]) + nd.r0;
  const int ke = min(h.K, k0 + 256);
  for (int q = 0; q < 16; ++q) {
    const int c = cb * 64 + wv * 16 + q;
    if (c >= st.N) break;
    double mx = 0.0;
    for (int k = k0 + ln; k < ke; k += 64) mx = fmax(mx, fabs(Mv[k + (int64_t)(nd.r0 + c) * ld]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if (ln == 0 && mx > 0.0) atomicMax(&bm[c], (unsigned long long)__double_as_longlong(mx));
  }
}

// Residues of the left operands: grid (node, row block of 64 x k block of 64, sub).
template <int L>
__global__ __launch_bounds__(256) void k_crt_lvl_splita(const NodeDesc* __restrict__ nodes, int kblocks, int beta,
                                                        Work w) {
  const NodeDesc nd = nodes[blockIdx.x];
  const NodeState st = w.st[nd.id];
  if (st.N < w.oz.min_n) return;
  const CrtHalf h = crt_half(nd, st, blockIdx.z);
  int r, kq;
  split_lane(1, r, kq);
  r += (blockIdx.y / kblocks) * 64;
  const int k0 = ((blockIdx.y % kblocks) * 4 + kq) * 16;
  if (r >= h.rows || k0 >= crt_kpad(h.K)) return;
  const int64_t ld = nd.ld;
  const int prow = nd.r0 + h.rowoff + r;
  const int E = row_exp(w.crt.amax[h.isV][prow], beta);
  if (k0 == 0) w.crt.Ea[h.isV][prow] = E;
  const double* G = (h.isV ? w.GV : w.GU) + nd.mat_off + (nd.r0 + h.rowoff) + (int64_t)(nd.r0 + h.kb) * ld;
  split16<L>(G, 1, ld, h.rows, h.K, r, k0, E, w.crt.A[h.isV] + (int64_t)prow * w.crt.P, w.crt.planeA);
}

// Residues of the right operands (columns of the vectors of M, k contiguous):
// grid (node, column block of 64 x k block of 64, sub).
template <int L>
__global__ __launch_bounds__(256) void k_crt_lvl_splitb(const NodeDesc* __restrict__ nodes, int kblocks, int beta,
                                                        Work w) {
  const NodeDesc nd = nodes[blockIdx.x];
  const NodeState st = w.st[nd.id];
  if (st.N < w.oz.min_n) return;
  const CrtHalf h = crt_half(nd, st, blockIdx.z);
  int c, kq;
  split_lane(2, c, kq);
  c += (blockIdx.y / kblocks) * 64;
  const int k0 = ((blockIdx.y % kblocks) * 4 + kq) * 16;
  if (c >= st.N || k0 >= crt_kpad(h.K)) return;
  const int64_t ld = nd.ld;
  const int pcol = nd.r0 + c;
  const unsigned long long* bm = h.bottom ? w.crt.bbmax[h.isV] : w.crt.btmax[h.isV];
  int* Eb = h.bottom ? w.crt.Ebb[h.isV] : w.crt.Ebt[h.isV];
  const int E = row_exp(bm[pcol], beta);
  if (k0 == 0) Eb[pcol] = E;
  const double* Mv = (h.isV ? w.VM : w.UM) + nd.mat_off + (nd.r0 + h.kb) + (int64_t)nd.r0 * ld;
  int8_t* out = (h.bottom ? w.crt.Bb[h.isV] : w.crt.Bt[h.isV]) + (int64_t)pcol * w.crt.P;
  split16<L>(Mv, ld, 1, st.N, h.K, c, k0, E, out, w.crt.planeB);
}

// Residue products: grid (node, tile slot, sub * L + modulus).
template <int L>
__global__ __launch_bounds__(256, 1) void k_crt_lvl_gemm(const NodeDesc* __restrict__ nodes, Work w) {
  __shared__ __attribute__((aligned(16))) CrtSmem sm;
  const NodeDesc nd = nodes[blockIdx.x];
  const NodeState st = w.st[nd.id];
  if (st.N < w.oz.min_n) return;
  const int sub = blockIdx.z / L, l = blockIdx.z % L;
  const CrtHalf h = crt_half(nd, st, sub);
  const int P = w.crt.P;
  const int8_t* A = w.crt.A[h.isV] + l * w.crt.planeA + (int64_t)(nd.r0 + h.rowoff) * P;
  const int8_t* B = (h.bottom ? w.crt.Bb[h.isV] : w.crt.Bt[h.isV]) + l * w.crt.planeB + (int64_t)nd.r0 * P;
  int8_t* C = w.crt.C[h.isV] + l * w.crt.planeC + (int64_t)nd.r0 * w.crt.ldr + nd.r0 + h.rowoff;
  const int nk = crt_kpad(h.K) / kKs;
  const int tiles_m = (h.rows + kTile - 1) / kTile, tiles_n = (st.N + kTileN - 1) / kTileN;
  for (int tile = blockIdx.y; tile < tiles_m * tiles_n; tile += gridDim.y) {
    const int tm = tile % tiles_m, tn = tile / tiles_m;
    const int row0 = tm * kTile, col0 = tn * kTileN;
    crt_tile(sm, A + (int64_t)row0 * P, B + (int64_t)col0 * P, P, nk, h.rows - row0, st.N - col0, l,
             C + (int64_t)col0 * w.crt.ldr + row0, w.crt.ldr);
  }
}

// Rebuild into the kept values' physical columns: grid (node, element block
// of 256, sub); element g = column * rows + row.
template <int L>
__global__ __launch_bounds__(256) void k_crt_lvl_combine(const NodeDesc* __restrict__ nodes, Work w) {
  const NodeDesc nd = nodes[blockIdx.x];
  const NodeState st = w.st[nd.id];
  if (st.N < w.oz.min_n) return;
  const CrtHalf h = crt_half(nd, st, blockIdx.z);
  const int64_t total = (int64_t)h.rows * st.N;
  const int64_t vo = nd.vec_off + nd.r0;
  double* dst = (h.isV ? w.Vw : w.Uw) + nd.mat_off + nd.r0 + h.rowoff;
  const int* Ea = w.crt.Ea[h.isV] + nd.r0 + h.rowoff;
  const int* Eb = (h.bottom ? w.crt.Ebb[h.isV] : w.crt.Ebt[h.isV]) + nd.r0;
  const int8_t* C = w.crt.C[h.isV] + (int64_t)nd.r0 * w.crt.ldr + nd.r0 + h.rowoff;
  for (int64_t g = (int64_t)blockIdx.y * 256 + threadIdx.x; g < total; g += (int64_t)gridDim.y * 256) {
    const int c = (int)(g / h.rows), i = (int)(g - (int64_t)c * h.rows);
    dst[i + (int64_t)w.scol[vo + c] * nd.ld] = garner<L>(C + (int64_t)c * w.crt.ldr + i, w.crt.planeC, -(Ea[i] + Eb[c]));
  }
}

template <int L>
void launch_crt_level(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, hipStream_t st) {
  const int rmax = max_m + 1;                  // rows of the largest half-side, bounded
  const int kmax = max_m;                      // kept values bound the product depth
  const int beta = crt_beta(L, crt_kpad(kmax));
  const int kc256 = (kmax + 255) / 256, kb64 = crt_kpad(kmax) / 64;
  hipLaunchKernelGGL(k_crt_lvl_clear, dim3(nnodes, 1, 4), dim3(256), 0, st, nodes, w);
  hipLaunchKernelGGL(k_crt_lvl_amax, dim3(nnodes, ((rmax + 255) / 256) * kc256, 4), dim3(256), 0, st, nodes, kc256,
                     w);
  hipLaunchKernelGGL(k_crt_lvl_bmax, dim3(nnodes, ((kmax + 63) / 64) * kc256, 4), dim3(256), 0, st, nodes, kc256, w);
  hipLaunchKernelGGL(k_crt_lvl_splita<L>, dim3(nnodes, ((rmax + 63) / 64) * kb64, 4), dim3(256), 0, st, nodes, kb64,
                     beta, w);
  hipLaunchKernelGGL(k_crt_lvl_splitb<L>, dim3(nnodes, ((kmax + 63) / 64) * kb64, 4), dim3(256), 0, st, nodes, kb64,
                     beta, w);
  const int tiles = ((rmax + kTile - 1) / kTile) * ((kmax + kTileN - 1) / kTileN);
  int gy = tiles;
  const int cap = std::max(1, 2048 / std::max(1, nnodes));
  if (gy > cap) gy = cap;
  hipLaunchKernelGGL(k_crt_lvl_gemm<L>, dim3(nnodes, gy, 4 * L), dim3(256), 0, st, nodes, w);
  const int64_t elems = (int64_t)rmax * kmax;
  int ey = (int)std::min<int64_t>((elems + 255) / 256, std::max(1, 8192 / std::max(1, nnodes)));
  hipLaunchKernelGGL(k_crt_lvl_combine<L>, dim3(nnodes, ey, 4), dim3(256), 0, st, nodes, w);
}

template <int L>
void gemm_crt_plain_L(int M, int N, int K, const double* A, int lda, const double* B, int ldb, double* C, int ldc,
                      const CrtBuffers& b, hipStream_t st) {
  const int P = crt_kpad(K);
  const int Mp = crt_rowpad(M), Np = crt_rowpad(N);
  const int beta = crt_beta(L, P);
  (void)hipMemsetAsync(b.amax, 0, sizeof(unsigned long long) * M, st);
  (void)hipMemsetAsync(b.bmax, 0, sizeof(unsigned long long) * N, st);
  // A: rows contiguous (column-major); B^T rows = columns of B, k contiguous
  k_crt_rowmax<<<dim3((M + 255) / 256, (K + 255) / 256), 256, 0, st>>>(A, 1, lda, M, K, b.amax);
  k_crt_rowmax<<<dim3((N + 255) / 256, (K + 255) / 256), 256, 0, st>>>(B, ldb, 1, N, K, b.bmax);
  const int64_t planeA = (int64_t)Mp * P, planeB = (int64_t)Np * P;
  k_crt_split<L><<<dim3(Mp / 64, P / 64), 256, 0, st>>>(A, 1, lda, M, K, b.amax, beta, b.ra, planeA, P, Mp, b.ea);
  k_crt_split<L><<<dim3(Np / 64, P / 64), 256, 0, st>>>(B, ldb, 1, N, K, b.bmax, beta, b.rb, planeB, P, Np, b.eb);
  const int ldr = Mp;
  const int64_t planeC = (int64_t)Mp * N;
  const int tiles = (Mp / kTile) * (Np / kTileN);
  k_crt_gemm<L><<<dim3(tiles, 1, L), 256, 0, st>>>(b.ra, b.rb, planeA, planeB, P, M, N, b.rc, planeC, ldr);
  const int64_t items = (int64_t)M * N;
  k_crt_combine<L><<<dim3((unsigned)((items + 255) / 256)), 256, 0, st>>>(b.rc, planeC, ldr, M, N, b.ea, b.eb, C,
                                                                          ldc);
}

}  // namespace

int crt_beta(int L, int P) {
  double lg = 0.0;
  for (int l = 0; l < L; ++l) lg += std::log2((double)kMod[l]);
  int lk = 0;
  while ((1 << lk) < P) ++lk;
  // K 2^(2 beta) <= (M - 1) / 2 with a little room for the log2 rounding;
  // at most 55, so that |A'| <= 2^55 fits the seven bytes split16 takes
  return std::min(kCrtMaxBeta, (int)std::floor((lg - 1.0 - lk - 1e-9) / 2.0));
}

bool crt_supported(int L) { return L >= kCrtMinMod && L <= kCrtMaxMod; }

size_t crt_plain_bytes(int L, int M, int N, int K, CrtBuffers* b) {
  const int P = crt_kpad(K), Mp = crt_rowpad(M), Np = crt_rowpad(N);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  const size_t ora = take((size_t)L * Mp * P), orb = take((size_t)L * Np * P), orc = take((size_t)L * Mp * N);
  const size_t oam = take(8 * (size_t)std::max(M, 1)), obm = take(8 * (size_t)std::max(N, 1));
  const size_t oea = take(4 * (size_t)std::max(M, 1)), oeb = take(4 * (size_t)std::max(N, 1));
  if (b) {
    char* base = (char*)b->base;
    b->ra = (int8_t*)(base + ora);
    b->rb = (int8_t*)(base + orb);
    b->rc = (int8_t*)(base + orc);
    b->amax = (unsigned long long*)(base + oam);
    b->bmax = (unsigned long long*)(base + obm);
    b->ea = (int*)(base + oea);
    b->eb = (int*)(base + oeb);
  }
  return off;
}

void launch_update_crt(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, hipStream_t st) {
  if (nnodes <= 0 || max_m < w.oz.min_n) return;
  switch (w.crt.L) {
    case 13: launch_crt_level<13>(nodes, nnodes, max_m, w, st); break;
    case 14: launch_crt_level<14>(nodes, nnodes, max_m, w, st); break;
    case 15: launch_crt_level<15>(nodes, nnodes, max_m, w, st); break;
    case 16: launch_crt_level<16>(nodes, nnodes, max_m, w, st); break;
    default: break;
  }
}

void launch_gemm_crt_plain(int L, int M, int N, int K, const double* A, int lda, const double* B, int ldb, double* C,
                           int ldc, const CrtBuffers& b, hipStream_t st) {
  switch (L) {
    case 13: gemm_crt_plain_L<13>(M, N, K, A, lda, B, ldb, C, ldc, b, st); break;
    case 14: gemm_crt_plain_L<14>(M, N, K, A, lda, B, ldb, C, ldc, b, st); break;
    case 15: gemm_crt_plain_L<15>(M, N, K, A, lda, B, ldb, C, ldc, b, st); break;
    case 16: gemm_crt_plain_L<16>(M, N, K, A, lda, B, ldb, C, ldc, b, st); break;
    default: break;
  }
}

}  // namespace bdc
