// Back-transformation of singular vectors (Section 4.3.3): C <- Q C or
// Q^T C for Q = H_0 H_1 ... H_{k-1}, H_i = I - tau_i y_i y_i^T, with the
// reflectors applied a block of b at a time in the modified compact WY form
// of eq. inv_t / larft_update: for a block Y (m' x b, rows from the block's
// first pivot down),
//   T^{-1} = Y^T Y above the diagonal, 1/tau_i on it      (gemm)
//   W      = Y^T C                                        (gemm)
//   Z      = T^{-1} \ W   (Q C)  or  T^{-T} \ W  (Q^T C)  (trsm)
//   C      = C - Y Z                                      (gemm)
// since the block's product is I - Y T Y^T.  Q C takes the blocks from the
// last to the first, Q^T C from the first to the last.  All three products
// run on FP64 matrix cores (v_mfma_f64_16x16x4f64); the products with the
// long m' dimension as their depth (Y^T Y, Y^T C) split it over several
// workgroups whose partial sums are added in a fixed order (deterministic).
#include <algorithm>
#include <mutex>

#include "bdc_internal.h"
#include "backtr.h"
#include "block_util.h"

namespace bdc {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kTK = 16;    // k slab
constexpr int kSK = 17;    // stride of k-contiguous LDS rows (odd: conflict-free reads)

// LDS of a tile: A as [k][m] (stride TM + 16) or, transposed in memory, as
// [m][k] (stride 17); B as [n][k] (stride 17); two buffers each.
template <int TM>
struct BtSmem {
  double A[2][TM * kSK > kTK * (TM + 16) ? TM * kSK : kTK * (TM + 16)];
  double B[2][128 * kSK];
};

// TM x 128 output tile over the depth range [k0, k1): four wavefronts in
// 2 x 2, each (TM/2) x 64 as (TM/32) x 4 blocks of 16 x 16.  A is M x K
// column-major (element (r, k) at A[r + k lda]) or, with TRANSA, stored
// K x M (element (r, k) at A[k + r lda]); B is K x N column-major.
template <bool TRANSA, int TM, class Store>
__device__ void bt_tile(BtSmem<TM>& sm, const double* __restrict__ A, int64_t lda, const double* __restrict__ B,
                        int64_t ldb, int M, int N, int k0, int k1, int tm0, int tn0, Store store) {
  constexpr int FA = TM * kTK / kBlock, FB = 128 * kTK / kBlock;
  constexpr int BA = TM / 32;
  constexpr int SA = TRANSA ? kSK : TM + 16;
  const int t = threadIdx.x, wv = t >> 6, l = t & 63;
  const int wm = wv & 1, wn = wv >> 1;
  const int li = l & 15, lk = l >> 4;
  v4d acc[BA][4];
#pragma unroll
  for (int a = 0; a < BA; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  double ra[FA], rb[FB];
  auto load = [&](int kb) {
#pragma unroll
    for (int q = 0; q < FA; ++q) {
      const int e = t + kBlock * q;
      int r, kk;
      if (TRANSA) {
        kk = e % kTK;
        r = e / kTK;
      } else {
        r = e % TM;
        kk = e / TM;
      }
      const int gr = tm0 + r, gk = kb + kk;
      ra[q] = (gr < M && gk < k1) ? (TRANSA ? A[gk + (int64_t)gr * lda] : A[gr + (int64_t)gk * lda]) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < FB; ++q) {
      const int e = t + kBlock * q;
      const int kk = e % kTK, c = e / kTK;
      const int gk = kb + kk, gc = tn0 + c;
      rb[q] = (gk < k1 && gc < N) ? B[gk + (int64_t)gc * ldb] : 0.0;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int q = 0; q < FA; ++q) {
      const int e = t + kBlock * q;
      if (TRANSA) sm.A[buf][(e / kTK) * kSK + e % kTK] = ra[q];
      else sm.A[buf][(e / TM) * SA + e % TM] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < FB; ++q) {
      const int e = t + kBlock * q;
      sm.B[buf][(e / kTK) * kSK + e % kTK] = rb[q];
    }
  };
  const int nslab = (k1 - k0 + kTK - 1) / kTK;
  __syncthreads();
  load(k0);
  stash(0);
  __syncthreads();
  for (int sl = 0; sl < nslab; ++sl) {
    const int buf = sl & 1;
    if (sl + 1 < nslab) load(k0 + (sl + 1) * kTK);
#pragma unroll
    for (int kk = 0; kk < kTK; kk += 4) {
      double af[BA], bf[4];
#pragma unroll
      for (int a = 0; a < BA; ++a) {
        const int row = wm * (TM / 2) + a * 16 + li;
        af[a] = TRANSA ? sm.A[buf][row * kSK + kk + lk] : sm.A[buf][(kk + lk) * SA + row];
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) bf[b] = sm.B[buf][(wn * 64 + b * 16 + li) * kSK + kk + lk];
#pragma unroll
      for (int a = 0; a < BA; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
    if (sl + 1 < nslab) {
      stash(buf ^ 1);
      __syncthreads();
    }
  }
  // D[i][j] of a 16x16 block sits in lane j + 16 (i % 4), register i / 4
#pragma unroll
  for (int a = 0; a < BA; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = tm0 + wm * (TM / 2) + a * 16 + lk + 4 * r;
        const int col = tn0 + wn * 64 + b * 16 + li;
        if (row < M && col < N) store(row, col, acc[a][b][r]);
      }
}

struct PartStore {
  double* P;
  int64_t ld;
  __device__ void operator()(int r, int c, double v) const { P[r + (int64_t)c * ld] = v; }
};
struct SubStore {
  double* C;
  int64_t ld;
  __device__ void operator()(int r, int c, double v) const { C[r + (int64_t)c * ld] -= v; }
};

// The block's reflectors as a dense m' x bw matrix (column c: zeros above
// its pivot, 1 at it, the stored entries below; an all-zero column when
// tau = 0, the identity).  Rows start at the block's first pivot r0.
__global__ __launch_bounds__(256) void k_bt_pack(const double* __restrict__ Y, int64_t rs, int64_t cs,
                                                 const double* __restrict__ tau, int m, int i0, int bw, int offset,
                                                 double* __restrict__ Yp, int ldp) {
  const int r0 = i0 + offset;
  const int rows = m - r0;
  const int64_t total = (int64_t)rows * bw;
  for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < total; g += (int64_t)gridDim.x * 256) {
    const int c = (int)(g / rows), rr = (int)(g - (int64_t)c * rows);
    const int r = r0 + rr, piv = r0 + c;
    double v = 0.0;
    if (tau[i0 + c] != 0.0) v = r < piv ? 0.0 : (r == piv ? 1.0 : Y[(int64_t)r * rs + (int64_t)(i0 + c) * cs]);
    Yp[rr + (int64_t)c * ldp] = v;
  }
}

// Y^T X in depth slices: grid (column tiles of 128, 1, slices); slice z
// covers rows [z * chunk, (z + 1) * chunk) and writes its partial product
// P + z * pstride (bw x N, ld bw).
__global__ __launch_bounds__(256, 1) void k_bt_ytx(const double* __restrict__ Yp, int ldp, const double* __restrict__ X,
                                                   int64_t ldx, int rows, int bw, int N, int chunk,
                                                   double* __restrict__ P, int64_t pstride) {
  __shared__ BtSmem<64> sm;
  const int k0 = blockIdx.z * chunk, k1 = min(rows, k0 + chunk);
  const int tn0 = blockIdx.x * 128;
  if (k0 >= k1) {
    // an empty slice still defines its partial sums
    for (int e = threadIdx.x; e < bw * 128; e += 256) {
      const int r = e % bw, c = tn0 + e / bw;
      if (c < N) P[blockIdx.z * pstride + r + (int64_t)c * bw] = 0.0;
    }
    return;
  }
  bt_tile<true, 64>(sm, Yp, ldp, X, ldx, bw, N, k0, k1, 0, tn0, PartStore{P + blockIdx.z * pstride, bw});
}

// Sum of the slices in order; with tfix, the result is T^{-1}: strictly
// upper part kept, 1/tau on the diagonal (1 for a tau = 0 identity), zeros
// below.
__global__ __launch_bounds__(256) void k_bt_reduce(const double* __restrict__ P, int64_t pstride, int slices,
                                                   int64_t total, double* __restrict__ out, int bw, int tfix,
                                                   const double* __restrict__ tau) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= total) return;
  double s = 0.0;
  for (int z = 0; z < slices; ++z) s += P[z * pstride + g];
  if (tfix) {
    const int r = (int)(g % bw), c = (int)(g / bw);
    if (r > c) s = 0.0;
    else if (r == c) s = tau[r] != 0.0 ? 1.0 / tau[r] : 1.0;
  }
  out[g] = s;
}

// Z = T^{-1} \ W (upper, back substitution) or T^{-T} \ W (lower, forward
// substitution), in place, one thread per column of W (bw x N, ld bw).
template <bool TRANS>
__global__ __launch_bounds__(256) void k_bt_trsm(const double* __restrict__ Ti, int bw, double* __restrict__ W, int N) {
  __shared__ double sT[kBtMaxBlock * kBtMaxBlock];
  for (int e = threadIdx.x; e < bw * bw; e += 256) sT[e] = Ti[e];
  __syncthreads();
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= N) return;
  double z[kBtMaxBlock];
#pragma unroll
  for (int i = 0; i < kBtMaxBlock; ++i) z[i] = i < bw ? W[i + (int64_t)c * bw] : 0.0;
  if (!TRANS) {
#pragma unroll
    for (int i = kBtMaxBlock - 1; i >= 0; --i) {
      if (i >= bw) continue;
      double s = z[i];
#pragma unroll
      for (int j = i + 1; j < kBtMaxBlock; ++j)
        if (j < bw) s -= sT[i + j * bw] * z[j];
      z[i] = s / sT[i + i * bw];
    }
  } else {
#pragma unroll
    for (int i = 0; i < kBtMaxBlock; ++i) {
      if (i >= bw) continue;
      double s = z[i];
#pragma unroll
      for (int j = 0; j < i; ++j) s -= sT[j + i * bw] * z[j];
      z[i] = s / sT[i + i * bw];
    }
  }
#pragma unroll
  for (int i = 0; i < kBtMaxBlock; ++i)
    if (i < bw) W[i + (int64_t)c * bw] = z[i];
}

// C (rows x N) -= Yp (rows x K) Z (K x N, ld ldz): grid (row tiles, column
// tiles).
__global__ __launch_bounds__(256, 1) void k_bt_update(const double* __restrict__ Yp, int ldp,
                                                      const double* __restrict__ Z, int ldz, int K,
                                                      double* __restrict__ C, int64_t ldc, int rows, int N) {
  __shared__ BtSmem<128> sm;
  bt_tile<false, 128>(sm, Yp, ldp, Z, ldz, rows, N, 0, K, blockIdx.x * 128, blockIdx.y * 128, SubStore{C, ldc});
}

}  // namespace

size_t backtr_bytes(int m, int panel, int block) {
  const size_t slices = kBtSlices;
  const size_t w = (size_t)block * std::max(panel, block);
  return 8 * ((size_t)m * block + (size_t)block * block + w + slices * w) + 4 * 256;
}

void launch_backtr(int trans, int m, int p, int k, int offset, const double* Y, int64_t rs, int64_t cs,
                   const double* tau, double* C, int ldc, int block, void* scratch, int panel, hipStream_t st) {
  if (panel < 1 || panel > p) panel = p;
  double* Yp = (double*)scratch;
  double* Ti = Yp + (size_t)m * block;
  double* W = Ti + (size_t)block * block;
  double* P = W + (size_t)block * std::max(panel, block);
  const int64_t pstride = (int64_t)block * std::max(panel, block);
  const int nblk = (k + block - 1) / block;
  for (int q = 0; q < nblk; ++q) {
    const int j = trans ? q : nblk - 1 - q;
    const int i0 = j * block;
    const int bw = std::min(block, k - i0);
    const int r0 = i0 + offset;
    if (r0 >= m) continue;  // reflectors past the last row: identities
    const int rows = m - r0;
    const int64_t ptot = (int64_t)rows * bw;
    hipLaunchKernelGGL(k_bt_pack, dim3((unsigned)std::min<int64_t>((ptot + 255) / 256, 4096)), dim3(256), 0, st, Y,
                       rs, cs, tau, m, i0, bw, offset, Yp, rows);
    // depth slices: about a thousand workgroups for W = Y^T C over all of
    // C's columns, at least 256 rows each (a function of rows and p only, so
    // every panel width sums in the same order)
    const int ctiles = (p + 127) / 128;
    const int slices = std::max(1, std::min({kBtSlices, (rows + 255) / 256, (1024 + ctiles - 1) / ctiles}));
    const int chunk = ((rows + slices - 1) / slices + kTK - 1) / kTK * kTK;
    // T^{-1} = Y^T Y (upper part), 1/tau on the diagonal
    hipLaunchKernelGGL(k_bt_ytx, dim3((bw + 127) / 128, 1, slices), dim3(256), 0, st, Yp, rows, Yp, (int64_t)rows,
                       rows, bw, bw, chunk, P, pstride);
    hipLaunchKernelGGL(k_bt_reduce, dim3((bw * bw + 255) / 256), dim3(256), 0, st, P, pstride, slices,
                       (int64_t)bw * bw, Ti, bw, 1, tau + i0);
    // the columns of C in panels of at most `panel` (every column is
    // transformed on its own, so the panels give the same results)
    for (int c0 = 0; c0 < p; c0 += panel) {
      const int pw = std::min(panel, p - c0);
      double* Cb = C + r0 + (int64_t)c0 * ldc;
      // W = Y^T C
      hipLaunchKernelGGL(k_bt_ytx, dim3((pw + 127) / 128, 1, slices), dim3(256), 0, st, Yp, rows, Cb, (int64_t)ldc,
                         rows, bw, pw, chunk, P, pstride);
      hipLaunchKernelGGL(k_bt_reduce, dim3((unsigned)(((int64_t)bw * pw + 255) / 256)), dim3(256), 0, st, P,
                         pstride, slices, (int64_t)bw * pw, W, bw, 0, tau);
      // Z = T^{-1} \ W  or  T^{-T} \ W
      if (trans)
        hipLaunchKernelGGL(k_bt_trsm<true>, dim3((pw + 255) / 256), dim3(256), 0, st, Ti, bw, W, pw);
      else
        hipLaunchKernelGGL(k_bt_trsm<false>, dim3((pw + 255) / 256), dim3(256), 0, st, Ti, bw, W, pw);
      // C -= Y Z
      hipLaunchKernelGGL(k_bt_update, dim3((rows + 127) / 128, (pw + 127) / 128), dim3(256), 0, st, Yp, rows, W,
                         bw, bw, Cb, (int64_t)ldc, rows, pw);
    }
  }
}

void launch_sub_product(int rows, int N, int K, const double* Y, int ldy, const double* Z, int ldz, double* C,
                        int ldc, hipStream_t st) {
  if (rows <= 0 || N <= 0 || K <= 0) return;
  hipLaunchKernelGGL(k_bt_update, dim3((rows + 127) / 128, (N + 127) / 128), dim3(256), 0, st, Y, ldy, Z, ldz, K,
                     C, (int64_t)ldc, rows, N);
}

// ---------------------------------------------------------------- fixed scratch
// Device memory of the allocation-free entry point: one array per GPU, held
// until the process ends.  Host code never passes `scratch` itself to a
// kernel (on the host the name stands for a host-side shadow, not a device
// address); it passes the address hipGetSymbolAddress returns for the
// current device.
static __device__ __align__(256) char scratch[kBtFixedScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kBtMaxDevices] = {};
bool g_scratch_done[kBtMaxDevices] = {};
}  // namespace

void* backtr_fixed_scratch(int device) {
  if (device < 0 || device >= kBtMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_done[device]) {
    // once per device, with that device current (the caller's guard)
    void* ptr = nullptr;
    const hipError_t rc = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_ptr[device] = rc == hipSuccess ? ptr : nullptr;
    g_scratch_done[device] = true;
  }
  return g_scratch_ptr[device];
}

}  // namespace bdc
