// Householder QR of a tall matrix and the explicit Q (Section 4.3.1-4.3.2,
// the tall-and-skinny path): blocked Householder QR in LAPACK's geqrf storage
// with the panel factored on the GPU and the trailing matrix updated in the
// modified compact WY form (eq. larfb with T^{-1} = Y^T Y of eq.
// larft_update), and Q = prod_k (I - Y_k T_k Y_k^T) I (eq. orgqr-q) with
// T^{-1} recomputed at its own block size.
//
// Panel (b <= 64 columns, rows j0..m-1): one cooperative grid of G
// workgroups.  Every workgroup keeps the panel's top b x b block (the rows of
// its pivots) in LDS and updates it redundantly, and owns a contiguous slice
// of the rows below it, also in LDS.  Column c of the panel:
//   1. the reflector of x (Section 4.1): alpha = the pivot entry, sigma =
//      ||x below the pivot||^2, beta = -sign(alpha) sqrt(alpha^2 + sigma),
//      y = x / (alpha - beta) below the pivot, 1 at it, tau = 2 / y^T y with
//      y^T y = 1 + sigma / (alpha - beta)^2 (tau = 0, the identity, when
//      sigma = 0);
//   2. one grid reduction: w = y^T X for the later columns (per-workgroup
//      partial sums, added by every workgroup in the same order:
//      deterministic), and the owned rows' sums of x^2 and y^2 of the next
//      column, so its sigma after the update x <- x - y tau w follows as
//      sum x^2 - 2 tau w sum x y + (tau w)^2 sum y^2 plus the top block's
//      rows -- recomputed by a second grid reduction when that difference
//      has cancelled by more than 7 bits;
//   3. X -= tau y w^T on the owned rows and the top block.
// One grid all-reduce per column (workgroups meet in groups of 16, each
// group's sum formed once, in workgroup order); every wait is bounded (a
// flag reports an expired wait and the kernel ends), and the launch is
// cooperative, so all workgroups are resident.
#include <algorithm>

#include "bdc_internal.h"
#include "backtr.h"
#include "block_util.h"
#include "qr.h"
#include "grid_sync.h"

namespace bdc {
namespace {

constexpr int kQrMaxB = 64;         // panel width, at most
constexpr int kQrBlock = 1024;      // threads of a panel workgroup (16 wavefronts)
constexpr int kQrWaves = kQrBlock / 64;
constexpr int kQrXCap = 160 * kQrMaxB;  // doubles of the owned rows: 10240 / b rows
struct PanelLds {
  double T[kQrMaxB * kQrMaxB];  // top block, T[i * b + k] = A(j0 + i, j0 + k)
  double X[kQrXCap];            // owned rows, X[r * b + k]
  double w[kQrMaxB];
  double tot[kQrMaxB + 2];
  double red[kQrWaves * (kQrMaxB + 2)];
  double sc[kQrWaves];
  unsigned sh[3];
};

// Sum over the workgroup of the wavefront partials of slot q, in wavefront
// order
__device__ __forceinline__ double red_waves(const double* red, int q) {
  constexpr int S = kQrMaxB + 2;
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < kQrWaves; ++u) s += red[u * S + q];
  return s;
}

// workgroup sum of one value per thread (every thread gets it), wavefronts
// added in order
__device__ inline double qr_block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int wv = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[wv] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < kQrWaves; ++u) s += sh[u];
  return s;
}

// grid: G workgroups (cooperative), kQrBlock threads.  slots: 2 x G x (64 + 2)
// doubles; gslots: 2 x grid_group_doubles(64 + 2).
__global__ __launch_bounds__(kQrBlock, 1) void k_qr_panel(double* __restrict__ A, int64_t lda, int m, int j0, int b,
                                                     int rows_per_wg, double* __restrict__ tau,
                                                     double* __restrict__ slots, double* __restrict__ gslots,
                                                     GridSync* sync) {
  constexpr int S = kQrMaxB + 2;  // slot stride: w partials, then two sums
  __shared__ PanelLds L;
  const int t = threadIdx.x, G = gridDim.x, g = blockIdx.x;
  const int ln = t & 63, wv = t >> 6;
  const int top = min(b, m - j0);                  // rows of the top block
  const int below0 = j0 + top;                     // first row below it
  const int r0 = below0 + g * rows_per_wg;         // owned rows [r0, r1)
  const int r1 = min(m, r0 + rows_per_wg);
  const int R = max(0, r1 - r0);
  double* Ap = A + j0 + (int64_t)j0 * lda;         // panel origin
  for (int e = t; e < top * b; e += kQrBlock) {
    const int i = e % top, k = e / top;
    L.T[i * b + k] = Ap[i + (int64_t)k * lda];
  }
  for (int e = t; e < R * b; e += kQrBlock) {
    const int r = e % R, k = e / R;
    L.X[r * b + k] = A[(r0 + r) + (int64_t)(j0 + k) * lda];
  }
  __syncthreads();
  int phase = 0;  // slot buffer of the next reduction
  // owned-row sum of squares of column c, reduced over the grid (exact)
  auto owned_sq = [&](int c) -> double {
    double* sl = slots + (size_t)phase * G * S;
    double* gsl = gslots + (size_t)phase * grid_group_doubles(S);
    phase ^= 1;
    double s = 0.0;
    for (int r = t; r < R; r += kQrBlock) s += L.X[r * b + c] * L.X[r * b + c];
    s = qr_block_sum(s, L.sc);
    if (t == 0) sl[(size_t)g * S] = s;
    if (!grid_allreduce(sync, sl, gsl, S, 1, L.tot, L.red, L.sh)) return -1.0;
    return L.tot[0];
  };
  // sigma of column 0: everything below its pivot
  double own = owned_sq(0);
  if (own < 0.0) return;
  for (int c = 0; c < b; ++c) {
    if (c >= top) {  // no pivot row left: identities
      if (g == 0 && t == 0) tau[j0 + c] = 0.0;
      continue;
    }
    double tp = 0.0;  // top block rows below the pivot (identical on every workgroup)
    for (int i = c + 1; i < top; ++i) tp += L.T[i * b + c] * L.T[i * b + c];
    const double sigma = own + tp;
    const double alpha = L.T[c * b + c];
    double beta = alpha, tc = 0.0, scale = 0.0;
    if (sigma > 0.0) {
      const double nrm = sqrt(alpha * alpha + sigma);
      beta = -copysign(nrm, alpha);
      const double den = alpha - beta;
      scale = 1.0 / den;
      tc = 2.0 / (1.0 + sigma / (den * den));
    }
    // every wavefront has read the top block's column c (tp) before it is
    // scaled
    __syncthreads();
    // y below the pivot: owned rows and the top block's rows c+1..
    for (int r = t; r < R; r += kQrBlock) L.X[r * b + c] *= scale;
    for (int i = c + 1 + t; i < top; i += kQrBlock) L.T[i * b + c] *= scale;
    __syncthreads();
    const int nk = b - c - 1;  // later columns
    if (nk > 0) {
      // one reduction: w_k = y^T X[:, k] (owned rows) for the later
      // columns, and for the next column sum x^2 and sum y^2 (owned rows),
      // from which its sigma after the update follows
      double* sl = slots + (size_t)phase * G * S;
      double* gsl = gslots + (size_t)phase * grid_group_doubles(S);
      phase ^= 1;
      const int k = c + 1 + ln;
      double s = 0.0, sxx = 0.0, syy = 0.0;
      for (int r = wv; r < R; r += kQrWaves) {
        const double y = L.X[r * b + c];
        if (k < b) s += y * L.X[r * b + k];
        if (ln == 0) {
          const double x = L.X[r * b + c + 1];
          sxx += x * x;
          syy += y * y;
        }
      }
      L.red[wv * S + ln] = s;
      if (ln == 0) {
        L.red[wv * S + kQrMaxB] = sxx;
        L.red[wv * S + kQrMaxB + 1] = syy;
      }
      __syncthreads();
      // slot layout: w partials 0..nk-1, then sum x^2, sum y^2
      if (t < nk) sl[(size_t)g * S + t] = red_waves(L.red, t);
      if (t == 64) sl[(size_t)g * S + nk] = red_waves(L.red, kQrMaxB);
      if (t == 65) sl[(size_t)g * S + nk + 1] = red_waves(L.red, kQrMaxB + 1);
      if (!grid_allreduce(sync, sl, gsl, S, nk + 2, L.tot, L.red, L.sh)) return;
      if (t < nk) {
        const int kk = c + 1 + t;
        const double tot = L.tot[t];
        double tq = L.T[c * b + kk];  // pivot row, y = 1
        for (int i = c + 1; i < top; ++i) tq += L.T[i * b + c] * L.T[i * b + kk];
        L.w[t] = tc * (tot + tq);
      }
      if (t == 0) {
        L.sc[1] = L.tot[0];       // owned rows' y^T x of the next column
        L.sc[2] = L.tot[nk];      // sum x^2
        L.sc[3] = L.tot[nk + 1];  // sum y^2
      }
      __syncthreads();
      // the next column's owned-row sum of squares after x <- x - y a,
      // a = tau w: sxx - 2 a sxy + a^2 syy
      {
        const double a = L.w[0], sxy = L.sc[1], sxx = L.sc[2], syy = L.sc[3];
        const double big = sxx + a * a * syy;
        own = (sxx - 2.0 * a * sxy) + a * a * syy;
        // cancelled by more than 7 bits: recompute after the update (a
        // decision every workgroup takes alike); big = 0 means the owned
        // rows of the next column are zero before and after
        if (big == 0.0) own = 0.0;
        else if (!(own > 0x1p-7 * big)) own = -2.0;
      }
      // X -= y (tau w)^T on the owned rows and the top block's rows c..
      for (int e = t; e < R * nk; e += kQrBlock) {
        const int r = e / nk, kq = e - r * nk;
        L.X[r * b + c + 1 + kq] -= L.X[r * b + c] * L.w[kq];
      }
      for (int e = t; e < (top - c) * nk; e += kQrBlock) {
        const int i = c + e / nk, kq = e % nk;
        const double y = i == c ? 1.0 : L.T[i * b + c];
        L.T[i * b + c + 1 + kq] -= y * L.w[kq];
      }
      __syncthreads();
      if (own == -2.0) {
        own = owned_sq(c + 1);
        if (own < 0.0) return;
      }
    }
    // the pivot entry becomes R's diagonal
    if (t == 0) {
      L.T[c * b + c] = beta;
      if (g == 0) tau[j0 + c] = tc;
    }
    __syncthreads();
  }
  // write back: owned rows, and the top block from workgroup 0
  for (int e = t; e < R * b; e += kQrBlock) {
    const int r = e % R, k = e / R;
    A[(r0 + r) + (int64_t)(j0 + k) * lda] = L.X[r * b + k];
  }
  if (g == 0)
    for (int e = t; e < top * b; e += kQrBlock) {
      const int i = e % top, k = e / top;
      Ap[i + (int64_t)k * lda] = L.T[i * b + k];
    }
}

__global__ __launch_bounds__(256) void k_qr_sync_init(GridSync* s) { grid_sync_clear(s); }

// Q (m x ncols, ldq) = the identity's first ncols columns
__global__ __launch_bounds__(256) void k_qr_eye(double* __restrict__ Q, int64_t ldq, int m, int ncols) {
  const int64_t total = (int64_t)m * ncols;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int c = (int)(e / m), r = (int)(e - (int64_t)c * m);
    Q[r + (int64_t)c * ldq] = r == c ? 1.0 : 0.0;
  }
}

}  // namespace

size_t qr_sync_bytes(int max_wg) {
  return kGridSyncBytes + 2 * ((size_t)max_wg * (kQrMaxB + 2) + grid_group_doubles(kQrMaxB + 2)) * sizeof(double);
}

int qr_max_block() { return kQrMaxB; }

int qr_panel_grid(int device, int rows_below, int b, int* grid, int* rows_per_wg) {
  int cus = 0, per = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return -1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(k_qr_panel), kQrBlock, 0) !=
      hipSuccess)
    return -1;
  const int maxg = std::max(1, std::min(kGridMaxWg, cus * std::max(per, 1)));
  // as few workgroups as the LDS allows: a grid all-reduce costs more with
  // more workgroups, and a workgroup's 16 wavefronts share its rows' work
  const int cap = kQrXCap / std::max(b, 1);
  int G = std::max(1, (rows_below + cap - 1) / cap);
  if (G > maxg) return 1;  // too many rows for the resident grid
  *grid = G;
  *rows_per_wg = std::max((rows_below + G - 1) / G, 0);
  return 0;
}

int launch_geqrf(int device, int m, int n, double* A, int lda, double* tau, int b, void* sync_buf, size_t sync_bytes,
                 void* bt_scratch, hipStream_t st) {
  GridSync* sync = reinterpret_cast<GridSync*>(sync_buf);
  double* slots = reinterpret_cast<double*>(reinterpret_cast<char*>(sync_buf) + kGridSyncBytes);
  hipLaunchKernelGGL(k_qr_sync_init, dim3(1), dim3(256), 0, st, sync);
  for (int j0 = 0; j0 < n; j0 += b) {
    const int bw = std::min(b, n - j0);
    const int top = std::min(bw, m - j0);
    const int rows_below = m - j0 - top;
    int G = 1, R = 0;
    if (qr_panel_grid(device, rows_below, bw, &G, &R) != 0) return BDC_ERR_TOO_LARGE;
    if (qr_sync_bytes(G) > sync_bytes) return BDC_ERR_TOO_LARGE;
    int64_t lda64 = lda;
    double* gslots = slots + 2 * (size_t)G * (kQrMaxB + 2);
    void* args[] = {&A, &lda64, &m, &j0, const_cast<int*>(&bw), &R, &tau, &slots, &gslots, &sync};
    if (hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_qr_panel), dim3(G), dim3(kQrBlock), args, 0, st) !=
        hipSuccess)
      return BDC_ERR_HIP;
    // trailing columns: A_t <- H_{bw-1} ... H_0 A_t = Q_panel^T A_t
    const int nt = n - j0 - bw;
    if (nt > 0)
      launch_backtr(1, m - j0, nt, bw, 0, A + j0 + (int64_t)j0 * lda, 1, lda, tau + j0,
                    A + j0 + (int64_t)(j0 + bw) * lda, lda, bw, bt_scratch, nt, st);
  }
  return BDC_OK;
}

void launch_orgqr(int m, int ncols, int k, const double* A, int lda, const double* tau, double* Q, int ldq, int b,
                  void* bt_scratch, hipStream_t st) {
  const int64_t total = (int64_t)m * ncols;
  hipLaunchKernelGGL(k_qr_eye, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 65536)), dim3(256), 0, st, Q,
                     (int64_t)ldq, m, ncols);
  // blocks from the last to the first; block j acts on rows and columns from
  // its first pivot j b on (the columns before it are still those of the
  // identity, which its reflectors leave unchanged)
  const int nblk = (k + b - 1) / b;
  for (int q = nblk - 1; q >= 0; --q) {
    const int i0 = q * b, bw = std::min(b, k - i0);
    if (i0 >= m || i0 >= ncols) continue;
    launch_backtr(0, m - i0, ncols - i0, bw, 0, A + i0 + (int64_t)i0 * lda, 1, lda, tau + i0,
                  Q + i0 + (int64_t)i0 * ldq, ldq, bw, bt_scratch, ncols - i0, st);
  }
}

}  // namespace bdc
