// Reduction of a dense m x n matrix (m >= n) to upper bidiagonal form
// B = Q^T A P by Householder reflectors (Section 4.1), blocked as the
// merged-rank-(2b) gebrd of Algorithm 1: every panel of b columns and rows
// is reduced by the labrd loop, which keeps the trailing matrix at its
// panel-start value and collects P = [v_1, x_1, ..., v_b, x_b] and
// Q = [y_1, u_1, ..., y_b, u_b] so that the reduced matrix is A - P Q^T
// (eq. bidiag-A-trail3); the trailing matrix is then updated by that one
// product.  Inside labrd (eq. bidiag-y-k3, bidiag-x-k3), column c:
//   (a) column c <- column c - P Q[c, :]^T;
//   (b) the reflector of its part from the diagonal down (Section 4.1:
//       beta = -sign(alpha) ||x||, v = x / (alpha - beta) below the pivot,
//       tau = 2 / v^T v), then y = tau (A^T v - Q (P^T v));
//   (c) row c <- row c - P[c, :] Q^T;
//   (d) the reflector of its part right of the diagonal, u, pi, then
//       x = pi (A u - P (Q^T u)),
// where A is the panel-start trailing matrix (its two matrix-vector
// products are the only passes over it).  One cooperative grid runs the
// whole panel: workgroup g owns a slice of the rows and a slice of the
// columns; the phases are separated by grid barriers (five per column), and
// partial sums cross workgroups through per-workgroup slots added in a fixed
// order (deterministic).  Storage as LAPACK's gebrd: d and e on the
// bidiagonal, v below the diagonal (unit pivot at row c), u right of the
// superdiagonal (unit pivot at column c + 1), tauq, taup.
#include <algorithm>

#include "bdc_internal.h"
#include "backtr.h"
#include "block_util.h"
#include "gebrd.h"
#include "grid_sync.h"

namespace bdc {
namespace {

constexpr int kBrdMaxB = 32;              // panel width, at most (2b <= 64 columns of P, Q)
constexpr int kSlot = 2 * kBrdMaxB + 2;   // doubles per workgroup per reduction

struct BrdLds {
  double q[2 * kBrdMaxB + 2];  // small vectors of the current phase
  double red[4 * 64];
  double sc[8];
  unsigned ok;
};

struct Refl {
  double beta, tau, scale;
};

// Householder reflector of (alpha, x) with sigma = ||x||^2 (Section 4.1)
__device__ inline Refl reflector(double alpha, double sigma) {
  Refl r{alpha, 0.0, 0.0};
  if (sigma > 0.0) {
    const double nrm = sqrt(alpha * alpha + sigma);
    r.beta = -copysign(nrm, alpha);
    const double den = alpha - r.beta;
    r.scale = 1.0 / den;
    r.tau = 2.0 / (1.0 + sigma / (den * den));
  }
  return r;
}

// workgroup sum of one value per thread (all threads get it)
__device__ inline double wg_sum(double v, double* sh) { return block_sum(v, sh); }

__global__ __launch_bounds__(256, 1) void k_brd_panel(double* __restrict__ A, int64_t lda, int m, int n, int j0,
                                                      int bw, double* __restrict__ P, int64_t ldp,
                                                      double* __restrict__ Qt, int ldq, double* __restrict__ tauq,
                                                      double* __restrict__ taup, double* __restrict__ dv,
                                                      double* __restrict__ ev, double* __restrict__ slots,
                                                      GridSync* sync, int rows_per_wg, int cols_per_wg) {
  __shared__ BrdLds L;
  const int t = threadIdx.x, G = gridDim.x, g = blockIdx.x;
  const int ln = t & 63, wv = t >> 6;
  const int rlo = j0 + g * rows_per_wg, rhi = min(m, rlo + rows_per_wg);
  const int clo = j0 + g * cols_per_wg, chi = min(n, clo + cols_per_wg);
  int phase = 0;
  auto slot = [&](int q) -> double* { return slots + (size_t)phase * G * kSlot + (size_t)q * kSlot; };
  // reduce `cnt` values (thread t < cnt holds value t) over the grid; every
  // thread t < cnt gets the total of value t
  auto grid_reduce = [&](double* vals_lds, int cnt) -> bool {
    double* mine = slot(g);
    for (int q = t; q < cnt; q += 256) mine[q] = vals_lds[q];
    if (!grid_barrier(sync, G, &L.ok)) return false;
    sum_slots(slots + (size_t)phase * G * kSlot, kSlot, G, cnt, vals_lds, L.red);
    phase ^= 1;
    return true;
  };
  for (int i = 0; i < bw; ++i) {
    const int c = j0 + i, nP = 2 * i;
    // ---- (a) column c over the owned rows from c down, and ||x below c||^2
    if (t < nP) L.q[t] = Qt[t + (int64_t)c * ldq];
    __syncthreads();
    double sg = 0.0;
    for (int r = max(rlo, c) + t; r < rhi; r += 256) {
      double a = A[r + (int64_t)c * lda];
      for (int q = 0; q < nP; ++q) a -= P[r + (int64_t)q * ldp] * L.q[q];
      A[r + (int64_t)c * lda] = a;
      if (r > c) sg += a * a;
    }
    sg = wg_sum(sg, L.sc);
    if (t == 0) L.q[0] = sg;
    __syncthreads();
    if (!grid_reduce(L.q, 1)) return;
    const double sigma = L.q[0];
    const Refl h = reflector(A[c + (int64_t)c * lda], sigma);
    __syncthreads();
    // ---- (b) v below the pivot (owned rows), P's column nP, and P^T v
    for (int r = max(rlo, c) + t; r < rhi; r += 256) {
      if (r == c) {
        P[r + (int64_t)nP * ldp] = 1.0;
      } else {
        const double v = A[r + (int64_t)c * lda] * h.scale;
        A[r + (int64_t)c * lda] = v;
        P[r + (int64_t)nP * ldp] = v;
      }
    }
    __syncthreads();  // v of the owned rows, read below by other threads
    // partial P^T v over the owned rows (column q of P by wavefront q % 4)
    for (int q = wv; q < nP; q += 4) {
      double s = 0.0;
      for (int r = max(rlo, c) + ln; r < rhi; r += 64) {
        const double v = r == c ? 1.0 : A[r + (int64_t)c * lda];
        s += P[r + (int64_t)q * ldp] * v;
      }
      s = wave_sum(s);
      if (ln == 0) L.q[q] = s;
    }
    __syncthreads();
    if (!grid_reduce(L.q, nP)) return;  // also publishes v, P's column nP and A's column c
    if (g == 0 && t == 0) {
      tauq[c] = h.tau;
      dv[c] = h.beta;
    }
    // ---- y = tau (A^T v - Q (P^T v)) over the owned columns k > c, then row
    // c over those columns: a_k = A[c, k] - P[c, :] Q[k, :]^T (with v, y)
    double sg2 = 0.0;
    {
      const double pc_v = 1.0;  // P[c, nP]
      for (int k = max(clo, c + 1) + wv; k < chi; k += 4) {
        double s = 0.0;
        for (int r = c + ln; r < m; r += 64) {
          const double v = r == c ? 1.0 : P[r + (int64_t)nP * ldp];
          s += A[r + (int64_t)k * lda] * v;
        }
        s = wave_sum(s);
        double y = s;
        for (int q = 0; q < nP; ++q) y -= Qt[q + (int64_t)k * ldq] * L.q[q];
        y *= h.tau;
        double a = A[c + (int64_t)k * lda] - pc_v * y;
        for (int q = 0; q < nP; ++q) a -= P[c + (int64_t)q * ldp] * Qt[q + (int64_t)k * ldq];
        if (ln == 0) {
          Qt[nP + (int64_t)k * ldq] = y;
          A[c + (int64_t)k * lda] = a;
        }
        if (k > c + 1) sg2 += (ln == 0) ? a * a : 0.0;
      }
    }
    if (c + 1 >= n) {  // the last column: no row reflector
      // every workgroup has read alpha (before the last reduction); the
      // diagonal entry is written after the barrier
      if (!grid_barrier(sync, G, &L.ok)) return;
      if (g == 0 && t == 0) {
        A[c + (int64_t)c * lda] = h.beta;
        taup[c] = 0.0;
      }
      continue;
    }
    sg2 = wg_sum(sg2, L.sc);
    if (t == 0) L.q[0] = sg2;
    __syncthreads();
    if (!grid_reduce(L.q, 1)) return;  // also publishes y and row c
    const double sigma2 = L.q[0];
    const Refl gr = reflector(A[c + (int64_t)(c + 1) * lda], sigma2);
    __syncthreads();
    // ---- (d) u right of the diagonal (owned columns), Q's column nP + 1,
    // and Q^T u (columns q = 0..nP of Q)
    for (int k = max(clo, c + 1) + t; k < chi; k += 256) {
      if (k == c + 1) {
        Qt[nP + 1 + (int64_t)k * ldq] = 1.0;
      } else {
        const double u = A[c + (int64_t)k * lda] * gr.scale;
        A[c + (int64_t)k * lda] = u;
        Qt[nP + 1 + (int64_t)k * ldq] = u;
      }
    }
    __syncthreads();  // u of the owned columns, read below by other threads
    for (int q = wv; q <= nP; q += 4) {
      double s = 0.0;
      for (int k = max(clo, c + 1) + ln; k < chi; k += 64) {
        const double u = k == c + 1 ? 1.0 : A[c + (int64_t)k * lda];
        s += Qt[q + (int64_t)k * ldq] * u;
      }
      s = wave_sum(s);
      if (ln == 0) L.q[q] = s;
    }
    __syncthreads();
    if (!grid_reduce(L.q, nP + 1)) return;  // also publishes u
    if (g == 0 && t == 0) {
      taup[c] = gr.tau;
      ev[c] = gr.beta;
    }
    // ---- x = pi (A u - P (Q^T u)) over the owned rows r > c
    for (int r0 = max(rlo, c + 1); r0 < rhi; r0 += 64) {
      const int r = r0 + ln;
      double s = 0.0;
      if (r < rhi)
        for (int k = c + 1 + wv; k < n; k += 4) {
          const double u = k == c + 1 ? 1.0 : Qt[nP + 1 + (int64_t)k * ldq];
          s += A[r + (int64_t)k * lda] * u;
        }
      L.red[wv * 64 + ln] = s;
      __syncthreads();
      if (t < 64 && r < rhi) {
        double x = (L.red[t] + L.red[64 + t]) + (L.red[128 + t] + L.red[192 + t]);
        for (int q = 0; q <= nP; ++q) x -= P[r + (int64_t)q * ldp] * L.q[q];
        P[r + (int64_t)(nP + 1) * ldp] = gr.tau * x;
      }
      __syncthreads();
    }
    if (!grid_barrier(sync, G, &L.ok)) return;  // publishes x
    // the diagonal and superdiagonal entries, after every workgroup has read
    // the alphas they held (nothing reads row c again in this panel)
    if (g == 0 && t == 0) {
      A[c + (int64_t)c * lda] = h.beta;
      A[c + (int64_t)(c + 1) * lda] = gr.beta;
    }
  }
}

__global__ void k_brd_sync_init(GridSync* s) {
  if (threadIdx.x == 0) {
    s->count = 0;
    s->gen = 0;
    s->expired = 0;
    s->pad = 0;
  }
}

}  // namespace

int gebrd_max_block() { return kBrdMaxB; }

size_t gebrd_work_bytes(int m, int n, int b, int max_wg) {
  return 256 + 8 * ((size_t)m * 2 * b + (size_t)2 * b * n + 2 * (size_t)max_wg * kSlot);
}

int launch_gebrd(int device, int m, int n, double* A, int lda, double* tauq, double* taup, double* d, double* e,
                 int b, void* work, size_t work_bytes, int max_wg, hipStream_t st) {
  int cus = 0, per = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return BDC_ERR_HIP;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(k_brd_panel), 256, 0) !=
      hipSuccess)
    return BDC_ERR_HIP;
  const int maxg = std::min(max_wg, std::max(1, cus * std::max(per, 1)));
  if (gebrd_work_bytes(m, n, b, maxg) > work_bytes) return BDC_ERR_TOO_LARGE;
  char* w = reinterpret_cast<char*>(work);
  GridSync* sync = reinterpret_cast<GridSync*>(w);
  double* P = reinterpret_cast<double*>(w + 256);
  double* Qt = P + (size_t)m * 2 * b;
  double* slots = Qt + (size_t)2 * b * n;
  const int ldq = 2 * b;
  hipLaunchKernelGGL(k_brd_sync_init, dim3(1), dim3(64), 0, st, sync);
  for (int j0 = 0; j0 < n; j0 += b) {
    const int bw = std::min(b, n - j0);
    // at least 16 rows per workgroup
    const int G = std::max(1, std::min(maxg, (m - j0 + 15) / 16));
    int rpw = (m - j0 + G - 1) / G, cpw = (n - j0 + G - 1) / G;
    int64_t lda64 = lda, ldp64 = m;
    int ldq_ = ldq;
    void* args[] = {&A, &lda64, &m, &n, &j0, const_cast<int*>(&bw), &P, &ldp64, &Qt, &ldq_, &tauq, &taup, &d, &e,
                    &slots, &sync, &rpw, &cpw};
    if (hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_brd_panel), dim3(G), dim3(256), args, 0, st) !=
        hipSuccess)
      return BDC_ERR_HIP;
    // trailing matrix: A <- A - P Q^T over rows and columns past the panel
    const int r0 = j0 + bw;
    if (r0 < n)
      launch_sub_product(m - r0, n - r0, 2 * bw, P + r0, m, Qt + (int64_t)r0 * ldq, ldq,
                         A + r0 + (int64_t)r0 * lda, lda, st);
  }
  return BDC_OK;
}

}  // namespace bdc
