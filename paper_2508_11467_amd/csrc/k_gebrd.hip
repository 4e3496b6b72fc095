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
// columns, and partial sums cross workgroups through per-workgroup slots
// added in a fixed order (deterministic).  Two grid barriers per column:
// the reduction after (a) carries ||x||^2, alpha and P^T x together (P^T v
// is P's pivot row plus the reflector's scale times P^T x), and the one after
// (c) carries the row's ||x||^2, alpha and Q^T x.  Until the scale is known
// the unscaled column (row) stands in P (Q) and every workgroup applies the
// scale as it reads; the owners scale their stored entries once every
// workgroup is past the reads (after the next barrier).  Storage as LAPACK's
// gebrd: d and e on the bidiagonal, v below the diagonal (unit pivot at row
// c), u right of the superdiagonal (unit pivot at column c + 1), tauq, taup.
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
  double q[2 * kBrdMaxB + 2];  // partial sums, then totals, of a reduction
  double qc[2 * kBrdMaxB];     // Q's row c (column c of Q^T)
  double pc[2 * kBrdMaxB];     // P's row c
  double pv[2 * kBrdMaxB + 2];  // P^T v, then Q^T u
  double xa[16];                // x of 16 rows
  double red[4 * 64];
  double sc[8];
  unsigned ok;
  unsigned sh[3];
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
                                                      double* __restrict__ gslots, GridSync* sync, int rows_per_wg,
                                                      int cols_per_wg) {
  __shared__ BrdLds L;
  const int t = threadIdx.x, G = gridDim.x, g = blockIdx.x;
  const int ln = t & 63, wv = t >> 6;
  const int rlo = j0 + g * rows_per_wg, rhi = min(m, rlo + rows_per_wg);
  const int clo = j0 + g * cols_per_wg, chi = min(n, clo + cols_per_wg);
  int phase = 0;
  // L.q[0, cnt) <- its totals over the grid
  auto grid_reduce = [&](int cnt) -> bool {
    double* base = slots + (size_t)phase * G * kSlot;
    double* gbase = gslots + (size_t)phase * grid_group_doubles(kSlot);
    for (int q = t; q < cnt; q += 256) base[(size_t)g * kSlot + q] = L.q[q];
    if (!grid_allreduce(sync, base, gbase, kSlot, cnt, L.q, L.red, L.sh)) return false;
    phase ^= 1;
    return true;
  };
  // the owned columns' entries of the previous row reflector, still unscaled
  auto scale_u = [&](int cp, double sc) {
    const int qp = 2 * (cp - j0) + 1;
    for (int k = max(clo, cp + 2) + t; k < chi; k += 256) {
      Qt[qp + (int64_t)k * ldq] *= sc;
      A[cp + (int64_t)k * lda] *= sc;
    }
  };
  double uscale = 0.0;  // scale of the previous column's row reflector
  bool upend = false;   // its owned entries are still unscaled
  for (int i = 0; i < bw; ++i) {
    const int c = j0 + i, nP = 2 * i;
    // ---- (a) column c from row c down (owned rows): x = A[:, c] - P Q[c, :]^T,
    // stored unscaled in A's column c and P's column nP (1 at the pivot)
    if (t < nP) L.qc[t] = Qt[t + (int64_t)c * ldq];
    __syncthreads();
    // 16 rows at a time.  Thread (rr, cg) holds P[r, q] for q = cg + 16 j
    // (registers): first the 2i products of the row, added over the 16
    // groups in a fixed order, then, once x_r is known, its share of P^T x
    // (rows below the pivot), added over the 16 rows by a butterfly
    const int rr = t & 15, cg = t >> 4;
    double sg = 0.0, al = 0.0;
    double ptx[4] = {0.0, 0.0, 0.0, 0.0};
    for (int r0 = max(rlo, c); r0 < rhi; r0 += 16) {
      const int r = r0 + rr;
      double pr[4], s = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int q = cg + 16 * j;
        pr[j] = (r < rhi && q < nP) ? P[r + (int64_t)q * ldp] : 0.0;
        if (q < nP) s += pr[j] * L.qc[q];
      }
      L.red[cg * 16 + rr] = s;
      __syncthreads();
      if (t < 16) {
        const int rw = r0 + t;
        double xr = 0.0;
        if (rw < rhi) {
          double acc = 0.0;
          for (int p = 0; p < 16; ++p) acc += L.red[p * 16 + t];
          const double a = A[rw + (int64_t)c * lda] - acc;
          A[rw + (int64_t)c * lda] = a;
          if (rw > c) {
            sg += a * a;
            xr = a;
            P[rw + (int64_t)nP * ldp] = a;
          } else {
            al = a;
            P[rw + (int64_t)nP * ldp] = 1.0;
          }
        }
        L.xa[t] = xr;
      }
      __syncthreads();
      const double xr = L.xa[rr];
#pragma unroll
      for (int j = 0; j < 4; ++j) ptx[j] += pr[j] * xr;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double v = ptx[j];
      for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      const int q = cg + 16 * j;
      if (rr == 0 && q < nP) L.q[2 + q] = v;
    }
    sg = wg_sum(sg, L.sc);
    al = wg_sum(al, L.sc);  // alpha from the pivot row's owner, 0 elsewhere
    if (t == 0) {
      L.q[0] = sg;
      L.q[1] = al;
    }
    __syncthreads();
    if (!grid_reduce(2 + nP)) return;  // also publishes x, P's row c and Q's updates
    const Refl h = reflector(L.q[1], L.q[0]);
    if (t < nP) {
      const double pc = P[c + (int64_t)t * ldp];
      L.pc[t] = pc;
      L.pv[t] = pc + h.scale * L.q[2 + t];  // P^T v
    }
    if (t == 0) {
      if (rlo <= c && c < rhi) A[c + (int64_t)c * lda] = h.beta;
      if (g == 0) {
        tauq[c] = h.tau;
        dv[c] = h.beta;
      }
    }
    if (upend) scale_u(c - 1, uscale);
    upend = false;
    __syncthreads();
    // ---- (b) y = tau (A^T v - Q (P^T v)) on the owned columns k > c, and
    // (c) row c there: x_k = A[c, k] - y_k - P[c, :] Q[k, :]^T, stored
    // unscaled in A's row c and Q's column nP + 1 (1 at the pivot)
    // 16 owned columns at a time: every thread accumulates A^T v over its
    // rows for all 16 (16 loads in flight), added over the waves in a fixed
    // order; then thread (kk, qg) finishes column kk with q = qg + 16 j of
    // Q's row (registers): the products with P^T v and P's row c by a
    // butterfly over the 16 lanes, and its share of Q^T x (q <= nP, Q's
    // column nP being y) for the columns right of the pivot
    const int kk = t >> 4, qg = t & 15;
    double qtx[4] = {0.0, 0.0, 0.0, 0.0};
    double sg2 = 0.0, al2 = 0.0;
    for (int kb = max(clo, c + 1); kb < chi; kb += 16) {
      const int nk = min(16, chi - kb);
      double acc[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[j] = 0.0;
      // unconditional loads (columns past the owned ones clamped to the last
      // and not used), so all 16 are in flight before the first product
      const double* Ab = A + (int64_t)kb * lda;
      int col[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) col[j] = min(j, nk - 1);
      for (int r = c + t; r < m; r += 256) {
        const double v = r == c ? 1.0 : P[r + (int64_t)nP * ldp] * h.scale;
        double av[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) av[j] = Ab[r + (int64_t)col[j] * lda];
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[j] += av[j] * v;
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const double v = wave_sum(acc[j]);
        if (ln == 0) L.red[wv * 16 + j] = v;
      }
      __syncthreads();
      const int k = kb + kk;
      const bool live = kk < nk;  // uniform over each 16-lane group
      double q4[4], d1 = 0.0, d2 = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int q = qg + 16 * j;
        q4[j] = (live && q < nP) ? Qt[q + (int64_t)k * ldq] : 0.0;
        if (q < nP) {
          d1 += q4[j] * L.pv[q];
          d2 += L.pc[q] * q4[j];
        }
      }
      for (int off = 8; off > 0; off >>= 1) {
        d1 += __shfl_xor(d1, off, 64);
        d2 += __shfl_xor(d2, off, 64);
      }
      if (live) {
        const double s = (L.red[kk] + L.red[16 + kk]) + (L.red[32 + kk] + L.red[48 + kk]);
        const double y = h.tau * (s - d1);
        const double a = A[c + (int64_t)k * lda] - y - d2;
        if (qg == 0) {
          Qt[nP + (int64_t)k * ldq] = y;
          A[c + (int64_t)k * lda] = a;
          Qt[nP + 1 + (int64_t)k * ldq] = k == c + 1 ? 1.0 : a;
          if (k == c + 1)
            al2 = a;
          else
            sg2 += a * a;
        }
        if (k > c + 1) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int q = qg + 16 * j;
            qtx[j] += (q == nP ? y : q4[j]) * a;
          }
        }
      }
      __syncthreads();  // L.red
    }
    if (c + 1 >= n) {  // the last column: no row reflector
      // nobody else reads this column's unscaled entries (no columns right
      // of it): scale the owned ones
      for (int r = max(rlo, c + 1) + t; r < rhi; r += 256) {
        P[r + (int64_t)nP * ldp] *= h.scale;
        A[r + (int64_t)c * lda] *= h.scale;
      }
      if (g == 0 && t == 0) taup[c] = 0.0;
      continue;
    }
    // Q^T x: over the 4 columns of a wave (lanes 16 and 32 apart), then
    // over the waves in a fixed order
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double v = qtx[j];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      if (ln < 16) L.red[wv * 64 + qg + 16 * j] = v;
    }
    sg2 = wg_sum(sg2, L.sc);
    al2 = wg_sum(al2, L.sc);
    if (t <= nP) L.q[2 + t] = (L.red[t] + L.red[64 + t]) + (L.red[128 + t] + L.red[192 + t]);
    if (t == 0) {
      L.q[0] = sg2;
      L.q[1] = al2;
    }
    __syncthreads();
    if (!grid_reduce(3 + nP)) return;  // also publishes y and row c
    const Refl gr = reflector(L.q[1], L.q[0]);
    if (t <= nP) L.pv[t] = Qt[t + (int64_t)(c + 1) * ldq] + gr.scale * L.q[2 + t];  // Q^T u
    if (t == 0) {
      if (clo <= c + 1 && c + 1 < chi) A[c + (int64_t)(c + 1) * lda] = gr.beta;
      if (g == 0) {
        taup[c] = gr.tau;
        ev[c] = gr.beta;
      }
    }
    // v: every workgroup has read the unscaled column
    for (int r = max(rlo, c + 1) + t; r < rhi; r += 256) {
      P[r + (int64_t)nP * ldp] *= h.scale;
      A[r + (int64_t)c * lda] *= h.scale;
    }
    __syncthreads();
    // ---- (d) x = pi (A u - P (Q^T u)) on the owned rows r > c: 16 rows at
    // a time, the columns of A and of P split over 16 groups of threads, the
    // 16 partial sums of a row added in a fixed order
    for (int r0 = max(rlo, c + 1); r0 < rhi; r0 += 16) {
      // rows past the owned ones are clamped to the last and not used; the
      // columns go in batches of 16 unconditional loads (past n: clamped)
      const int r = min(r0 + rr, rhi - 1);
      double s = 0.0;
      for (int k0 = c + 1 + cg; k0 < n; k0 += 256) {
        double av[16], uv[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int k = min(k0 + 16 * j, n - 1);
          av[j] = A[r + (int64_t)k * lda];
          uv[j] = Qt[nP + 1 + (int64_t)k * ldq];
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int k = k0 + 16 * j;
          if (k < n) s += av[j] * (k == c + 1 ? 1.0 : uv[j] * gr.scale);
        }
      }
      for (int q = cg; q <= nP; q += 16) s -= P[r + (int64_t)q * ldp] * L.pv[q];
      L.red[cg * 16 + rr] = s;
      __syncthreads();
      if (t < 16 && r0 + t < rhi) {
        double x = 0.0;
        for (int p = 0; p < 16; ++p) x += L.red[p * 16 + t];
        P[r0 + t + (int64_t)(nP + 1) * ldp] = gr.tau * x;
      }
      __syncthreads();
    }
    upend = true;
    uscale = gr.scale;
  }
  // the panel's last row reflector: scale once every workgroup has read it
  if (upend) {
    if (!grid_barrier(sync, G, &L.ok)) return;
    scale_u(j0 + bw - 1, uscale);
  }
}

__global__ __launch_bounds__(256) void k_brd_sync_init(GridSync* s) { grid_sync_clear(s); }

}  // namespace

int gebrd_max_block() { return kBrdMaxB; }

size_t gebrd_work_bytes(int m, int n, int b, int max_wg) {
  return kGridSyncBytes +
         8 * ((size_t)m * 2 * b + (size_t)2 * b * n + 2 * (size_t)max_wg * kSlot + 2 * grid_group_doubles(kSlot));
}

int launch_gebrd(int device, int m, int n, double* A, int lda, double* tauq, double* taup, double* d, double* e,
                 int b, void* work, size_t work_bytes, int max_wg, hipStream_t st) {
  int cus = 0, per = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return BDC_ERR_HIP;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(k_brd_panel), 256, 0) !=
      hipSuccess)
    return BDC_ERR_HIP;
  const int maxg = std::min(std::min(max_wg, kGridMaxWg), std::max(1, cus * std::max(per, 1)));
  if (gebrd_work_bytes(m, n, b, maxg) > work_bytes) return BDC_ERR_TOO_LARGE;
  char* w = reinterpret_cast<char*>(work);
  GridSync* sync = reinterpret_cast<GridSync*>(w);
  double* P = reinterpret_cast<double*>(w + kGridSyncBytes);
  double* Qt = P + (size_t)m * 2 * b;
  double* slots = Qt + (size_t)2 * b * n;
  double* gslots = slots + 2 * (size_t)maxg * kSlot;
  const int ldq = 2 * b;
  hipLaunchKernelGGL(k_brd_sync_init, dim3(1), dim3(256), 0, st, sync);
  for (int j0 = 0; j0 < n; j0 += b) {
    const int bw = std::min(b, n - j0);
    // at least 16 rows per workgroup
    const int G = std::max(1, std::min(maxg, (m - j0 + 15) / 16));
    int rpw = (m - j0 + G - 1) / G, cpw = (n - j0 + G - 1) / G;
    int64_t lda64 = lda, ldp64 = m;
    int ldq_ = ldq;
    void* args[] = {&A, &lda64, &m, &n, &j0, const_cast<int*>(&bw), &P, &ldp64, &Qt, &ldq_, &tauq, &taup, &d, &e,
                    &slots, &gslots, &sync, &rpw, &cpw};
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
