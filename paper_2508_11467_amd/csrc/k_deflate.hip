// z formation, sorting and deflation of a merge (Algorithm 3, the GPU-based
// lasd2; the deflation rules of eq. M-condition and the cases after it).
//
// One 256-thread workgroup per merge node; all nodes of a tree level run in
// one launch.  Unlike the paper, the decisions stay on the GPU: the parallel
// part (z, scaling, merge positions by binary search, small-z tests,
// compaction) runs on all threads, and the inherently sequential scan over
// the remaining candidates (each close-pair test compares with the last kept
// value, which earlier rotations may have changed) runs on one thread from
// LDS-staged chunks.  The rotations found are only recorded here; they are
// applied row-parallel by the next kernel.
//
// Every decision must match an independent implementation bit for bit, so
// this file is compiled with floating-point contraction off, and uses only
// correctly rounded +, -, *, / and sqrt; the merge is scaled by a power of
// two (exact).
#include <float.h>

#include "bdc_internal.h"
#include "block_util.h"

namespace bdc {
namespace {

constexpr double kEps = 0x1p-52;
constexpr int kChunk = 1024;

// number of a[0..n) (ascending) strictly below x
__device__ inline int count_less(const double* a, int n, double x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// number of a[0..n) (ascending) at or below x
__device__ inline int count_leq(const double* a, int n, double x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] <= x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_prep(const NodeDesc* __restrict__ nodes, Work w) {
  __shared__ double shd[8];
  __shared__ int shi[kBlock * 6];
  __shared__ int c_pos[kChunk];
  __shared__ double c_d[kChunk];
  __shared__ double c_z[kChunk];
  __shared__ int c_sup[kChunk];
  __shared__ int sh_cnt[4];

  const NodeDesc nd = nodes[blockIdx.x];
  const int m = nd.m, k = nd.k, s = nd.s, r0 = nd.r0, m2 = nd.m - nd.k;
  const int64_t ld = nd.ld, pv = nd.vec_off, vo = nd.vec_off + nd.r0;
  double* V = w.Vw + nd.mat_off;
  const int t = threadIdx.x;

  // the middle row of the split: alpha in the left child's last column,
  // beta in the right child's first column
  const double alpha = w.d[pv + r0 + k - 1];
  const double beta = w.e[pv + r0 + k - 1];
  if (t == 0 && !(fabs(alpha) <= DBL_MAX && fabs(beta) <= DBL_MAX)) atomicOr(&w.ctl->nonfinite, 1);

  // ---- scale: a power of two bringing every value of the merge below 1
  double vmax = fmax(fabs(alpha), fabs(beta));
  for (int c = t; c < m; c += kBlock)
    if (c != k - 1) vmax = fmax(vmax, fabs(w.sig[vo + c]));
  vmax = block_max(vmax, shd);
  double p = 1.0;
  if (vmax > 0.0 && vmax <= DBL_MAX) {
    int ex;
    frexp(vmax, &ex);
    p = ldexp(1.0, ex);
  }
  const double a_s = alpha / p;
  const double b_s = beta / p;

  // ---- z_1 and the rotation (c0, s0) that combines the children's null
  // vectors: x1 = c0 [q1; 0] + s0 [0; q2] carries z_1, y = -s0 [q1; 0] + c0 [0; q2]
  // is the node's own null vector
  const double lam1 = V[(r0 + k - 1) + (int64_t)(r0 + k - 1) * ld];
  const double phi2 = s ? V[(r0 + k) + (int64_t)(r0 + m) * ld] : 0.0;
  const double a = a_s * lam1;
  const double b = b_s * phi2;
  const double rr = sqrt(a * a + b * b);
  double c0 = 1.0, s0 = 0.0;
  if (rr != 0.0) {
    c0 = a / rr;
    s0 = b / rr;
  }

  // ---- z and d of every node column, and its place in the sorted order:
  // the new d = 0 first, then the two ascending child lists merged (ties
  // take the left child first)
  const double* sig = w.sig + vo;
  double lmax = 0.0;
  for (int c = t; c < m; c += kBlock) {
    double dv, zv;
    int pc, pos, sup;
    if (c < k - 1) {
      pc = w.col[vo + c];
      const double sv = sig[c];
      dv = sv / p;
      const int row = r0 + k - 1;  // last row of the left child's right basis
      const double q = (row >= w.vlo[pv + pc] && row < w.vhi[pv + pc]) ? V[row + (int64_t)pc * ld] : 0.0;
      zv = a_s * q;
      pos = 1 + c + count_less(sig + k, m2, sv);
      sup = 1;
    } else if (c == k - 1) {
      pc = r0 + k - 1;
      dv = 0.0;
      zv = rr;
      pos = 0;
      sup = 0;
    } else {
      pc = w.col[vo + c];
      const double sv = sig[c];
      dv = sv / p;
      const int row = r0 + k;  // first row of the right child's right basis
      const double q = (row >= w.vlo[pv + pc] && row < w.vhi[pv + pc]) ? V[row + (int64_t)pc * ld] : 0.0;
      zv = b_s * q;
      pos = 1 + (c - k) + count_leq(sig, k - 1, sv);
      sup = 3;
    }
    w.ps_d[vo + pos] = dv;
    w.ps_z[vo + pos] = zv;
    w.ps_c[vo + pos] = c;
    w.ps_col[vo + pos] = pc;
    w.ps_sup[vo + pos] = sup;
    w.ps_rot[vo + pos] = 0;
    w.status[vo + pos] = 0;
    lmax = fmax(lmax, fmax(dv, fabs(zv)));
  }
  // tol stands for eps * ||M||: 8 * 2^-52 * max(max d, max |z|)
  const double tol = 8.0 * kEps * block_max(lmax, shd);

  // ---- small z components (independent of each other): z_j -> 0.  The
  // others are compacted, in order, into the candidate list.
  {
    const int per = (m - 1 + kBlock - 1) / kBlock;
    const int b0 = 1 + t * per;
    const int b1 = min(m, b0 + per);
    int cnt[1] = {0}, tot[1];
    for (int pos = b0; pos < b1; ++pos) {
      const double z = w.ps_z[vo + pos];
      if (!(fabs(z) < tol || z == 0.0)) ++cnt[0];
    }
    block_exscan<1>(cnt, tot, shi);
    int ci = cnt[0];
    for (int pos = b0; pos < b1; ++pos) {
      const double z = w.ps_z[vo + pos];
      if (fabs(z) < tol || z == 0.0) {
        w.status[vo + pos] = 1;
        w.ps_z[vo + pos] = 0.0;
      } else {
        w.cand[vo + ci++] = pos;
      }
    }
    if (t == 0) sh_cnt[0] = tot[0];
    __syncthreads();
  }
  const int ncand = sh_cnt[0];

  // ---- the sequential scan (one thread): a value within tol of d_1 = 0 is
  // rotated into z_1 from the right and set to 0; a value within tol of the
  // last kept value is rotated into it from both sides, the earlier position
  // keeping the combined z and taking the later value; otherwise it is kept.
  double z0 = 0.0, dlast = 0.0, zlast = 0.0;
  int last = -1, suplast = 0, rotlast = 0, nrot = 0, nzero = 0, nclose = 0;
  const int64_t rb = 2 * vo;
  if (t == 0) z0 = w.ps_z[vo];
  for (int base = 0; base < ncand; base += kChunk) {
    const int nb = min(kChunk, ncand - base);
    __syncthreads();
    for (int i = t; i < nb; i += kBlock) {
      const int pos = w.cand[vo + base + i];
      c_pos[i] = pos;
      c_d[i] = w.ps_d[vo + pos];
      c_z[i] = w.ps_z[vo + pos];
      c_sup[i] = w.ps_sup[vo + pos];
    }
    __syncthreads();
    if (t == 0) {
      for (int i = 0; i < nb; ++i) {
        const int j = c_pos[i];
        const double dj = c_d[i], zj = c_z[i];
        if (dj < tol || dj == 0.0) {
          const double r = sqrt(z0 * z0 + zj * zj);
          const double c = z0 / r, sn = zj / r;
          w.rot_pos[rb + 2 * nrot] = 0;
          w.rot_pos[rb + 2 * nrot + 1] = j;
          w.rot_col[rb + 2 * nrot] = r0 + k - 1;
          w.rot_col[rb + 2 * nrot + 1] = w.ps_col[vo + j];
          w.rot_cs[rb + 2 * nrot] = c;
          w.rot_cs[rb + 2 * nrot + 1] = sn;
          ++nrot;
          z0 = r;
          w.ps_z[vo + j] = 0.0;
          w.ps_d[vo + j] = 0.0;
          w.status[vo + j] = 2;
          w.ps_rot[vo + j] = kRotV;
          ++nzero;
        } else if (last >= 0 && (dj - dlast < tol || dj == dlast)) {
          const double r = sqrt(zlast * zlast + zj * zj);
          const double c = zlast / r, sn = zj / r;
          w.rot_pos[rb + 2 * nrot] = last;
          w.rot_pos[rb + 2 * nrot + 1] = j;
          w.rot_col[rb + 2 * nrot] = w.ps_col[vo + last];
          w.rot_col[rb + 2 * nrot + 1] = w.ps_col[vo + j];
          w.rot_cs[rb + 2 * nrot] = c;
          w.rot_cs[rb + 2 * nrot + 1] = sn;
          ++nrot;
          zlast = r;
          dlast = dj;
          rotlast = kRotU | kRotV;
          w.ps_z[vo + j] = 0.0;
          w.status[vo + j] = 3;
          w.ps_rot[vo + j] = kRotU | kRotV;
          if (suplast != c_sup[i]) {
            suplast = 2;
            w.ps_sup[vo + j] = 2;
          }
          ++nclose;
        } else {
          if (last >= 0) {
            w.ps_d[vo + last] = dlast;
            w.ps_z[vo + last] = zlast;
            w.ps_sup[vo + last] = suplast;
            w.ps_rot[vo + last] = rotlast;
          }
          last = j;
          dlast = dj;
          zlast = zj;
          suplast = c_sup[i];
          rotlast = 0;
        }
      }
    }
  }
  if (t == 0) {
    if (last >= 0) {
      w.ps_d[vo + last] = dlast;
      w.ps_z[vo + last] = zlast;
      w.ps_sup[vo + last] = suplast;
      w.ps_rot[vo + last] = rotlast;
    }
    if (z0 < tol) z0 = tol;  // small z_1 is raised to tol
    w.ps_z[vo] = z0;
    sh_cnt[1] = nrot;
    sh_cnt[2] = nzero;
    sh_cnt[3] = nclose;
  }
  __syncthreads();

  // ---- kept values (ascending), the update order [left | d=0 | both | right]
  // and the deflated values in ascending order (the zeros of the d~0 case
  // first, then the rest in scan order)
  const int per2 = (m + kBlock - 1) / kBlock;
  const int p0 = t * per2, p1 = min(m, p0 + per2);
  int cv[6] = {0, 0, 0, 0, 0, 0}, tot6[6];
  for (int pos = p0; pos < p1; ++pos) {
    const int stt = w.status[vo + pos];
    if (stt == 0) {
      ++cv[0];
      const int sup = w.ps_sup[vo + pos];
      if (pos > 0) ++cv[sup];  // sup in {1, 2, 3}
    } else if (stt == 2) {
      ++cv[4];
    } else {
      ++cv[5];
    }
  }
  block_exscan<6>(cv, tot6, shi);
  const int N = tot6[0], n1 = tot6[1], n2 = tot6[2], n3 = tot6[3], nz = tot6[4];
  double rho = 0.0;
  for (int pos = p0; pos < p1; ++pos) {
    const int stt = w.status[vo + pos];
    if (stt == 0) {
      const int i = cv[0]++;
      int g;
      if (pos == 0) {
        g = n1;
      } else {
        const int sup = w.ps_sup[vo + pos];
        if (sup == 1) g = cv[1]++;
        else if (sup == 2) g = n1 + 1 + cv[2]++;
        else g = n1 + 1 + n2 + cv[3]++;
      }
      const double zz = w.ps_z[vo + pos];
      w.sd[vo + i] = w.ps_d[vo + pos];
      w.sz[vo + i] = zz;
      w.scol[vo + i] = w.ps_col[vo + pos];
      w.srot[vo + i] = w.ps_rot[vo + pos];
      w.sgrp[vo + i] = g;
      w.gsurv[vo + g] = i;
      rho += zz * zz;
    } else {
      const int q = (stt == 2) ? cv[4]++ : nz + cv[5]++;
      w.dval[vo + q] = w.ps_d[vo + pos];
      w.dcol[vo + q] = w.ps_col[vo + pos];
      w.drot[vo + q] = w.ps_rot[vo + pos];
    }
  }
  rho = block_sum(rho, shd);

  // ---- x1 and y in place: rotate the children's null vectors (V columns
  // r0+k-1 and r0+m) by (c0, s0) over the node's rows
  for (int row = t; row < m + s; row += kBlock) {
    const int64_t gr = r0 + row;
    const double q1 = row < k ? V[gr + (int64_t)(r0 + k - 1) * ld] : 0.0;
    const double q2 = (s && row >= k) ? V[gr + (int64_t)(r0 + m) * ld] : 0.0;
    V[gr + (int64_t)(r0 + k - 1) * ld] = c0 * q1 + s0 * q2;
    if (s) V[gr + (int64_t)(r0 + m) * ld] = -s0 * q1 + c0 * q2;
  }
  if (t == 0) {
    w.vlo[pv + r0 + k - 1] = r0;
    w.vhi[pv + r0 + k - 1] = r0 + m + s;
    if (s) {
      w.vlo[pv + r0 + m] = r0;
      w.vhi[pv + r0 + m] = r0 + m + s;
    }
    NodeState st;
    st.N = N;
    st.n1 = n1;
    st.n2 = n2;
    st.n3 = n3;
    st.nrot = sh_cnt[1];
    st.nzero_d = sh_cnt[2];
    st.nclose = sh_cnt[3];
    st.nsmall_z = m - 1 - ncand;
    st.scale = p;
    st.tol = tol;
    st.c0 = c0;
    st.s0 = s0;
    st.rho = rho;
    w.st[nd.id] = st;
  }
}

}  // namespace

void launch_prep(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, hipStream_t st) {
  (void)max_m;
  if (nnodes <= 0) return;
  hipLaunchKernelGGL(k_prep, dim3(nnodes), dim3(kBlock), 0, st, nodes, w);
}

}  // namespace bdc
