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

struct MergeHead {
  double p, a_s, b_s, rr, c0, s0;
};

// Scale, z_1 and the rotation (c0, s0) combining the children's null vectors:
// x1 = c0 [q1; 0] + s0 [0; q2] carries z_1 = rr, y = -s0 [q1; 0] + c0 [0; q2]
// is the node's own null vector.  The scale is the power of two above the
// largest of |alpha|, |beta| and the children's largest values (the last of
// each ascending list).
__device__ inline MergeHead merge_head(const NodeDesc& nd, const Work& w) {
  const int k = nd.k, s = nd.s, r0 = nd.r0, m = nd.m;
  const int64_t ld = nd.ld, pv = nd.vec_off, vo = nd.vec_off + nd.r0;
  const double* V = w.Vw + nd.mat_off;
  // the middle row of the split: alpha in the left child's last column,
  // beta in the right child's first column
  const double alpha = w.d[pv + r0 + k - 1];
  const double beta = w.e[pv + r0 + k - 1];
  double vmax = fmax(fmax(fabs(alpha), fabs(beta)), fmax(w.sig[vo + k - 2], w.sig[vo + m - 1]));
  MergeHead h;
  h.p = 1.0;
  if (vmax > 0.0 && vmax <= DBL_MAX) {
    int ex;
    frexp(vmax, &ex);
    h.p = ldexp(1.0, ex);
  }
  h.a_s = alpha / h.p;
  h.b_s = beta / h.p;
  const double lam1 = V[(r0 + k - 1) + (int64_t)(r0 + k - 1) * ld];
  const double phi2 = s ? V[(r0 + k) + (int64_t)(r0 + m) * ld] : 0.0;
  const double a = h.a_s * lam1;
  const double b = h.b_s * phi2;
  h.rr = sqrt(a * a + b * b);
  h.c0 = 1.0;
  h.s0 = 0.0;
  if (h.rr != 0.0) {
    h.c0 = a / h.rr;
    h.s0 = b / h.rr;
  }
  return h;
}

// z and d of every node column and its place in the sorted order: the new
// d = 0 first, then the two ascending child lists merged (ties take the left
// child first).  Many workgroups per node; the largest of d and |z| is
// combined with an atomic max on the bit pattern (non-negative doubles order
// like their bits).
__global__ __launch_bounds__(256) void k_zsort(const NodeDesc* __restrict__ nodes, Work w) {
  __shared__ double shd[8];
  const NodeDesc nd = nodes[blockIdx.x];
  const int m = nd.m, k = nd.k, r0 = nd.r0, m2 = nd.m - nd.k;
  const int64_t ld = nd.ld, pv = nd.vec_off, vo = nd.vec_off + nd.r0;
  const double* V = w.Vw + nd.mat_off;
  if ((int)blockIdx.y * kBlock >= m) return;
  const MergeHead h = merge_head(nd, w);
  if (blockIdx.y == 0 && threadIdx.x == 0 &&
      !(fabs(w.d[pv + r0 + k - 1]) <= DBL_MAX && fabs(w.e[pv + r0 + k - 1]) <= DBL_MAX))
    atomicOr(&w.ctl->nonfinite, 1);
  const double* sig = w.sig + vo;
  double lmax = 0.0;
  for (int c = blockIdx.y * kBlock + threadIdx.x; c < m; c += gridDim.y * kBlock) {
    double dv, zv;
    int pc, pos, sup;
    if (c < k - 1) {
      pc = w.col[vo + c];
      const double sv = sig[c];
      dv = sv / h.p;
      const int row = r0 + k - 1;  // last row of the left child's right basis
      const double q = (row >= w.vlo[pv + pc] && row < w.vhi[pv + pc]) ? V[row + (int64_t)pc * ld] : 0.0;
      zv = h.a_s * q;
      pos = 1 + c + count_less(sig + k, m2, sv);
      sup = 1;
    } else if (c == k - 1) {
      pc = r0 + k - 1;
      dv = 0.0;
      zv = h.rr;
      pos = 0;
      sup = 0;
    } else {
      pc = w.col[vo + c];
      const double sv = sig[c];
      dv = sv / h.p;
      const int row = r0 + k;  // first row of the right child's right basis
      const double q = (row >= w.vlo[pv + pc] && row < w.vhi[pv + pc]) ? V[row + (int64_t)pc * ld] : 0.0;
      zv = h.b_s * q;
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
  lmax = block_max(lmax, shd);
  if (threadIdx.x == 0)
    atomicMax(&w.st[nd.id].zmax_bits, (unsigned long long)__double_as_longlong(lmax));
}

// Deflation of one node (one workgroup).  The scan of the paper's rules over
// positions 2..m is sequential as written, but its decisions are not: after
// a candidate (a position whose z is not small and whose value is not within
// tol of 0) has been processed, the "last kept value" it is compared with is
// always that candidate's own sorted value -- it either became the last kept
// value or was merged into it, which sets the kept value to it.  So each
// close-pair decision is d_j - d_prev < tol with d_prev the previous
// candidate's value, computed in parallel; only the z accumulation along a
// run of close pairs (kept value followed by the values merged into it) and
// the rotations into z_1 stay sequential, one thread per run.
template <int BS>
__global__ __launch_bounds__(BS) void k_prep(const NodeDesc* __restrict__ nodes, Work w) {
  __shared__ double shd[BS / 64];
  __shared__ int shi[BS * 6];
  __shared__ double shl[BS];
  __shared__ int shh[BS];
  __shared__ int sh_cnt[4];

  const NodeDesc nd = nodes[blockIdx.x];
  const int m = nd.m, k = nd.k, s = nd.s, r0 = nd.r0;
  const int64_t ld = nd.ld, pv = nd.vec_off, vo = nd.vec_off + nd.r0;
  double* V = w.Vw + nd.mat_off;
  const int t = threadIdx.x;
  const MergeHead h = merge_head(nd, w);
  const double p = h.p, c0 = h.c0, s0 = h.s0;
  const double zmax = __longlong_as_double((long long)w.st[nd.id].zmax_bits);
  // tol stands for eps * ||M||: 8 * 2^-52 * max(max d, max |z|)
  const double tol = 8.0 * kEps * zmax;
  const int64_t rb = 2 * vo;

  // positions 1..m-1 in contiguous segments, one per thread
  const int per = (m - 1 + BS - 1) / BS;
  const int b0 = min(m, 1 + t * per);
  const int b1 = min(m, b0 + per);

  // pass 1: classes; the last candidate value of each segment
  int cnt[3] = {0, 0, 0}, tot[3];  // near-zero values, candidates, close-pair followers
  double seg_last = 0.0;
  int seg_has = 0;
  for (int pos = b0; pos < b1; ++pos) {
    const double z = w.ps_z[vo + pos], d = w.ps_d[vo + pos];
    if (fabs(z) < tol || z == 0.0) continue;
    if (d < tol || d == 0.0) {
      ++cnt[0];
      continue;
    }
    ++cnt[1];
    seg_last = d;
    seg_has = 1;
  }
  // previous candidate value at each segment start: right-most defined value
  // among earlier segments.  Inside a wavefront a shuffle scan with "later
  // defined wins"; across wavefronts the last defined value of the earlier
  // ones (LDS, one entry per wavefront).
  double dprev = 0.0;
  int has_prev = 0;
  {
    const int lane = t & 63, wv = t >> 6;
    double lv = seg_last;
    int lh = seg_has;
    for (int off = 1; off < 64; off <<= 1) {
      const double ov = __shfl_up(lv, off, 64);
      const int oh = __shfl_up(lh, off, 64);
      if (lane >= off && !lh && oh) {
        lv = ov;
        lh = 1;
      }
    }
    // inclusive value of this lane; the exclusive one is the previous lane's
    double ev = __shfl_up(lv, 1, 64);
    int eh = __shfl_up(lh, 1, 64);
    if (lane == 0) {
      ev = 0.0;
      eh = 0;
    }
    if (lane == 63) {
      shl[wv] = lv;
      shh[wv] = lh;
    }
    __syncthreads();
    if (!eh)
      for (int u = wv - 1; u >= 0; --u)
        if (shh[u]) {
          ev = shl[u];
          eh = 1;
          break;
        }
    dprev = ev;
    has_prev = eh;
  }
  __syncthreads();
  // pass 1b: close-pair followers in the segment
  {
    double dp = dprev;
    int hp = has_prev;
    for (int pos = b0; pos < b1; ++pos) {
      const double z = w.ps_z[vo + pos], d = w.ps_d[vo + pos];
      if (fabs(z) < tol || z == 0.0 || d < tol || d == 0.0) continue;
      if (hp && (d - dp < tol || d == dp)) ++cnt[2];
      dp = d;
      hp = 1;
    }
  }
  block_exscan_w<3, BS>(cnt, tot, shi);
  const int nzero = tot[0], ncand = tot[1], nclose = tot[2];
  // pass 2: statuses, lists, rotation slots of the followers
  {
    int iz = cnt[0], ic = cnt[1], ifl = cnt[2];
    double dp = dprev;
    int hp = has_prev;
    for (int pos = b0; pos < b1; ++pos) {
      const double z = w.ps_z[vo + pos], d = w.ps_d[vo + pos];
      if (fabs(z) < tol || z == 0.0) {
        w.status[vo + pos] = 1;  // small z component: z_j -> 0
        w.ps_z[vo + pos] = 0.0;
        continue;
      }
      if (d < tol || d == 0.0) {
        w.status[vo + pos] = 2;  // within tol of d_1 = 0: rotated into z_1, value 0
        w.cand[vo + iz++] = pos;
        continue;
      }
      const bool close = hp && (d - dp < tol || d == dp);
      w.status[vo + pos] = close ? 3 : 0;
      // rotation slot of a follower, kept in sgrp until the lists are built
      w.sgrp[vo + pos] = close ? nzero + ifl++ : -1;
      w.cand[vo + nzero + ic++] = pos;
      dp = d;
      hp = 1;
    }
  }
  __syncthreads();

  // rotations into z_1 (one thread; all near-zero values precede every
  // candidate in the scan order, so they take rotation slots 0..nzero-1)
  if (t == 0) {
    double z0 = w.ps_z[vo];
    for (int q = 0; q < nzero; ++q) {
      const int j = w.cand[vo + q];
      const double zj = w.ps_z[vo + j];
      const double r = sqrt(z0 * z0 + zj * zj);
      const double c = z0 / r, sn = zj / r;
      w.rot_pos[rb + 2 * q] = 0;
      w.rot_pos[rb + 2 * q + 1] = j;
      w.rot_col[rb + 2 * q] = r0 + k - 1;
      w.rot_col[rb + 2 * q + 1] = w.ps_col[vo + j];
      w.rot_cs[rb + 2 * q] = c;
      w.rot_cs[rb + 2 * q + 1] = sn;
      z0 = r;
      w.ps_z[vo + j] = 0.0;
      w.ps_d[vo + j] = 0.0;
      w.ps_rot[vo + j] = kRotV;
    }
    if (z0 < tol) z0 = tol;  // small z_1 is raised to tol (after the scan)
    w.ps_z[vo] = z0;
  }
  // runs of close pairs: each kept candidate absorbs the followers after it
  for (int u = t; u < ncand; u += BS) {
    const int pp = w.cand[vo + nzero + u];
    if (w.status[vo + pp] != 0) continue;
    double zl = w.ps_z[vo + pp], dl = w.ps_d[vo + pp];
    int sup = w.ps_sup[vo + pp], rot = 0;
    for (int v = u + 1; v < ncand; ++v) {
      const int j = w.cand[vo + nzero + v];
      if (w.status[vo + j] != 3) break;
      const double zj = w.ps_z[vo + j];
      const double r = sqrt(zl * zl + zj * zj);
      const double c = zl / r, sn = zj / r;
      const int q = w.sgrp[vo + j];
      w.rot_pos[rb + 2 * q] = pp;
      w.rot_pos[rb + 2 * q + 1] = j;
      w.rot_col[rb + 2 * q] = w.ps_col[vo + pp];
      w.rot_col[rb + 2 * q + 1] = w.ps_col[vo + j];
      w.rot_cs[rb + 2 * q] = c;
      w.rot_cs[rb + 2 * q + 1] = sn;
      zl = r;
      dl = w.ps_d[vo + j];
      rot = kRotU | kRotV;
      w.ps_z[vo + j] = 0.0;
      w.ps_rot[vo + j] = kRotU | kRotV;
      const int sj = w.ps_sup[vo + j];
      if (sup != sj) {
        sup = 2;
        w.ps_sup[vo + j] = 2;
      }
    }
    w.ps_z[vo + pp] = zl;
    w.ps_d[vo + pp] = dl;
    w.ps_sup[vo + pp] = sup;
    w.ps_rot[vo + pp] = rot;
  }
  if (t == 0) {
    sh_cnt[0] = ncand;
    sh_cnt[1] = nzero + nclose;
    sh_cnt[2] = nzero;
    sh_cnt[3] = nclose;
  }
  __syncthreads();

  // ---- kept values (ascending), the update order [left | d=0 | both | right]
  // and the deflated values in ascending order (the zeros of the d~0 case
  // first, then the rest in scan order)
  const int per2 = (m + BS - 1) / BS;
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
  block_exscan_w<6, BS>(cv, tot6, shi);
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
  rho = block_sum_n<BS>(rho, shd);

  // ---- x1 and y in place: rotate the children's null vectors (V columns
  // r0+k-1 and r0+m) by (c0, s0) over the node's rows
  for (int row = t; row < m + s; row += BS) {
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
    NodeState st = w.st[nd.id];
    st.N = N;
    st.n1 = n1;
    st.n2 = n2;
    st.n3 = n3;
    st.nrot = sh_cnt[1];
    st.nzero_d = sh_cnt[2];
    st.nclose = sh_cnt[3];
    st.nsmall_z = m - 1 - sh_cnt[0] - sh_cnt[2];
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
  if (nnodes <= 0) return;
  int gy = (max_m + kBlock - 1) / kBlock;
  const int cap = 4096 / nnodes;
  if (gy > cap) gy = cap > 0 ? cap : 1;
  hipLaunchKernelGGL(k_zsort, dim3(nnodes, gy), dim3(kBlock), 0, st, nodes, w);
  // large merges: 1024 threads, a quarter of the sequential segment per thread
  if (max_m >= 2048) hipLaunchKernelGGL(k_prep<1024>, dim3(nnodes), dim3(1024), 0, st, nodes, w);
  else hipLaunchKernelGGL(k_prep<256>, dim3(nnodes), dim3(256), 0, st, nodes, w);
}

}  // namespace bdc
