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

// Rotations of the values within tol of d_1 = 0 into z_1 (one thread; all
// near-zero values precede every candidate in the scan order, so they take
// rotation slots 0..nzero-1).  cand[0..nzero) lists their positions.
__device__ inline void zero_rotations(const Work& w, int64_t vo, int64_t rb, int r0, int k, int nzero,
                                      double tol) {
  if (threadIdx.x != 0) return;
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

// Runs of close pairs: each kept candidate (status 0) absorbs the followers
// (status 3) after it in the candidate list cand[nzero .. nzero+ncand), one
// thread per run; a follower's rotation slot is in sgrp[its position].
template <int BS>
__device__ inline void absorb_runs(const Work& w, int64_t vo, int64_t rb, int nzero, int ncand) {
  for (int u = threadIdx.x; u < ncand; u += BS) {
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
}

// x1 and y in place -- the children's null vectors (V columns r0+k-1 and
// r0+m) rotated by (c0, s0) over the node's rows -- their row supports, and
// the node's state (st carries the counts and rho; the scale, tol and the
// rotation are set here).
template <int BS>
__device__ inline void finish_node(const NodeDesc& nd, const Work& w, const MergeHead& h, double tol,
                                   NodeState st) {
  const int m = nd.m, k = nd.k, s = nd.s, r0 = nd.r0;
  const int64_t ld = nd.ld, pv = nd.vec_off;
  double* V = w.Vw + nd.mat_off;
  const double c0 = h.c0, s0 = h.s0;
  for (int row = threadIdx.x; row < m + s; row += BS) {
    const int64_t gr = r0 + row;
    const double q1 = row < k ? V[gr + (int64_t)(r0 + k - 1) * ld] : 0.0;
    const double q2 = (s && row >= k) ? V[gr + (int64_t)(r0 + m) * ld] : 0.0;
    V[gr + (int64_t)(r0 + k - 1) * ld] = c0 * q1 + s0 * q2;
    if (s) V[gr + (int64_t)(r0 + m) * ld] = -s0 * q1 + c0 * q2;
  }
  if (threadIdx.x == 0) {
    w.vlo[pv + r0 + k - 1] = r0;
    w.vhi[pv + r0 + k - 1] = r0 + m + s;
    if (s) {
      w.vlo[pv + r0 + m] = r0;
      w.vhi[pv + r0 + m] = r0 + m + s;
    }
    st.scale = h.p;
    st.tol = tol;
    st.c0 = c0;
    st.s0 = s0;
    w.st[nd.id] = st;
  }
}

// z and d of every node column and its place in the sorted order (as
// k_zsort), done by one workgroup for its own merge of at most 64 * Q * BS/64
// values: each thread takes Q columns, the children's values are staged in
// LDS (ssig) for the binary searches, and the loads of the Q columns are
// issued together (the V entry is fetched beside its support bounds and
// dropped when the row lies outside them; row < m and column < m keep it
// inside the node's block).  Returns the largest of d and |z|; the positions
// are written before the closing barrier.
template <int BS, int Q>
__device__ double zsort_node(const NodeDesc& nd, const Work& w, const MergeHead& h, double* ssig, double* shd) {
  const int m = nd.m, k = nd.k, r0 = nd.r0, m2 = nd.m - nd.k;
  const int64_t ld = nd.ld, pv = nd.vec_off, vo = nd.vec_off + nd.r0;
  const double* V = w.Vw + nd.mat_off;
  const int t = threadIdx.x;
  if (t == 0 && !(fabs(w.d[pv + r0 + k - 1]) <= DBL_MAX && fabs(w.e[pv + r0 + k - 1]) <= DBL_MAX))
    atomicOr(&w.ctl->nonfinite, 1);
  const double* sig = w.sig + vo;
  int pc[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int c = t + q * BS;
    double sv = 0.0;
    pc[q] = r0 + k - 1;
    if (c < m) {
      sv = sig[c];
      if (c != k - 1) pc[q] = w.col[vo + c];
    }
    ssig[c] = sv;
  }
  double qv[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int c = t + q * BS;
    const int row = c < k ? r0 + k - 1 : r0 + k;  // boundary row of the child's right basis
    const int lo = w.vlo[pv + pc[q]], hi = w.vhi[pv + pc[q]];
    const double v = c < m ? V[row + (int64_t)pc[q] * ld] : 0.0;
    qv[q] = (row >= lo && row < hi) ? v : 0.0;
  }
  __syncthreads();
  double lmax = 0.0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int c = t + q * BS;
    if (c >= m) continue;
    double dv, zv;
    int pos, sup;
    if (c < k - 1) {
      const double sv = ssig[c];
      dv = sv / h.p;
      zv = h.a_s * qv[q];
      pos = 1 + c + count_less(ssig + k, m2, sv);
      sup = 1;
    } else if (c == k - 1) {
      dv = 0.0;
      zv = h.rr;
      pos = 0;
      sup = 0;
    } else {
      const double sv = ssig[c];
      dv = sv / h.p;
      zv = h.b_s * qv[q];
      pos = 1 + (c - k) + count_leq(ssig, k - 1, sv);
      sup = 3;
    }
    w.ps_d[vo + pos] = dv;
    w.ps_z[vo + pos] = zv;
    w.ps_c[vo + pos] = c;
    w.ps_col[vo + pos] = pc[q];
    w.ps_sup[vo + pos] = sup;
    w.ps_rot[vo + pos] = 0;
    w.status[vo + pos] = 0;
    lmax = fmax(lmax, fmax(dv, fabs(zv)));
  }
  return block_max_n<BS>(lmax, shd);
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
  const int m = nd.m, k = nd.k, r0 = nd.r0;
  const int64_t vo = nd.vec_off + nd.r0;
  const int t = threadIdx.x;
  const MergeHead h = merge_head(nd, w);
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

  zero_rotations(w, vo, rb, r0, k, nzero, tol);
  absorb_runs<BS>(w, vo, rb, nzero, ncand);
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

  NodeState st = w.st[nd.id];
  st.N = N;
  st.n1 = n1;
  st.n2 = n2;
  st.n3 = n3;
  st.nrot = sh_cnt[1];
  st.nzero_d = sh_cnt[2];
  st.nclose = sh_cnt[3];
  st.nsmall_z = m - 1 - sh_cnt[0] - sh_cnt[2];
  st.rho = rho;
  finish_node<BS>(nd, w, h, tol, st);
}


// lanes below this one with their bit set in M
__device__ inline int rank_below(uint64_t M) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(M >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)M, 0u));
}

// Exclusive prefix over the wavefronts of K wave-uniform counts c (lane 0 of
// each wavefront publishes them); before[] gets the sum over earlier
// wavefronts, total[] the sum over all.  sh holds K * BS/64 ints.
template <int K, int BS>
__device__ inline void wave_exscan(const int (&c)[K], int (&before)[K], int (&total)[K], int* sh) {
  constexpr int NW = BS / 64;
  const int wv = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
    for (int q = 0; q < K; ++q) sh[q * NW + wv] = c[q];
  __syncthreads();
  for (int q = 0; q < K; ++q) {
    int b = 0, a = 0;
    for (int u = 0; u < NW; ++u) {
      const int x = sh[q * NW + u];
      if (u < wv) b += x;
      a += x;
    }
    before[q] = b;
    total[q] = a;
  }
}

// The same deflation as k_prep, laid out for the memory system: position
// pos = 64 (wv Q + q) + lane is handled by lane `lane` of wavefront wv at step
// q, so every load and store of a step is one contiguous 64-element run, and
// the node's z and d stay in registers between the passes.  Ranks inside a
// step come from ballots (scan order = position order = step-major,
// lane-minor); the previous candidate of a position is the nearest lower lane
// of its step with a candidate, else the last candidate of the earlier steps
// and wavefronts.  Decisions, lists and rotations are those of k_prep bit for
// bit.  Needs m <= 64 Q BS/64.
template <int BS, int Q, bool kFused>
__global__ __launch_bounds__(BS) void k_prep_w(const NodeDesc* __restrict__ nodes, Work w) {
  constexpr int NW = BS / 64;
  constexpr int kCap = 64 * Q * NW;  // positions the workgroup covers
  static_assert(Q <= 32, "class bits are kept in 32-bit masks");
  __shared__ double sh_last[NW];
  __shared__ int sh_has[NW];
  __shared__ int shi[6 * NW];
  __shared__ double shd[NW];
  __shared__ double sh_rho[NW * Q];  // rho per 64-position block
  __shared__ double ssig[kFused ? kCap : 1];

  const NodeDesc nd = nodes[blockIdx.x];
  const int m = nd.m, k = nd.k, r0 = nd.r0;
  const int64_t vo = nd.vec_off + nd.r0;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const MergeHead h = merge_head(nd, w);
  double zmax;
  if constexpr (kFused) {
    // k_zsort's work for a merge this workgroup holds whole: the children's
    // values staged in LDS for the merge-position searches
    zmax = zsort_node<BS, Q>(nd, w, h, ssig, shd);
  } else {
    zmax = __longlong_as_double((long long)w.st[nd.id].zmax_bits);
  }
  // tol stands for eps * ||M||: 8 * 2^-52 * max(max d, max |z|)
  const double tol = 8.0 * kEps * zmax;
  const int64_t rb = 2 * vo;
  const int pbase = wv * 64 * Q + lane;

  // ---- pass 1: classes of positions 1..m-1 (bit q of each mask), in
  // chunks of up to 8 steps whose z and d are loaded together; with more
  // than one chunk, d is loaded again for the close-pair pass
  constexpr int QC = Q < 8 ? Q : 8;
  double dq[QC];
  uint32_t b_small = 0, b_zero = 0, b_cand = 0;
  double wl = 0.0;  // the wavefront's last candidate value
  int wh = 0;
#pragma unroll
  for (int q0 = 0; q0 < Q; q0 += QC) {
    double zc[QC];
#pragma unroll
    for (int u = 0; u < QC; ++u) {
      const int pos = pbase + 64 * (q0 + u);
      zc[u] = pos < m ? w.ps_z[vo + pos] : 0.0;
      dq[u] = pos < m ? w.ps_d[vo + pos] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < QC; ++u) {
      const int q = q0 + u, pos = pbase + 64 * q;
      if (pos < 1 || pos >= m) continue;
      const double z = zc[u], d = dq[u];
      if (fabs(z) < tol || z == 0.0) b_small |= 1u << q;
      else if (d < tol || d == 0.0) b_zero |= 1u << q;
      else b_cand |= 1u << q;
    }
#pragma unroll
    for (int u = 0; u < QC; ++u) {
      const uint64_t M = __ballot((b_cand >> (q0 + u)) & 1u);
      const double v = __shfl(dq[u], M ? 63 - __clzll((long long)M) : 0, 64);
      if (M) {
        wl = v;
        wh = 1;
      }
    }
  }
  if (lane == 0) {
    sh_last[wv] = wl;
    sh_has[wv] = wh;
  }
  __syncthreads();
  double carry = 0.0;
  int chas = 0;
  for (int u = wv - 1; u >= 0; --u)
    if (sh_has[u]) {
      carry = sh_last[u];
      chas = 1;
      break;
    }
  // close-pair followers: d - d_prev < tol against the previous candidate
  uint32_t b_close = 0;
  int cnt3[3] = {0, 0, 0};  // near-zero values, candidates, followers (this wavefront)
#pragma unroll
  for (int q0 = 0; q0 < Q; q0 += QC) {
    if (Q > QC) {
#pragma unroll
      for (int u = 0; u < QC; ++u) {
        const int pos = pbase + 64 * (q0 + u);
        dq[u] = pos < m ? w.ps_d[vo + pos] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < QC; ++u) {
      const int q = q0 + u;
      const bool c = (b_cand >> q) & 1u;
      const uint64_t M = __ballot(c);
      const uint64_t Mlt = M & ((1ull << lane) - 1ull);
      const double v = __shfl(dq[u], Mlt ? 63 - __clzll((long long)Mlt) : 0, 64);
      const double dp = Mlt ? v : carry;
      const int hp = Mlt ? 1 : chas;
      const bool close = c && hp && (dq[u] - dp < tol || dq[u] == dp);
      if (close) b_close |= 1u << q;
      const uint64_t Mz = __ballot((b_zero >> q) & 1u), Mf = __ballot(close);
      cnt3[0] += __popcll(Mz);
      cnt3[1] += __popcll(M);
      cnt3[2] += __popcll(Mf);
      const double last = __shfl(dq[u], M ? 63 - __clzll((long long)M) : 0, 64);
      if (M) {
        carry = last;
        chas = 1;
      }
    }
  }
  int base3[3], tot3[3];
  wave_exscan<3, BS>(cnt3, base3, tot3, shi);
  const int nzero = tot3[0], ncand = tot3[1], nclose = tot3[2];
  // statuses, lists, rotation slots of the followers
  {
    int bz = base3[0], bc = base3[1], bf = base3[2];
#pragma unroll 2
    for (int q = 0; q < Q; ++q) {
      const int pos = pbase + 64 * q;
      const bool sm = (b_small >> q) & 1u, zr = (b_zero >> q) & 1u, cd = (b_cand >> q) & 1u,
                 cl = (b_close >> q) & 1u;
      const uint64_t Mz = __ballot(zr), Mc = __ballot(cd), Mf = __ballot(cl);
      if (sm) {
        w.status[vo + pos] = 1;  // small z component: z_j -> 0
        w.ps_z[vo + pos] = 0.0;
      } else if (zr) {
        w.status[vo + pos] = 2;  // within tol of d_1 = 0: rotated into z_1, value 0
        w.cand[vo + bz + rank_below(Mz)] = pos;
      } else if (cd) {
        w.status[vo + pos] = cl ? 3 : 0;
        w.sgrp[vo + pos] = cl ? nzero + bf + rank_below(Mf) : -1;
        w.cand[vo + nzero + bc + rank_below(Mc)] = pos;
      }
      bz += __popcll(Mz);
      bc += __popcll(Mc);
      bf += __popcll(Mf);
    }
  }
  __syncthreads();
  zero_rotations(w, vo, rb, r0, k, nzero, tol);
  if (nclose > 0) absorb_runs<BS>(w, vo, rb, nzero, ncand);
  __syncthreads();

  // ---- kept values (ascending), the update order [left | d=0 | both | right]
  // and the deflated values (the zeros of the d~0 case first, then the rest,
  // each in position order)
  // status code per step: 0 kept, 2 zero-d, 1 other deflated, -1 none
  auto code = [&](int q) -> int {
    const int pos = pbase + 64 * q;
    if (pos >= m) return -1;
    if (((b_small | b_close) >> q) & 1u) return 1;
    if ((b_zero >> q) & 1u) return 2;
    return 0;  // candidates that stayed, and position 0
  };
  // supports of this thread's positions, 2 bits per step (loaded in chunks)
  uint32_t supbits = 0;
#pragma unroll
  for (int q0 = 0; q0 < Q; q0 += QC) {
    int sc[QC];
#pragma unroll
    for (int u = 0; u < QC; ++u) {
      const int pos = pbase + 64 * (q0 + u);
      sc[u] = pos < m ? w.ps_sup[vo + pos] : 0;
    }
#pragma unroll
    for (int u = 0; u < QC; ++u) supbits |= (uint32_t)(sc[u] & 3) << (2 * (q0 + u));
  }
  auto supq = [&](int q) -> int { return (int)((supbits >> (2 * q)) & 3u); };
  int cnt6[6] = {0, 0, 0, 0, 0, 0};  // kept, sup 1, sup 2, sup 3, zero-d, other
#pragma unroll 4
  for (int q = 0; q < Q; ++q) {
    const int cq = code(q);
    const int pos = pbase + 64 * q;
    const int sup = supq(q);
    const bool kept = cq == 0, sk = kept && pos > 0;
    cnt6[0] += __popcll(__ballot(kept));
    cnt6[1] += __popcll(__ballot(sk && sup == 1));
    cnt6[2] += __popcll(__ballot(sk && sup == 2));
    cnt6[3] += __popcll(__ballot(sk && sup == 3));
    cnt6[4] += __popcll(__ballot(cq == 2));
    cnt6[5] += __popcll(__ballot(cq == 1));
  }
  int base6[6], tot6[6];
  wave_exscan<6, BS>(cnt6, base6, tot6, shi);
  const int N = tot6[0], n1 = tot6[1], n2 = tot6[2], n3 = tot6[3], nz = tot6[4];
  double rho = 0.0;
  // the copies, four steps' loads at a time
  constexpr int QW = Q >= 8 ? 4 : (Q < 2 ? Q : 2);
#pragma unroll 1
  for (int q0 = 0; q0 < Q; q0 += QW) {
    double zc[QW], dc[QW];
    int cc[QW], rc[QW];
#pragma unroll
    for (int u = 0; u < QW; ++u) {
      const int pos = pbase + 64 * (q0 + u);
      const bool in = pos < m;
      zc[u] = in ? w.ps_z[vo + pos] : 0.0;
      dc[u] = in ? w.ps_d[vo + pos] : 0.0;
      cc[u] = in ? w.ps_col[vo + pos] : 0;
      rc[u] = in ? w.ps_rot[vo + pos] : 0;
    }
#pragma unroll
    for (int u = 0; u < QW; ++u) {
      const int q = q0 + u;
      const int cq = code(q);
      const int pos = pbase + 64 * q;
      const int sup = supq(q);
      const bool kept = cq == 0, sk = kept && pos > 0;
      const uint64_t M0 = __ballot(kept), M1 = __ballot(sk && sup == 1), M2 = __ballot(sk && sup == 2),
                     M3 = __ballot(sk && sup == 3), M4 = __ballot(cq == 2), M5 = __ballot(cq == 1);
      if (kept) {
        const int i = base6[0] + rank_below(M0);
        int g;
        if (pos == 0) g = n1;
        else if (sup == 1) g = base6[1] + rank_below(M1);
        else if (sup == 2) g = n1 + 1 + base6[2] + rank_below(M2);
        else g = n1 + 1 + n2 + base6[3] + rank_below(M3);
        w.sd[vo + i] = dc[u];
        w.sz[vo + i] = zc[u];
        w.scol[vo + i] = cc[u];
        w.srot[vo + i] = rc[u];
        w.sgrp[vo + i] = g;
        w.gsurv[vo + g] = i;
      } else if (cq >= 0) {
        const int qq = cq == 2 ? base6[4] + rank_below(M4) : nz + base6[5] + rank_below(M5);
        w.dval[vo + qq] = dc[u];
        w.dcol[vo + qq] = cc[u];
        w.drot[vo + qq] = rc[u];
      }
      // rho: each 64-position block's kept z^2 summed across its lanes
      const double bz = wave_sum(kept ? zc[u] * zc[u] : 0.0);
      if (lane == 0) sh_rho[wv * Q + q] = bz;
      base6[0] += __popcll(M0);
      base6[1] += __popcll(M1);
      base6[2] += __popcll(M2);
      base6[3] += __popcll(M3);
      base6[4] += __popcll(M4);
      base6[5] += __popcll(M5);
    }
  }
  // the blocks added in position order (block wv Q + q holds positions
  // 64 (wv Q + q) ..): the same sums in the same order for any workgroup
  // shape, so a merge gets the same rho whichever form its level launches
  __syncthreads();
  if (t == 0)
    for (int b = 0; b < NW * Q; ++b) rho += sh_rho[b];

  NodeState st = w.st[nd.id];
  st.N = N;
  st.n1 = n1;
  st.n2 = n2;
  st.n3 = n3;
  st.nrot = nzero + nclose;
  st.nzero_d = nzero;
  st.nclose = nclose;
  st.nsmall_z = m - 1 - ncand - nzero;
  st.rho = rho;
  finish_node<BS>(nd, w, h, tol, st);
}

}  // namespace

constexpr int kPrepWide = 256;

void launch_prep(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, hipStream_t st) {
  if (nnodes <= 0) return;
  int gy = (max_m + kBlock - 1) / kBlock;
  const int cap = 4096 / nnodes;
  if (gy > cap) gy = cap > 0 ? cap : 1;
  // one wavefront per node up to 256 values, then 4 and 16 (4 to 16 steps
  // per lane); beyond 16384 values the segment-per-thread kernel.  Merges of
  // at most 1024 values: the one workgroup per node does k_zsort's work too.
  const dim3 g(nnodes);
  // A level of at most kPrepWide merges (a CU each) gives every value of a
  // merge its own thread (fewer dependent steps per merge); a level of more
  // merges keeps several values per thread, which fills the CUs better
  // (measured: the single 16384 problem's deflation 0.236 against 0.252 ms,
  // the 2000-problem batch's 0.49 against 0.56).  Both give the same results.
  const bool wide = nnodes <= kPrepWide;
  if (max_m <= 64) hipLaunchKernelGGL((k_prep_w<64, 1, true>), g, dim3(64), 0, st, nodes, w);
  else if (max_m <= 128 && wide) hipLaunchKernelGGL((k_prep_w<128, 1, true>), g, dim3(128), 0, st, nodes, w);
  else if (max_m <= 128) hipLaunchKernelGGL((k_prep_w<64, 2, true>), g, dim3(64), 0, st, nodes, w);
  else if (max_m <= 256 && wide) hipLaunchKernelGGL((k_prep_w<256, 1, true>), g, dim3(256), 0, st, nodes, w);
  else if (max_m <= 256) hipLaunchKernelGGL((k_prep_w<64, 4, true>), g, dim3(64), 0, st, nodes, w);
  else if (max_m <= 1024 && wide) hipLaunchKernelGGL((k_prep_w<1024, 1, true>), g, dim3(1024), 0, st, nodes, w);
  else if (max_m <= 1024) hipLaunchKernelGGL((k_prep_w<256, 4, true>), g, dim3(256), 0, st, nodes, w);
  else {
    hipLaunchKernelGGL(k_zsort, dim3(nnodes, gy), dim3(kBlock), 0, st, nodes, w);
    if (max_m <= 4096) hipLaunchKernelGGL((k_prep_w<1024, 4, false>), g, dim3(1024), 0, st, nodes, w);
    else if (max_m <= 8192) hipLaunchKernelGGL((k_prep_w<1024, 8, false>), g, dim3(1024), 0, st, nodes, w);
    else if (max_m <= 16384) hipLaunchKernelGGL((k_prep_w<1024, 16, false>), g, dim3(1024), 0, st, nodes, w);
    else hipLaunchKernelGGL(k_prep<1024>, g, dim3(1024), 0, st, nodes, w);
  }
}

}  // namespace bdc
