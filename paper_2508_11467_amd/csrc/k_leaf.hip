// Leaf solves of the divide-and-conquer tree (Algorithm 2 step (1): the
// bottom subproblems by QR iteration).
//
// One 64-lane wavefront per leaf of m <= 32 rows and m+s columns.  The
// bidiagonal lives in LDS; every lane computes the same scalar Givens
// sequence (implicit-shift Golub-Kahan sweeps with a Wilkinson shift, zero
// diagonal chasing), and lane r applies each rotation to row r of the
// accumulated W (m x m) and Q ((m+s) x (m+s)), stored column-major in LDS so
// the 64 lanes touch consecutive words.  The leaf is first scaled by a power
// of two so no square can overflow; the values are scaled back on output.
// Output columns are written sorted by value (ascending); each physical
// column records the leaf's row range as its support.
#include "bdc_internal.h"

namespace bdc {
namespace {

constexpr double kEps = 0x1p-52;

// lane k's value of a per-lane double, as a wave-uniform value
__device__ inline double lane_val(double v, int k) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
  return __hiloint2double(hi, lo);
}

// (c, s, r) with c f + s g = r >= 0 and -s f + c g = 0.  The leaf is scaled
// so that |f|, |g| <= 2; the reciprocal square root (hardware estimate and
// two Newton steps) is used unless f^2 + g^2 is near underflow.
__device__ inline void givens(double f, double g, double& c, double& s, double& r) {
  if (g == 0.0) {
    c = f >= 0.0 ? 1.0 : -1.0;
    s = 0.0;
    r = fabs(f);
    return;
  }
  const double q = fma(f, f, g * g);
  if (q > 0x1p-960) {
    double y = __builtin_amdgcn_rsq(q);
    const double hq = 0.5 * q;
    y = y * fma(-hq * y, y, 1.5);
    y = y * fma(-hq * y, y, 1.5);
    c = f * y;
    s = g * y;
    r = q * y;
  } else {
    r = hypot(f, g);
    c = f / r;
    s = g / r;
  }
}

// columns (i, j) of an LDS matrix (column stride ld) <- (c a_i + s a_j,
// -s a_i + c a_j), row = lane
__device__ inline void rot_cols(double* A, int ld, int rows, int i, int j, double c, double s, int lane) {
  if (lane < rows) {
    const double ai = A[lane + i * ld];
    const double aj = A[lane + j * ld];
    A[lane + i * ld] = c * ai + s * aj;
    A[lane + j * ld] = -s * ai + c * aj;
  }
}

__device__ inline double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// One 64-lane wavefront per leaf.  Lane L holds d_L and e_L (the
// superdiagonal entry right of d_L) in registers; the Givens chain runs on
// wave-uniform values read with readlane, and each rotation of W and Q is
// applied by lane r to row r of the column-major LDS copies.  Along a sweep
// the column being rotated forward stays in a register, so each step reads
// one new column (independent of the chain) and writes one.
// The LDS copies are sized for leaves of at most ML rows, so launches of
// small leaves fit more wavefronts per CU (the chain is latency-bound, and a
// batch has many leaves per SIMD).
template <int ML>
__global__ __launch_bounds__(64) void k_leaf(const LeafDesc* __restrict__ leaves, Work w) {
  constexpr int kLd = ML + 1;  // LDS column stride (doubles)
  __shared__ double W[ML * kLd];
  __shared__ double Q[(ML + 1) * kLd];

  const LeafDesc L = leaves[blockIdx.x];
  const int m = L.m, s = L.s, ms = m + s, r0 = L.r0;
  const int lane = threadIdx.x;
  const int64_t ld = L.ld;
  const int64_t pv = L.vec_off;
  unsigned long long nrot_w = 0, nrot_q = 0;  // rotations applied to W and to Q

  for (int i = lane; i < ML * kLd; i += 64) W[i] = 0.0;
  for (int i = lane; i < (ML + 1) * kLd; i += 64) Q[i] = 0.0;
  __syncthreads();
  if (lane < m) W[lane + lane * kLd] = 1.0;
  if (lane < ms) Q[lane + lane * kLd] = 1.0;

  // load and scale by a power of two
  double dv = 0.0, ev = 0.0;
  if (lane < m) dv = w.d[pv + r0 + lane];
  if (lane < m - 1 + s) ev = w.e[pv + r0 + lane];
  // every entry of d and e belongs to exactly one leaf or one merge's middle
  // row, so leaves and merges between them check all of the input
  const bool bad = !(fabs(dv) <= 1.79769313486231570e308) || !(fabs(ev) <= 1.79769313486231570e308);
  if (__any(bad) && lane == 0) atomicOr(&w.ctl->nonfinite, 1);
  const double amax = wave_max(fmax(fabs(dv), fabs(ev)));
  double p = 1.0;
  if (amax > 0.0 && amax <= 1.79e308) {
    int ex;
    frexp(amax, &ex);
    p = ldexp(1.0, ex);
  }
  double dreg = dv / p;  // d_lane
  double ereg = ev / p;  // e_lane (lane m-1: the extra column's entry when s = 1)
  const double tiny = kEps * (amax / p);
  __syncthreads();

  // s = 1: remove the extra column's entry, bottom row first.  The right
  // rotation of columns (j, m) zeroes B[j, m] and moves a fill-in to B[j-1, m].
  if (s == 1) {
    double f = lane_val(ereg, m - 1);
    if (lane == m - 1) ereg = 0.0;
    for (int j = m - 1; j >= 0; --j) {
      double c, sn, r;
      givens(lane_val(dreg, j), f, c, sn, r);
      if (lane == j) dreg = r;
      if (j > 0) {
        const double t = lane_val(ereg, j - 1);
        if (lane == j - 1) ereg = c * t;
        f = -sn * t;
      }
      rot_cols(Q, kLd, ms, j, m, c, sn, lane);
      ++nrot_q;
    }
  }

  const int max_steps = w.max_leaf_sweeps * (m > 0 ? m : 1);
  int steps = 0;
  int hi = m - 1;
  while (hi > 0) {
    // negligible superdiagonals -> 0; then the unreduced block [lo, hi]
    const double dnext = __shfl_down(dreg, 1, 64);
    if (lane < hi && fabs(ereg) <= kEps * (fabs(dreg) + fabs(dnext))) ereg = 0.0;
    const unsigned long long nz = __ballot(lane < hi && ereg != 0.0);
    if (!((nz >> (hi - 1)) & 1ull)) {
      --hi;
      continue;
    }
    if (steps >= max_steps) {
      if (lane == 0) atomicAdd(&w.ctl->leaf_capped, 1);
      break;
    }
    ++steps;
    const unsigned long long zero_below = ~nz & ((1ull << (hi - 1)) - 1ull);
    const int lo = zero_below ? 64 - __builtin_clzll(zero_below) : 0;
    const unsigned long long zd = __ballot(lane >= lo && lane <= hi && fabs(dreg) <= tiny);
    if (zd) {
      const int i = __builtin_ctzll(zd);
      if (lane == i) dreg = 0.0;
      if (i < hi) {
        // chase B[i, i+1] along row i with left rotations of rows (j, i)
        double f = lane_val(ereg, i);
        if (lane == i) ereg = 0.0;
        for (int j = i + 1; j <= hi; ++j) {
          double c, sn, r;
          givens(lane_val(dreg, j), f, c, sn, r);
          if (lane == j) dreg = r;
          if (j < hi) {
            const double t = lane_val(ereg, j);
            f = -sn * t;
            if (lane == j) ereg = c * t;
          }
          rot_cols(W, kLd, m, j, i, c, sn, lane);
          ++nrot_w;
        }
      } else {
        // chase B[hi-1, hi] up column hi with right rotations of columns (j, hi)
        double f = lane_val(ereg, hi - 1);
        if (lane == hi - 1) ereg = 0.0;
        for (int j = hi - 1; j >= lo; --j) {
          double c, sn, r;
          givens(lane_val(dreg, j), f, c, sn, r);
          if (lane == j) dreg = r;
          if (j > lo) {
            const double t = lane_val(ereg, j - 1);
            f = -sn * t;
            if (lane == j - 1) ereg = c * t;
          }
          rot_cols(Q, kLd, ms, j, hi, c, sn, lane);
          ++nrot_q;
        }
      }
      continue;
    }
    // Wilkinson shift: eigenvalue of the trailing 2x2 of B^T B nearer its end
    double mu;
    {
      const double dm = lane_val(dreg, hi - 1), dn = lane_val(dreg, hi), fm = lane_val(ereg, hi - 1);
      const double g = (hi - 1 > lo) ? lane_val(ereg, hi - 2) : 0.0;
      const double t11 = dm * dm + g * g, t12 = dm * fm, t22 = dn * dn + fm * fm;
      if (t12 == 0.0) {
        mu = t22;
      } else {
        const double delta = 0.5 * (t11 - t22);
        const double root = hypot(delta, t12);
        const double denom = delta + (delta >= 0.0 ? root : -root);
        mu = t22 - t12 * t12 / denom;
      }
    }
    // one implicit-shift sweep, bulge chased from lo to hi
    double dk = lane_val(dreg, lo), ek = lane_val(ereg, lo);
    double y = dk * dk - mu;
    double z = dk * ek;
    double bulge = 0.0, eprev = 0.0;
    double qk = lane < ms ? Q[lane + lo * kLd] : 0.0;
    double wk = lane < m ? W[lane + lo * kLd] : 0.0;
    for (int k = lo; k < hi; ++k) {
      // next columns of Q and W (independent of the Givens chain)
      const double qk1 = lane < ms ? Q[lane + (k + 1) * kLd] : 0.0;
      const double wk1 = lane < m ? W[lane + (k + 1) * kLd] : 0.0;
      const double dk1 = lane_val(dreg, k + 1);
      const double ek1 = (k < hi - 1) ? lane_val(ereg, k + 1) : 0.0;
      if (k > lo) {
        y = eprev;
        z = bulge;
      }
      double c, sn, r;
      givens(y, z, c, sn, r);
      if (k > lo && lane == k - 1) ereg = r;
      const double ndk = c * dk + sn * ek;
      const double nek = -sn * dk + c * ek;
      bulge = sn * dk1;
      const double ndk1 = c * dk1;
      {
        const double a = c * qk + sn * qk1, b = -sn * qk + c * qk1;
        if (lane < ms) Q[lane + k * kLd] = a;
        qk = b;
      }
      givens(ndk, bulge, c, sn, r);
      if (lane == k) dreg = r;
      eprev = c * nek + sn * ndk1;  // e_k
      dk = -sn * nek + c * ndk1;    // d_{k+1}
      ek = ek1;
      if (k < hi - 1) {
        bulge = sn * ek1;
        ek = c * ek1;  // e_{k+1}
      }
      {
        const double a = c * wk + sn * wk1, b = -sn * wk + c * wk1;
        if (lane < m) W[lane + k * kLd] = a;
        wk = b;
      }
    }
    if (lane == hi - 1) ereg = eprev;
    if (lane == hi) dreg = dk;
    if (lane < ms) Q[lane + hi * kLd] = qk;
    if (lane < m) W[lane + hi * kLd] = wk;
    nrot_q += hi - lo;
    nrot_w += hi - lo;
  }

  // signs, ranks (ascending, ties by index) and output
  __syncthreads();
  double sv = 0.0;
  int rank = 0;
  if (lane < m) {
    sv = fabs(dreg);
    if (dreg < 0.0)
      for (int r = 0; r < m; ++r) W[r + lane * kLd] = -W[r + lane * kLd];
  }
  for (int j = 0; j < m; ++j) {
    const double sj = fabs(lane_val(dreg, j));
    rank += (lane < m && (sj < sv || (sj == sv && j < lane))) ? 1 : 0;
  }
  __syncthreads();
  double* Uw = w.Uw + L.mat_off;
  double* Vw = w.Vw + L.mat_off;
  for (int c = 0; c < m; ++c) {
    const int rc = __shfl(rank, c, 64);
    const int64_t pc = r0 + rc;
    if (lane < m) Uw[(r0 + lane) + pc * ld] = W[lane + c * kLd];
    if (lane < ms) Vw[(r0 + lane) + pc * ld] = Q[lane + c * kLd];
  }
  if (s == 1 && lane < ms) Vw[(r0 + lane) + (int64_t)(r0 + m) * ld] = Q[lane + m * kLd];
  if (lane < m) {
    w.sig[pv + r0 + rank] = sv * p;
    w.col[pv + r0 + lane] = r0 + lane;
    w.ulo[pv + r0 + lane] = r0;
    w.uhi[pv + r0 + lane] = r0 + m;
    w.vlo[pv + r0 + lane] = r0;
    w.vhi[pv + r0 + lane] = r0 + ms;
  }
  if (s == 1 && lane == 0) {
    w.vlo[pv + r0 + m] = r0;
    w.vhi[pv + r0 + m] = r0 + ms;
  }
  // 6 flops per row per rotation
  if (lane == 0) w.leaf_fl[blockIdx.x] = 6ull * (nrot_w * (unsigned long long)m + nrot_q * (unsigned long long)ms);
}

__global__ __launch_bounds__(256) void k_reset(Ctl* ctl, NodeState* st, SecCount* sec, int nnodes) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->nonfinite = 0;
    ctl->leaf_capped = 0;
  }
  for (int i = blockIdx.x * 256 + threadIdx.x; i < nnodes; i += gridDim.x * 256) {
    st[i].zmax_bits = 0ull;
    sec[i].evals = 0ull;
    sec[i].terms = 0ull;
    sec[i].capped = 0ull;
  }
}

}  // namespace

void launch_reset(Ctl* ctl, NodeState* nst, SecCount* sec, int nnodes, hipStream_t st) {
  int blocks = (nnodes + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 64) blocks = 64;
  hipLaunchKernelGGL(k_reset, dim3(blocks), dim3(256), 0, st, ctl, nst, sec, nnodes);
}

void launch_leaf(const LeafDesc* leaves, int nleaves, int max_m, const Work& w, hipStream_t st) {
  if (nleaves <= 0) return;
  if (max_m <= 8) hipLaunchKernelGGL(k_leaf<8>, dim3(nleaves), dim3(64), 0, st, leaves, w);
  else if (max_m <= 16) hipLaunchKernelGGL(k_leaf<16>, dim3(nleaves), dim3(64), 0, st, leaves, w);
  else if (max_m <= 24) hipLaunchKernelGGL(k_leaf<24>, dim3(nleaves), dim3(64), 0, st, leaves, w);
  else hipLaunchKernelGGL(k_leaf<kMaxLeaf>, dim3(nleaves), dim3(64), 0, st, leaves, w);
}

}  // namespace bdc
