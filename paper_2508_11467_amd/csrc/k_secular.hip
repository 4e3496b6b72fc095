// Merge stage after deflation (Algorithm 4, the GPU-based lasd3), entirely
// on the GPU:
//   k_secular  roots of the secular equation (eq. M-svd-val), one lane per
//              root.  The paper solves them on CPU threads with LAPACK's
//              lasd4; here each root is bracketed, its origin pole chosen by
//              the sign of f at the interval midpoint (in omega^2) -- or,
//              with the learned start, by the half of the interval holding
//              the proposed position, where the first evaluation is made and
//              from which an iterate that crosses the midpoint is moved to
//              the other pole's frame -- and the
//              iteration uses R.-C. Li's two-pole "middle way" rational model
//              matched in value and slope, with bisection whenever a step
//              leaves the bracket.  A root is stored as omega = d[o] + tau so
//              every d_j^2 - omega^2 is formed as ((d_j - d_o) - tau)(d_j + d_o
//              + tau) without cancellation.  The sums over poles left of the
//              root's interval run upwards and those right of it downwards
//              (far to near); all lanes of a wavefront read the same pole at
//              each step.
//   k_lowner   Gu-Eisenstat recomputation of z (eq. bdc-zi): one wavefront
//              per pole, each lane a strided partial product of the ratios,
//              then a cross-lane product reduction (the paper's block-i /
//              thread-j product with shuffles).
//   k_vectors  singular vectors of M~ (eq. M-svd-vec), one wavefront per root
//              column, written in the row order of the vector update and
//              normalised.
#include <type_traits>

#include "bdc_internal.h"
#include "block_util.h"
#include "mlp_device.h"

namespace bdc {
namespace {

constexpr double kEps = 0x1p-52;

constexpr int kSecRoots = 64;    // roots per workgroup (one per lane)
constexpr int kSecWaves = 4;     // wavefronts splitting the pole sums
constexpr int kSecChunk = 512;   // poles staged in LDS per wavefront

// 1/x to full precision: the hardware estimate refined by two Newton steps
__device__ inline double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

struct Part {
  double s, ds, E;
};

// Sum the pole terms j = j0, j0+step, ... (count terms) in that order.  Four
// terms are formed at a time so their reciprocals overlap; they are still
// accumulated one by one in order.
__device__ inline void sum_terms(const double* __restrict__ dj, const double* __restrict__ zz, int j0, int step,
                                 int count, double ov, double tau, Part& P) {
  int q = 0;
  for (; q + 4 <= count; q += 4) {
    double t[4], r[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + (q + u) * step;
      const double dd = dj[j];
      const double del = ((dd - ov) - tau) * ((dd + ov) + tau);  // d_j^2 - omega^2
      r[u] = recip(del);
      t[u] = zz[j] * r[u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      P.s += t[u];
      P.ds = fma(t[u], r[u], P.ds);
      P.E += fabs(t[u]);
    }
  }
  for (; q < count; ++q) {
    const int j = j0 + q * step;
    const double dd = dj[j];
    const double del = ((dd - ov) - tau) * ((dd + ov) + tau);
    const double r = recip(del);
    const double t = zz[j] * r;
    P.s += t;
    P.ds = fma(t, r, P.ds);
    P.E += fabs(t);
  }
}

// One root's iteration state (one lane).  The start, the origin choice, the
// model step, the safeguard, the stopping rule and the learned start's
// re-referencing are the same in both secular kernels.
struct Root {
  int i, lp, rp, o, iters, capped;
  bool last, need, first;
  double dl, dr, ov, tau, lo, hi, mu, base_v, h;

  __device__ void init(const double* __restrict__ d, int N, double rho, double z0, int i_, bool active,
                       bool learned, float xp) {
    i = i_;
    last = i == N - 1;
    lp = active ? (last ? N - 2 : i) : 0;  // left model pole
    rp = lp + 1;
    dl = dr = ov = tau = lo = hi = mu = base_v = h = 0.0;
    o = iters = capped = 0;
    need = active && N > 1;
    first = true;
    if (active && N == 1) tau = fabs(z0);  // f = 1 - z^2/omega^2: omega = |z| exactly
    if (!need) return;
    dl = d[lp];
    dr = d[rp];
    if (learned) {
      // first evaluation at the proposed position x of the interval; its
      // half (split at the midpoint in omega^2) gives the origin pole
      const double x = fmin(fmax((double)xp, 0x1p-20), 1.0 - 0x1p-20);
      first = false;
      if (last) {
        h = rho / (dr + sqrt(dr * dr + rho));
        o = rp;
        tau = x * h;
        lo = 0.0;
        hi = h;
      } else {
        h = dr - dl;
        mu = 0.5 * (dr - dl) * (dr + dl);
        const double t0 = x * h;
        if (t0 * (2.0 * dl + t0) > mu) {
          o = rp;
          tau = (x - 1.0) * h;
          lo = -h;
          hi = 0.0;
        } else {
          o = lp;
          tau = t0;
          lo = 0.0;
          hi = h;
        }
      }
      ov = o == rp ? dr : dl;
    } else {
      // first evaluation: the midpoint in omega^2 of the root's interval
      base_v = last ? dr : dl;
      mu = last ? 0.5 * rho : 0.5 * (dr - dl) * (dr + dl);
      ov = base_v;
      tau = mu / (base_v + sqrt(base_v * base_v + mu));
    }
  }

  // After an evaluation f (E = 1 + sum |terms|) at the current point.
  __device__ void update(double f, double dpsi, double dphi, double E, double rho, int maxit, bool learned) {
    ++iters;
    bool conv = fabs(f) <= 8.0 * kEps * E;
    if (first) {
      first = false;
      // origin: the pole nearer the root, by the sign of f at the midpoint
      const bool go_right = !last && f < 0.0;
      o = (last || go_right) ? rp : lp;
      const double wmid = base_v + tau;
      ov = o == rp ? dr : dl;
      if (go_right) tau = -mu / (dr + wmid);
      if (last) {
        lo = 0.0;
        hi = rho / (dr + sqrt(dr * dr + rho));
        if (f < 0.0) lo = tau;
        else hi = tau;
      } else if (go_right) {
        lo = tau;
        hi = 0.0;
      } else {
        lo = 0.0;
        hi = tau;
      }
    } else {
      if (f < 0.0) lo = tau;
      else hi = tau;
    }
    if (!conv && iters < maxit) {
      // two-pole rational model at the current point
      const double Dl = ((dl - ov) - tau) * ((dl + ov) + tau);
      const double Dr = ((dr - ov) - tau) * ((dr + ov) + tau);
      const double c = f - Dl * dpsi - Dr * dphi;
      const double a = (Dl + Dr) * f - Dl * Dr * (dpsi + dphi);
      const double b = Dl * Dr * f;
      const double disc = sqrt(fabs(a * a - 4.0 * b * c));
      double eta;
      if (c == 0.0) eta = b / a;
      else if (last) eta = (a >= 0.0) ? (a + disc) / (2.0 * c) : 2.0 * b / (a - disc);
      else eta = (a <= 0.0) ? (a - disc) / (2.0 * c) : 2.0 * b / (a + disc);
      const double om = ov + tau;
      const double omn = sqrt(om * om + eta);
      double tn = tau + eta / (om + omn);
      if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
      // a step at the rounding level is accepted without another evaluation
      if (fabs(tn - tau) <= 2.0 * kEps * fabs(tn)) conv = true;
      tau = tn;
      if (learned && !last) {
        // an iterate that crossed the midpoint is re-referenced to the
        // other pole and evaluated there before it may stop
        if (o == lp && tau * (2.0 * dl + tau) > mu) {
          o = rp;
          ov = dr;
          tau -= h;
          lo -= h;
          hi -= h;
          conv = false;
        } else if (o == rp && tau * (2.0 * dr + tau) < -mu) {
          o = lp;
          ov = dl;
          tau += h;
          lo += h;
          hi += h;
          conv = false;
        }
      }
    }
    if (!conv && iters >= maxit) capped = 1;
    need = !conv && iters < maxit;
  }
};


// Pole staging of the secular kernel; with the in-kernel learned start the
// network's weights and activations share its LDS (they are done with before
// the poles are staged).
struct PoleLds {
  double cd[kSecWaves][kSecChunk];
  double cz[kSecWaves][kSecChunk];
};
// Activations of R rows, and the feature scratch for MB far-field blocks in
// A.a1 .. A.a2 (the network's weights are read from global memory).
template <int R, int MB>
struct MlpSharedT {
  using Feat = FeatLdsT<MB, R>;
  FastActT<R> A;
  static_assert(sizeof(Feat) <= sizeof(A.a1) + sizeof(A.a2), "feature scratch");
};
using MlpShared = MlpSharedT<kRows, kMaxBlocks>;
template <int kMode>
struct SecLds {
  PoleLds p;
};
template <>
struct SecLds<2> {
  union {
    PoleLds p;
    MlpShared m;
  };
};

// The network's proposals for roots base .. base+nrows-1 (nrows a multiple
// of 16, at most 64) into xs (all threads of the workgroup; LDS of m is free
// afterwards).
template <class MS>
__device__ void learned_proposals(const Work& w, MS& m, const double* __restrict__ d,
                                  const double* __restrict__ z, int N, double rho, int base, float* xs,
                                  int nrows) {
  using Feat = typename MS::Feat;
  Feat& F = *reinterpret_cast<Feat*>(m.A.a1);
  const int B = far_block(N);
  for (int q = threadIdx.x; q < nrows * kFP; q += blockDim.x) m.A.a0[q] = 0;
  far_moments(d, z, N, B, F);
  __syncthreads();
  block_features(
      d, z, N, rho, base, B, F, [&](int r, int q, float v) { m.A.a0[r * kFP + q] = bf16_bits(v); }, nrows);
  forward_fast(w.mlp_pk, reinterpret_cast<const float*>(w.mlp_pk + kPkHalf), m.A, xs, nrows);
}

// Evaluation counters of a wavefront's roots, added to its node's own
// counters (one address per node: a level's many merges do not serialise on
// a single atomic, which measured tens of microseconds per level).
__device__ inline void count_roots(const Work& w, int node, int N, int iters, int capped) {
  int it_sum = iters, cap_sum = capped;
  for (int off = 32; off > 0; off >>= 1) {
    it_sum += __shfl_xor(it_sum, off, 64);
    cap_sum += __shfl_xor(cap_sum, off, 64);
  }
  if ((threadIdx.x & 63) == 0 && it_sum) {
    atomicAdd(&w.sec[node].evals, (unsigned long long)it_sum);
    atomicAdd(&w.sec[node].terms, (unsigned long long)it_sum * (unsigned long long)N);
    if (cap_sum) atomicAdd(&w.sec[node].capped, (unsigned long long)cap_sum);
  }
}

// Start of the iteration: 0 the interval midpoint, 1 a caller-given position
// (w.xs), 2 the network's proposal computed here (w.mlp_pk).
//
// Secular roots of one node with more than sec_small_n kept values: 64 roots
// per workgroup, one per lane; the four wavefronts each sum a quarter of the
// poles for all 64 roots (staged in LDS, read by every lane at the same
// address), and wavefront 0 combines the partial sums -- left-pole sums in
// ascending quarter order, right-pole sums in descending order, so both stay
// summed from far to near -- and advances each root's iteration.
template <int kMode>
struct WideLds {
  SecLds<kMode> L;
  float s_x[kSecRoots];
  double part[kSecWaves][5][kSecRoots];
  double b_ov[kSecRoots], b_tau[kSecRoots];
  int b_need[kSecRoots];
  int b_go;
};

template <int kMode>
__device__ void secular_wide(const NodeDesc& nd, int N, const Work& w, WideLds<kMode>& S) {
  SecLds<kMode>& L = S.L;
  float* s_x = S.s_x;
  double (*part)[5][kSecRoots] = S.part;
  double* b_ov = S.b_ov;
  double* b_tau = S.b_tau;
  int* b_need = S.b_need;
  int& b_go = S.b_go;
  const double rho = w.st[nd.id].rho;
  const int64_t vo = nd.vec_off + nd.r0;
  const double* __restrict__ d = w.sd + vo;
  const double* __restrict__ z = w.sz + vo;
  const int maxit = w.max_secular_iters;
  // the network proposes the first points of merges of at least
  // learned_min_n kept values; smaller ones start at the midpoint (uniform
  // over the workgroup: one merge per workgroup)
  const bool net = kMode == 2 && N >= w.learned_min_n;
  const bool learned = kMode == 1 || net;
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
  double (*cd)[kSecChunk] = L.p.cd;
  double (*cz)[kSecChunk] = L.p.cz;
  // this wavefront's quarter of the poles
  const int Q = (N + kSecWaves - 1) / kSecWaves;
  const int q0 = min(N, wv * Q), q1 = min(N, q0 + Q);
  const bool resident = (q1 - q0) <= kSecChunk;  // the quarter fits in LDS once
  const bool run = (int)blockIdx.y * kSecRoots < N;

  if (kMode != 2 && resident && run) {
    for (int j = q0 + lane; j < q1; j += 64) {
      cd[wv][j - q0] = d[j];
      cz[wv][j - q0] = z[j] * z[j];
    }
  }
  for (int base = blockIdx.y * kSecRoots; base < N; base += gridDim.y * kSecRoots) {
    if constexpr (kMode == 2) {
      // the network's proposals for roots base .. base+63, then the poles
      __syncthreads();
      if (net) learned_proposals(w, L.m, d, z, N, rho, base, s_x, kRows);
      if (resident)
        for (int j = q0 + lane; j < q1; j += 64) {
          cd[wv][j - q0] = d[j];
          cz[wv][j - q0] = z[j] * z[j];
        }
    }
    const int i = base + lane;
    const bool active = i < N;
    Root R;
    const float xp = net ? s_x[lane] : (kMode == 1 && active ? w.xs[vo + i] : 0.0f);
    R.init(d, N, rho, N == 1 ? z[0] : 0.0, i, active, learned, xp);
    for (;;) {
      if (wv == 0) {
        b_ov[lane] = R.ov;
        b_tau[lane] = R.tau;
        b_need[lane] = R.need ? 1 : 0;
        const int any = __any(R.need) ? 1 : 0;
        if (lane == 0) b_go = any;
      }
      __syncthreads();
      if (!b_go) break;
      // ---- partial sums of this wavefront's quarter
      const bool nd_l = b_need[lane] != 0;
      const double eov = b_ov[lane], etau = b_tau[lane];
      const int lp = R.lp;
      Part PL{0.0, 0.0, 0.0}, PR{0.0, 0.0, 0.0};
      for (int c0 = q0; c0 < q1; c0 += kSecChunk) {
        const int c1 = min(q1, c0 + kSecChunk);
        if (!resident) {
          __builtin_amdgcn_wave_barrier();
          for (int j = c0 + lane; j < c1; j += 64) {
            cd[wv][j - c0] = d[j];
            cz[wv][j - c0] = z[j] * z[j];
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (nd_l) {
          // left poles j <= lp in this chunk, upwards
          const int le = min(c1, lp + 1);
          if (le > c0) sum_terms(cd[wv], cz[wv], 0, 1, le - c0, eov, etau, PL);
        }
      }
      for (int c1 = q1; c1 > q0; c1 -= kSecChunk) {
        const int c0 = max(q0, c1 - kSecChunk);
        if (!resident) {
          __builtin_amdgcn_wave_barrier();
          for (int j = c0 + lane; j < c1; j += 64) {
            cd[wv][j - c0] = d[j];
            cz[wv][j - c0] = z[j] * z[j];
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (nd_l) {
          // right poles j > lp in this chunk, downwards
          const int ls = max(c0, lp + 1);
          if (c1 > ls) sum_terms(cd[wv], cz[wv], c1 - 1 - c0, -1, c1 - ls, eov, etau, PR);
        }
      }
      part[wv][0][lane] = PL.s;
      part[wv][1][lane] = PL.ds;
      part[wv][2][lane] = PR.s;
      part[wv][3][lane] = PR.ds;
      part[wv][4][lane] = PL.E + PR.E;
      __syncthreads();
      if (wv == 0 && R.need) {
        double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0, E = 0.0;
        for (int q = 0; q < kSecWaves; ++q) {
          psi += part[q][0][lane];
          dpsi += part[q][1][lane];
          E += part[q][4][lane];
        }
        for (int q = kSecWaves - 1; q >= 0; --q) {
          phi += part[q][2][lane];
          dphi += part[q][3][lane];
        }
        const double f = (1.0 + psi) + phi;
        R.update(f, dpsi, dphi, 1.0 + E, rho, maxit, learned);
      }
      __syncthreads();
    }
    if (wv == 0) {
      if (active) {
        w.o[vo + i] = R.o;
        w.tau[vo + i] = R.tau;
        w.iters[vo + i] = R.iters;
      }
      count_roots(w, nd.id, N, R.iters, R.capped);
    }
    __syncthreads();
  }
}

// Secular roots of a node with at most kLanesMaxN kept values, L lanes per
// root (L = 8 or 16; 256/L roots per 256-thread workgroup).  Lane `part` of a
// root sums the poles j = part (mod L) in ascending order into left (j <= lp)
// and right sums, so every lane of a wavefront makes the same number of steps
// whatever its root's interval (the summation order inside a lane differs
// from the wide kernel's far-to-near order on the right side); the L partial sums are combined with DPP row
// permutations (no LDS, no barrier), and every lane of a root advances the
// same iteration state.  A wavefront holds 64/L roots, so it iterates only as
// long as the slowest of those few.
constexpr int kLanesMaxN = kSecLanesMaxN;
// The lanes-per-root kernel's network: at most 32 rows (its roots per
// workgroup) and, for N <= kLanesMaxN = 256, at most 16 far-field blocks.
struct SmallMlp {
  MlpSharedT<32, 16> m;
};

// v summed over the aligned group of L lanes (L in {8, 16}; within a DPP row)
template <int L>
__device__ inline double group_sum(double v) {
  static_assert(L == 8 || L == 16, "lanes per root");
  auto step = [](double x, auto ctrl) -> double {
    constexpr int c = decltype(ctrl)::value;
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), c, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), c, 0xF, 0xF, false);
    return x + __hiloint2double(hi, lo);
  };
  v = step(v, std::integral_constant<int, 0xB1>{});   // quad_perm [1,0,3,2]: lane ^ 1
  v = step(v, std::integral_constant<int, 0x4E>{});   // quad_perm [2,3,0,1]: lane ^ 2
  v = step(v, std::integral_constant<int, 0x141>{});  // row_half_mirror: the other quad of 8
  if constexpr (L == 16) v = step(v, std::integral_constant<int, 0x140>{});  // row_mirror
  return v;
}

template <int kMode, int L>
struct LanesLds {
  double cd[kLanesMaxN + L], cz[kLanesMaxN + L];
  float s_x[kSecRoots];
  typename std::conditional<kMode == 2, SmallMlp, char>::type M;
};

template <int kMode, int L>
__device__ void secular_lanes(const NodeDesc& nd, int N, const Work& w, LanesLds<kMode, L>& S) {
  constexpr int kRoots = 256 / L;
  double* cd = S.cd;
  double* cz = S.cz;
  float* s_x = S.s_x;
  auto& M = S.M;
  const int base = blockIdx.y * kRoots;
  if (base >= N) return;  // uniform over the workgroup
  const double rho = w.st[nd.id].rho;
  const int64_t vo = nd.vec_off + nd.r0;
  const double* __restrict__ d = w.sd + vo;
  const double* __restrict__ z = w.sz + vo;
  // the network proposes the first points of merges of at least
  // learned_min_n kept values; smaller ones start at the midpoint
  const bool net = kMode == 2 && N >= w.learned_min_n;
  const bool learned = kMode == 1 || net;
  const int t = threadIdx.x;
  // network proposals for the workgroup's own roots
  if constexpr (kMode == 2) {
    static_assert(kRoots % 16 == 0 && kRoots <= 32, "whole 16-row strips, at most SmallMlp's rows");
    static_assert(kLanesMaxN <= 16 * 16, "far_block(N) gives at most 16 blocks for N <= 256");
    if (N > 1 && net) learned_proposals(w, M.m, d, z, N, rho, base, s_x, kRoots);
  }
  // poles, padded to whole steps with far poles of weight 0 (their terms are
  // exact zeros: d^2 - omega^2 is about 2^1000, its reciprocal a normal number)
  const int steps = (N + L - 1) / L;
  for (int j = t; j < steps * L; j += 256) {
    cd[j] = j < N ? d[j] : 0x1p+500;
    cz[j] = j < N ? z[j] * z[j] : 0.0;
  }
  __syncthreads();
  const int part = t & (L - 1);
  const int i = base + t / L;
  const bool active = i < N;
  Root R;
  const float xp = net ? s_x[i - base] : (kMode == 1 && active ? w.xs[vo + i] : 0.0f);
  R.init(cd, N, rho, N == 1 ? z[0] : 0.0, i, active, learned, xp);
  while (R.need) {
    // left model poles j <= lp, right ones above (for the last root the
    // right side is the last pole alone, below the root like the others)
    double sL = 0.0, sR = 0.0, dL = 0.0, dR = 0.0;
    for (int q = 0; q < steps; ++q) {
      const int j = part + q * L;
      const double dd = cd[j];
      const double del = ((dd - R.ov) - R.tau) * ((dd + R.ov) + R.tau);  // d_j^2 - omega^2
      const double r = recip(del);
      const double tj = cz[j] * r;
      const double tl = j <= R.lp ? tj : 0.0, tg = tj - tl;  // exact split
      sL += tl;
      sR += tg;
      dL = fma(tl, r, dL);
      dR = fma(tg, r, dR);
    }
    sL = group_sum<L>(sL);
    sR = group_sum<L>(sR);
    dL = group_sum<L>(dL);
    dR = group_sum<L>(dR);
    // left terms are negative and right ones positive (the last root's one
    // right term is negative too): sum |t| = |sR| - sL
    const double f = (1.0 + sL) + sR;
    R.update(f, dL, dR, 1.0 + (fabs(sR) - sL), rho, w.max_secular_iters, learned);
  }
  const bool writer = active && part == 0;
  if (writer) {
    w.o[vo + i] = R.o;
    w.tau[vo + i] = R.tau;
    w.iters[vo + i] = R.iters;
  }
  count_roots(w, nd.id, N, writer ? R.iters : 0, writer ? R.capped : 0);
}

// One launch per level: a node with at most sec_small_n (<= kLanesMaxN) kept
// values is solved by the lanes-per-root body, a larger one by the wide body;
// the two share the workgroup's LDS.
template <int kMode, int L>
__global__ __launch_bounds__(256) void k_secular(const NodeDesc* __restrict__ nodes, Work w) {
  __shared__ union {
    WideLds<kMode> wide;
    LanesLds<kMode, L> lanes;
  } S;
  const NodeDesc nd = nodes[blockIdx.x];
  const int N = w.st[nd.id].N;
  if (N <= w.sec_small_n && N <= kLanesMaxN) secular_lanes<kMode, L>(nd, N, w, S.lanes);
  else secular_wide<kMode>(nd, N, w, S.wide);
}

// Levels whose merges all take the lanes-per-root body (every merge at most
// sec_small_n <= kLanesMaxN values): the LDS of that body alone, so more
// workgroups fit on a CU.
template <int kMode, int L>
__global__ __launch_bounds__(256) void k_secular_lanes(const NodeDesc* __restrict__ nodes, Work w) {
  __shared__ LanesLds<kMode, L> S;
  const NodeDesc nd = nodes[blockIdx.x];
  secular_lanes<kMode, L>(nd, w.st[nd.id].N, w, S);
}

__global__ __launch_bounds__(256) void k_lowner(const NodeDesc* __restrict__ nodes, Work w) {
  const NodeDesc nd = nodes[blockIdx.x];
  const int N = w.st[nd.id].N;
  const int64_t vo = nd.vec_off + nd.r0;
  const double* __restrict__ d = w.sd + vo;
  const double* __restrict__ z = w.sz + vo;
  const int* __restrict__ o = w.o + vo;
  const double* __restrict__ tau = w.tau + vo;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int base = blockIdx.y * 4; base < N; base += gridDim.y * 4) {
    const int i = base + wv;
    if (i >= N) continue;  // the whole wavefront
    const double di = d[i];
    double prod = 1.0;
    for (int kk = lane; kk < N; kk += 64) {
      const double ok = d[o[kk]], tk = tau[kk];
      const double num = ((ok - di) + tk) * ((ok + di) + tk);  // w_k^2 - d_i^2
      double f = num;
      if (kk != N - 1) {
        const double pole = kk < i ? d[kk] : d[kk + 1];
        f = num / ((pole - di) * (pole + di));
      }
      prod *= f;
    }
    prod = wave_prod(prod);
    if (lane == 0) w.zt[vo + i] = copysign(sqrt(prod), z[i]);
  }
}

// One wavefront per root column, four per workgroup: lane l takes rows
// g = l, l + 64, ...; the first 256 rows stay in registers between the sums
// of squares (wavefront reductions, no barrier) and the scaled stores,
// longer columns are written once and rescaled in place.  Merges of at most
// 64 kept values take two columns per wavefront.
__global__ __launch_bounds__(256) void k_vectors(const NodeDesc* __restrict__ nodes, Work w) {
  const NodeDesc nd = nodes[blockIdx.x];
  const int N = w.st[nd.id].N;
  const int64_t vo = nd.vec_off + nd.r0;
  const int64_t ld = nd.ld;
  const double* __restrict__ d = w.sd + vo;
  const double* __restrict__ zt = w.zt + vo;
  const int* __restrict__ gsurv = w.gsurv + vo;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (N > 1 && N <= 64) {
    // one row per lane: two columns per wavefront (i and i + S), their rows'
    // d and z~ read once and both columns' loads in flight together; each
    // column's arithmetic is the general path's
    const int S = gridDim.y * 4;
    const bool act = lane < N;
    int j = 0;
    double dj = 0.0, zj = 0.0;
    if (act) {
      j = gsurv[lane];
      dj = d[j];
      zj = zt[j];
    }
    for (int i = blockIdx.y * 4 + wv; i < N; i += 2 * S) {
      const int i2 = i + S;
      const bool has2 = i2 < N;
      const double ov1 = d[w.o[vo + i]], t1 = w.tau[vo + i];
      const double ov2 = has2 ? d[w.o[vo + i2]] : 0.0, t2 = has2 ? w.tau[vo + i2] : 0.0;
      double v1 = 0.0, u1 = 0.0, v2 = 0.0, u2 = 0.0;
      if (act) {
        v1 = zj / (((dj - ov1) - t1) * ((dj + ov1) + t1));  // z~_j / (d_j^2 - w_i^2)
        u1 = (j == 0) ? -1.0 : dj * v1;
        if (has2) {
          v2 = zj / (((dj - ov2) - t2) * ((dj + ov2) + t2));
          u2 = (j == 0) ? -1.0 : dj * v2;
        }
      }
      const double rv1 = 1.0 / sqrt(wave_sum(v1 * v1)), ru1 = 1.0 / sqrt(wave_sum(u1 * u1));
      const double rv2 = 1.0 / sqrt(wave_sum(v2 * v2)), ru2 = 1.0 / sqrt(wave_sum(u2 * u2));
      if (act) {
        const int64_t c1 = nd.mat_off + nd.r0 + (int64_t)(nd.r0 + i) * ld;
        w.VM[c1 + lane] = v1 * rv1;
        w.UM[c1 + lane] = u1 * ru1;
        if (has2) {
          const int64_t c2 = nd.mat_off + nd.r0 + (int64_t)(nd.r0 + i2) * ld;
          w.VM[c2 + lane] = v2 * rv2;
          w.UM[c2 + lane] = u2 * ru2;
        }
      }
    }
    return;
  }
  for (int i = blockIdx.y * 4 + wv; i < N; i += gridDim.y * 4) {
    double* ucol = w.UM + nd.mat_off + nd.r0 + (int64_t)(nd.r0 + i) * ld;
    double* vcol = w.VM + nd.mat_off + nd.r0 + (int64_t)(nd.r0 + i) * ld;
    if (N == 1) {
      // M~ = [zt_1], omega = |zt_1|: u = [-1], v = zt/(0 - omega^2) normalised = [-1]
      if (lane == 0) {
        ucol[0] = -1.0;
        vcol[0] = -1.0;
      }
      continue;
    }
    const double ov = d[w.o[vo + i]], ti = w.tau[vo + i];
    auto entry = [&](int g, double& v, double& u) {
      const int j = gsurv[g];
      const double dj = d[j];
      const double del = ((dj - ov) - ti) * ((dj + ov) + ti);  // d_j^2 - w_i^2
      v = zt[j] / del;
      u = (j == 0) ? -1.0 : dj * v;
    };
    double su = 0.0, sv = 0.0;
    double vr[4], ur[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int g = lane + 64 * q;
      vr[q] = ur[q] = 0.0;
      if (g < N) entry(g, vr[q], ur[q]);
      sv += vr[q] * vr[q];
      su += ur[q] * ur[q];
    }
    for (int g = lane + 256; g < N; g += 64) {
      double v, u;
      entry(g, v, u);
      vcol[g] = v;
      ucol[g] = u;
      sv += v * v;
      su += u * u;
    }
    const double rv = 1.0 / sqrt(wave_sum(sv)), ru = 1.0 / sqrt(wave_sum(su));
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int g = lane + 64 * q;
      if (g < N) {
        vcol[g] = vr[q] * rv;
        ucol[g] = ur[q] * ru;
      }
    }
    for (int g = lane + 256; g < N; g += 64) {
      vcol[g] *= rv;
      ucol[g] *= ru;
    }
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

}  // namespace

void launch_secular(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, hipStream_t st) {
  if (nnodes <= 0) return;
  // 8 lanes per root while the merges are at most 64 values, else 16
  const bool l8 = max_m <= 64;
  const int small_max = std::min(std::min(w.sec_small_n, kLanesMaxN), max_m);
  const int ys = (small_max + (l8 ? 32 : 16) - 1) / (l8 ? 32 : 16);
  const int yw = max_m > small_max ? (max_m + kSecRoots - 1) / kSecRoots : 0;
  const int gy = grid_y(nnodes, std::max(ys, yw), 4096 + nnodes * ys);
  const dim3 grid(nnodes, gy), block(256);
  const int mode = w.mlp_pk ? 2 : (w.xs ? 1 : 0);
  const bool lanes_only = max_m <= small_max;  // every merge has N <= max_m <= small_max
#define BDC_LAUNCH_SEC(M)                                                                        \
  do {                                                                                           \
    if (lanes_only && l8) hipLaunchKernelGGL((k_secular_lanes<M, 8>), grid, block, 0, st, nodes, w); \
    else if (lanes_only) hipLaunchKernelGGL((k_secular_lanes<M, 16>), grid, block, 0, st, nodes, w); \
    else if (l8) hipLaunchKernelGGL((k_secular<M, 8>), grid, block, 0, st, nodes, w);            \
    else hipLaunchKernelGGL((k_secular<M, 16>), grid, block, 0, st, nodes, w);                   \
  } while (0)
  if (mode == 2) BDC_LAUNCH_SEC(2);
  else if (mode == 1) BDC_LAUNCH_SEC(1);
  else BDC_LAUNCH_SEC(0);
#undef BDC_LAUNCH_SEC
}

void launch_lowner(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, hipStream_t st) {
  if (nnodes <= 0) return;
  const int gy = grid_y(nnodes, (max_m + 3) / 4, 4096);
  hipLaunchKernelGGL(k_lowner, dim3(nnodes, gy), dim3(256), 0, st, nodes, w);
}

void launch_vectors(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, hipStream_t st) {
  if (nnodes <= 0) return;
  // merges of at most 64 values: two columns per wavefront
  const int gy = grid_y(nnodes, max_m <= 64 ? (max_m + 7) / 8 : (max_m + 3) / 4, 4096);
  hipLaunchKernelGGL(k_vectors, dim3(nnodes, gy), dim3(kBlock), 0, st, nodes, w);
}

}  // namespace bdc
