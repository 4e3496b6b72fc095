// Merge stage after deflation (Algorithm 4, the GPU-based lasd3), entirely
// on the GPU:
//   k_secular  roots of the secular equation (eq. M-svd-val), one lane per
//              root.  The paper solves them on CPU threads with LAPACK's
//              lasd4; here each root is bracketed, its origin pole chosen by
//              the sign of f at the interval midpoint (in omega^2), and the
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
//   k_vectors  singular vectors of M~ (eq. M-svd-vec), one workgroup per root
//              column, written in the row order of the vector update and
//              normalised in place.
#include "bdc_internal.h"
#include "block_util.h"

namespace bdc {
namespace {

constexpr double kEps = 0x1p-52;

struct Eval {
  double f, dpsi, dphi, E;
};

// f(omega) and the pieces of the rational model at omega = ov + tau; poles
// 0..lp form psi, lp+1..N-1 form phi.
__device__ inline Eval evaluate(const double* __restrict__ d, const double* __restrict__ z, int N,
                                double ov, double tau, int lp) {
  double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0, E = 0.0;
  for (int j = 0; j <= lp; ++j) {
    const double dj = d[j], zj = z[j];
    const double del = ((dj - ov) - tau) * ((dj + ov) + tau);
    const double r = 1.0 / del;
    const double tt = (zj * zj) * r;
    psi += tt;
    dpsi += tt * r;
    E += fabs(tt);
  }
  for (int j = N - 1; j > lp; --j) {
    const double dj = d[j], zj = z[j];
    const double del = ((dj - ov) - tau) * ((dj + ov) + tau);
    const double r = 1.0 / del;
    const double tt = (zj * zj) * r;
    phi += tt;
    dphi += tt * r;
    E += fabs(tt);
  }
  Eval ev;
  ev.f = (1.0 + psi) + phi;
  ev.dpsi = dpsi;
  ev.dphi = dphi;
  ev.E = 1.0 + E;
  return ev;
}

__global__ __launch_bounds__(64) void k_secular(const NodeDesc* __restrict__ nodes, Work w) {
  const NodeDesc nd = nodes[blockIdx.x];
  const int N = w.st[nd.id].N;
  const double rho = w.st[nd.id].rho;
  const int64_t vo = nd.vec_off + nd.r0;
  const double* __restrict__ d = w.sd + vo;
  const double* __restrict__ z = w.sz + vo;
  const int maxit = w.max_secular_iters;

  for (int base = blockIdx.y * 64; base < N; base += gridDim.y * 64) {
    const int i = base + threadIdx.x;
    const bool active = i < N;
    int o = 0, iters = 0, capped = 0;
    double tau = 0.0;
    if (active && N == 1) {
      tau = fabs(z[0]);  // f = 1 - z^2/omega^2: omega = |z| exactly
    } else if (active) {
      const bool last = (i == N - 1);
      const int lp = last ? N - 2 : i;  // left model pole
      const int rp = lp + 1;            // right model pole
      const double dl = d[lp], dr = d[rp];
      // first evaluation: the midpoint in omega^2 of the root's interval
      const double base_v = last ? dr : dl;
      const double mu = last ? 0.5 * rho : 0.5 * (dr - dl) * (dr + dl);
      const double tmid = mu / (base_v + sqrt(base_v * base_v + mu));
      Eval ev = evaluate(d, z, N, base_v, tmid, lp);
      iters = 1;
      const bool go_right = !last && ev.f < 0.0;
      o = (last || go_right) ? rp : lp;
      const double ov = d[o];
      const double wmid = base_v + tmid;
      tau = go_right ? -mu / (dr + wmid) : tmid;
      double lo, hi;
      if (last) {
        lo = 0.0;
        hi = rho / (dr + sqrt(dr * dr + rho));
        if (ev.f < 0.0) lo = tau;
        else hi = tau;
      } else if (go_right) {
        lo = tau;
        hi = 0.0;
      } else {
        lo = 0.0;
        hi = tau;
      }
      bool done = fabs(ev.f) <= 8.0 * kEps * ev.E;
      while (!done) {
        // two-pole model at the current point (pole differences in omega^2)
        const double Dl = ((dl - ov) - tau) * ((dl + ov) + tau);
        const double Dr = ((dr - ov) - tau) * ((dr + ov) + tau);
        const double f = ev.f;
        const double c = f - Dl * ev.dpsi - Dr * ev.dphi;
        const double a = (Dl + Dr) * f - Dl * Dr * (ev.dpsi + ev.dphi);
        const double b = Dl * Dr * f;
        const double disc = sqrt(fabs(a * a - 4.0 * b * c));
        double eta;
        if (c == 0.0) eta = b / a;
        else if (last) eta = (a >= 0.0) ? (a + disc) / (2.0 * c) : 2.0 * b / (a - disc);
        else eta = (a <= 0.0) ? (a - disc) / (2.0 * c) : 2.0 * b / (a + disc);
        // omega^2 step eta -> tau step
        const double om = ov + tau;
        const double omn = sqrt(om * om + eta);
        double tn = tau + eta / (om + omn);
        if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        const bool small_step = fabs(tn - tau) <= 2.0 * kEps * fabs(tn);
        tau = tn;
        ev = evaluate(d, z, N, ov, tau, lp);
        ++iters;
        if (ev.f < 0.0) lo = tau;
        else hi = tau;
        const bool conv = fabs(ev.f) <= 8.0 * kEps * ev.E;
        if (!conv && !small_step && iters >= maxit) capped = 1;
        done = conv || small_step || iters >= maxit;
      }
    }
    if (active) {
      w.o[vo + i] = o;
      w.tau[vo + i] = tau;
      w.iters[vo + i] = iters;
    }
    // counters: one atomic per wavefront
    int it_sum = iters, cap_sum = capped;
    for (int off = 32; off > 0; off >>= 1) {
      it_sum += __shfl_xor(it_sum, off, 64);
      cap_sum += __shfl_xor(cap_sum, off, 64);
    }
    if (threadIdx.x == 0) {
      atomicAdd(&w.ctl->secular_evals, (unsigned long long)it_sum);
      atomicAdd(&w.ctl->secular_terms, (unsigned long long)it_sum * (unsigned long long)N);
      if (cap_sum) atomicAdd(&w.ctl->secular_capped, cap_sum);
    }
  }
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

__global__ __launch_bounds__(256) void k_vectors(const NodeDesc* __restrict__ nodes, Work w) {
  __shared__ double sh[8];
  const NodeDesc nd = nodes[blockIdx.x];
  const int N = w.st[nd.id].N;
  const int64_t vo = nd.vec_off + nd.r0;
  const int64_t ld = nd.ld;
  const double* __restrict__ d = w.sd + vo;
  const double* __restrict__ zt = w.zt + vo;
  const int* __restrict__ gsurv = w.gsurv + vo;
  const int t = threadIdx.x;
  for (int i = blockIdx.y; i < N; i += gridDim.y) {
    double* ucol = w.UM + nd.mat_off + nd.r0 + (int64_t)(nd.r0 + i) * ld;
    double* vcol = w.VM + nd.mat_off + nd.r0 + (int64_t)(nd.r0 + i) * ld;
    if (N == 1) {
      // M~ = [zt_1], omega = |zt_1|: u = [-1], v = zt/(0 - omega^2) normalised = [-1]
      if (t == 0) {
        ucol[0] = -1.0;
        vcol[0] = -1.0;
      }
      continue;
    }
    const double ov = d[w.o[vo + i]], ti = w.tau[vo + i];
    double su = 0.0, sv = 0.0;
    for (int g = t; g < N; g += kBlock) {
      const int j = gsurv[g];
      const double dj = d[j];
      const double del = ((dj - ov) - ti) * ((dj + ov) + ti);  // d_j^2 - w_i^2
      const double v = zt[j] / del;
      const double u = (j == 0) ? -1.0 : dj * v;
      vcol[g] = v;
      ucol[g] = u;
      sv += v * v;
      su += u * u;
    }
    const double nv = sqrt(block_sum(sv, sh));
    const double nu = sqrt(block_sum(su, sh + 4));
    for (int g = t; g < N; g += kBlock) {
      vcol[g] = vcol[g] / nv;
      ucol[g] = ucol[g] / nu;
    }
    __syncthreads();
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
  const int gy = grid_y(nnodes, (max_m + 63) / 64, 8192);
  hipLaunchKernelGGL(k_secular, dim3(nnodes, gy), dim3(64), 0, st, nodes, w);
}

void launch_lowner(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, hipStream_t st) {
  if (nnodes <= 0) return;
  const int gy = grid_y(nnodes, (max_m + 3) / 4, 4096);
  hipLaunchKernelGGL(k_lowner, dim3(nnodes, gy), dim3(256), 0, st, nodes, w);
}

void launch_vectors(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, hipStream_t st) {
  if (nnodes <= 0) return;
  const int gy = grid_y(nnodes, max_m, 4096);
  hipLaunchKernelGGL(k_vectors, dim3(nnodes, gy), dim3(kBlock), 0, st, nodes, w);
}

}  // namespace bdc
