// Device pieces of the learned secular start shared by the training kernels
// and the secular solver: bfloat16 rounding, the activation, the 19 features
// of a root, and the inference pass of the 19 -> 64 -> 64 -> 64 -> 1 network
// on the bfloat16 matrix cores (v_mfma_f32_16x16x16_bf16, FP32 accumulation).
//
// Features (FP64 arithmetic, FP32 results), for root i of a secular problem
// with kept values 0 = d_0 < ... < d_{N-1}, z and rho = sum z^2: the interval
// (lo, hi) with width h and w2 = hi^2 - lo^2 (interior: lo = d_i,
// hi = d_{i+1}, w2 = h (hi + lo); last: lo = d_{N-1}, hi = sqrt(lo^2 + rho),
// h = rho / (lo + hi), w2 = rho); for the 4 poles j <= i and the 4 poles
// j > i the gap (d_j - lo)/h (clamped to >= -4 and <= 5) and the strength
// log2(z_j^2 / w2)/32 (clamped to [-2, 2]); a missing pole has gap -4 or 5
// and strength -2; feature 16 is log2(rho / w2)/32 clamped to [-2, 2].
// Features 17 and 18 describe the far field (f without those 8 poles) at the
// interval's midpoint lam = lo^2 + w2/2: asinh(v)/8 and asinh(s w2)/8
// (clamped to [-4, 4]) with v = 1 + sum z_j^2/(d_j^2 - lam) and s = sum
// z_j^2/(d_j^2 - lam)^2 over the far poles.  The sum takes O(sqrt N) terms:
// poles are cut into blocks of B (least power of two >= 4 with B^2 >= N and
// 512 B >= N); a block that holds one of the root's 8 poles is summed term by
// term in ascending order, every other block contributes one monopole term
// Z_k/(D_k - lam) (Z_k = sum z_j^2, D_k = sum z_j^2 d_j^2 / Z_k, ascending).
// Four threads share a root's far field, each summing every fourth block;
// their partial sums are added in thread order.
#pragma once

#include "bdc_internal.h"

namespace bdc {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kRows = 64;  // rows (roots) per workgroup
constexpr int kF = 19;     // features
constexpr int kFP = 32;    // features padded to two k-steps of 16
constexpr int kH = 64;     // hidden width
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kF * kH, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH,
              kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kH * kH, kOffW4 = kOffB3 + kH, kOffB4 = kOffW4 + kH,
              kParams = kOffB4 + 1;
static_assert(kParams == BDC_MLP_PARAMS, "parameter layout");

// float -> bfloat16 bits, round to nearest, ties to even
__device__ inline unsigned short bf16_bits(float x) {
  unsigned int u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float bf16_val(unsigned short b) { return __uint_as_float(((unsigned int)b) << 16); }

constexpr float kGc = 0.7978845608028654f;  // sqrt(2/pi)
constexpr float kGa = 0.044715f;
__device__ inline float gelu_f(float x) { return 0.5f * x * (1.0f + tanhf(kGc * (x + kGa * x * x * x))); }
__device__ inline float gelu_d(float x) {
  const float t = tanhf(kGc * (x + kGa * x * x * x));
  return 0.5f * (1.0f + t) + 0.5f * x * (1.0f - t * t) * kGc * (1.0f + 3.0f * kGa * x * x);
}
__device__ inline float logistic(float v) { return 1.0f / (1.0f + expf(-v)); }

// ---------------------------------------------------------------- features
__device__ inline float clampd(double v, double lo, double hi) { return (float)fmin(fmax(v, lo), hi); }

__device__ inline float strength(double zj, double w2) {
  const double c = (zj * zj) / w2;
  if (c == 0.0) return -2.0f;
  if (isinf(c)) return 2.0f;
  return clampd(log2(c) / 32.0, -2.0, 2.0);
}

__device__ inline float asinh8(double x) { return (float)fmin(fmax(asinh(x) / 8.0, -4.0), 4.0); }

constexpr int kMaxBlocks = 512;  // far-field blocks (B is chosen so that nb <= 512)

__device__ inline int far_block(int N) {
  int B = 4;
  while ((int64_t)B * B < N || 512 * (int64_t)B < N) B *= 2;
  return B;
}

// Feature scratch for at most MB far-field blocks and R rows.
template <int MB, int R>
struct FeatLdsT {
  static constexpr int kBlocks = MB;
  double Z[MB];
  double D[MB];
  double pv[4][R];
  double ps[4][R];
};
using FeatLds = FeatLdsT<kMaxBlocks, kRows>;

// Block moments Z_k, D_k by the whole workgroup (call, then synchronise).
template <class FL>
__device__ void far_moments(const double* __restrict__ d, const double* __restrict__ z, int N, int B, FL& F) {
  const int nb = (N + B - 1) / B;
  for (int k = threadIdx.x; k < nb; k += blockDim.x) {
    double zs = 0.0, ms = 0.0;
    const int j1 = min(N, (k + 1) * B);
    for (int j = k * B; j < j1; ++j) {
      const double zz = z[j] * z[j];
      zs += zz;
      ms += zz * (d[j] * d[j]);
    }
    F.Z[k] = zs;
    F.D[k] = zs > 0.0 ? ms / zs : 0.0;
  }
}

__device__ inline void interval_of(const double* __restrict__ d, int N, double rho, int i, double& lo, double& h,
                                   double& w2) {
  lo = d[i];
  if (i < N - 1) {
    const double hi = d[i + 1];
    h = hi - lo;
    w2 = h * (hi + lo);
  } else {
    const double hi = sqrt(lo * lo + rho);
    h = rho / (lo + hi);
    w2 = rho;
  }
}

// Features of roots base .. base+nrows-1 (nrows <= 64) by the whole
// workgroup (moments already in F).  Row r's features go to out(r, q, value)
// for roots < N.  The far-field sums are work items (row, quarter), each
// summed in block order; the features are work items (row, pole or far
// field), so a workgroup of 256 threads spreads the transcendental functions
// over its lanes.  The values do not depend on how items fall on threads.
template <class FL, class Out>
__device__ void block_features(const double* __restrict__ d, const double* __restrict__ z, int N, double rho,
                               int base, int B, FL& F, Out out, int nrows = kRows) {
  const int nb = (N + B - 1) / B;
  for (int item = threadIdx.x; item < 4 * nrows; item += blockDim.x) {
    const int r = item % nrows, part = item / nrows, i = base + r;
    double v = 0.0, sl = 0.0;
    if (i < N) {
      double lo, h, w2;
      interval_of(d, N, rho, i, lo, h, w2);
      const double lam = lo * lo + 0.5 * w2;
      for (int k = part; k < nb; k += 4) {
        const int j0 = k * B, j1 = min(N, (k + 1) * B);
        if (j1 > i - 3 && j0 <= i + 4) {
          for (int j = j0; j < j1; ++j) {
            if (j >= i - 3 && j <= i + 4) continue;
            const double den = d[j] * d[j] - lam;
            const double t = (z[j] * z[j]) / den;
            v += t;
            sl += t / den;
          }
        } else if (F.Z[k] > 0.0) {
          const double den = F.D[k] - lam;
          const double t = F.Z[k] / den;
          v += t;
          sl += t / den;
        }
      }
    }
    F.pv[part][r] = v;
    F.ps[part][r] = sl;
  }
  __syncthreads();
  // items: 0..3 the poles j = i - q, 4..7 the poles j = i + 1 + (q - 4),
  // 8 feature 16, 9 features 17 and 18
  for (int item = threadIdx.x; item < 10 * nrows; item += blockDim.x) {
    const int r = item % nrows, task = item / nrows, i = base + r;
    if (i >= N) continue;
    double lo, h, w2;
    interval_of(d, N, rho, i, lo, h, w2);
    if (task < 4) {
      const int q = task, j = i - q;
      if (j >= 0) {
        out(r, 2 * q, (float)fmax((d[j] - lo) / h, -4.0));
        out(r, 2 * q + 1, strength(z[j], w2));
      } else {
        out(r, 2 * q, -4.0f);
        out(r, 2 * q + 1, -2.0f);
      }
    } else if (task < 8) {
      const int q = task - 4, j = i + 1 + q;
      if (j < N) {
        out(r, 8 + 2 * q, (float)fmin((d[j] - lo) / h, 5.0));
        out(r, 9 + 2 * q, strength(z[j], w2));
      } else {
        out(r, 8 + 2 * q, 5.0f);
        out(r, 9 + 2 * q, -2.0f);
      }
    } else if (task == 8) {
      out(r, 16, clampd(log2(rho / w2) / 32.0, -2.0, 2.0));
    } else {
      const double vv = 1.0 + (((F.pv[0][r] + F.pv[1][r]) + F.pv[2][r]) + F.pv[3][r]);
      const double ss = ((F.ps[0][r] + F.ps[1][r]) + F.ps[2][r]) + F.ps[3][r];
      out(r, 17, asinh8(vv));
      out(r, 18, asinh8(ss * w2));
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------- inference
// Parameters packed once per solve for inference: weights as bfloat16,
// transposed (output-major, input contiguous), the 64 -> 1 layer as column 0
// of a 64 x 16 block, then the FP32 biases.
constexpr int kPkW1 = 0;                  // 64 x 32 (inputs 19..31 zero)
constexpr int kPkW2 = kPkW1 + kH * kFP;   // 64 x 64
constexpr int kPkW3 = kPkW2 + kH * kH;    // 64 x 64
constexpr int kPkW4 = kPkW3 + kH * kH;    // 16 x 64 (row 0 = w4, rest zero)
constexpr int kPkHalf = kPkW4 + 16 * kH;  // bfloat16 entries
constexpr int kPkBias = 3 * kH + 1;       // b1, b2, b3, b4 (FP32)
constexpr size_t kPackBytes = (size_t)kPkHalf * 2 + (size_t)kPkBias * 4;

// Activations of R rows (bfloat16 bits)
template <int R>
struct FastActT {
  static constexpr int kR = R;
  unsigned short a0[R * kFP];
  unsigned short a1[R * kH];
  unsigned short a2[R * kH];
};
using FastAct = FastActT<kRows>;


// acc[nt] += A(16 rows from r0, K) * Bt(64 cols, K)^T with A row-major (lda)
// and Bt output-major (ldb), both bfloat16: one 8-byte read per operand.
__device__ inline void mm_fast(const unsigned short* A, int lda, const unsigned short* Bt, int ldb, int r0, int K,
                               int ntiles, f32x4* acc) {
  const int lane = threadIdx.x & 63;
  const int rr = lane & 15, kq = (lane >> 4) * 4;
  for (int k0 = 0; k0 < K; k0 += 16) {
    const bf16x4 a = *(const bf16x4*)(A + (r0 + rr) * lda + k0 + kq);
    for (int nt = 0; nt < ntiles; ++nt) {
      const bf16x4 b = *(const bf16x4*)(Bt + (nt * 16 + rr) * ldb + k0 + kq);
      acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[nt], 0, 0, 0);
    }
  }
}

// Inference of nrows rows (a multiple of 16, at most 64; inputs in A.a0):
// the proposed positions in xout[0 .. nrows).  a1 and a2 alternate as the
// hidden activations (layer 3 writes a1 again).  A layer's work items are
// (16-row strip, 16-column tile) pairs dealt to the wavefronts; each output
// element's sum runs over K in the same k-steps whatever the split.
// wts / bias: the packed bfloat16 weights and FP32 biases (global memory,
// read by the MFMA operand loads directly: every workgroup shares them in
// the caches, so no workgroup stages them).
template <class Act>
__device__ void forward_fast(const unsigned short* __restrict__ wts, const float* __restrict__ bias, Act& A,
                             float* xout, int nrows = Act::kR) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  const int strips = nrows / 16;
  for (int l = 0; l < 3; ++l) {
    const unsigned short* in = l == 0 ? A.a0 : (l == 1 ? A.a1 : A.a2);
    unsigned short* outl = l == 1 ? A.a2 : A.a1;
    const unsigned short* wt = wts + (l == 0 ? kPkW1 : (l == 1 ? kPkW2 : kPkW3));
    const float* bl = bias + l * kH;
    const int K = l == 0 ? kFP : kH;
    for (int item = wv; item < 4 * strips; item += nw) {
      const int r0 = (item >> 2) * 16, nt = item & 3;
      f32x4 acc[1] = {f32x4{0.f, 0.f, 0.f, 0.f}};
      mm_fast(in, K, wt + nt * 16 * K, K, r0, K, 1, acc);
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + 4 * (lane >> 4) + r, col = nt * 16 + (lane & 15);
        outl[row * kH + col] = bf16_bits(gelu_f(acc[0][r] + bl[col]));
      }
    }
    __syncthreads();
  }
  // 64 -> 1 as column 0 of a 16-wide product
  for (int strip = wv; strip < strips; strip += nw) {
    const int r0 = strip * 16;
    f32x4 acc[1] = {f32x4{0.f, 0.f, 0.f, 0.f}};
    mm_fast(A.a1, kH, wts + kPkW4, kH, r0, kH, 1, acc);
    if ((lane & 15) == 0)
      for (int r = 0; r < 4; ++r) xout[r0 + 4 * (lane >> 4) + r] = logistic(acc[0][r] + bias[3 * kH]);
  }
  __syncthreads();
}

}  // namespace
}  // namespace bdc
