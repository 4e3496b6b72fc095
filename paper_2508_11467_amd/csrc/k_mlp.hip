// Learned start of the secular iteration: a 19 -> 64 -> 64 -> 64 -> 1 MLP
// proposes each root's fractional position in its interval.
//
//   k_start    inside a solve, per merge level: the features of 64 roots per
//              workgroup (from the kept values, z and rho of the merge),
//              the forward pass, and the proposals written for k_secular
//   k_harvest  after k_secular: features, the computed root's position and a
//              (merge, root) tag appended to caller buffers, as training data
//   k_features the features of one secular problem (d, z) given directly
//   k_mlp      forward (and with kGrad the backward pass) of 64 rows per
//              workgroup for caller-provided feature rows; per-workgroup
//              weight gradients go to a partial buffer
//   k_adam     sums the partial gradients in workgroup order, and optionally
//              takes one Adam step on the FP32 parameters
//
// Arithmetic.  The three hidden-layer products run on the matrix cores with
// bfloat16 operands and FP32 accumulation (v_mfma_f32_16x16x16_bf16): inputs,
// weights and hidden activations are rounded to bfloat16 (nearest, ties to
// even) where they enter a product, and in the backward pass so are the
// back-propagated gradients.  Biases, GELU (tanh form), the logistic output,
// the 64 -> 1 layer (a dot product per row on the vector units) and every
// bias gradient stay in FP32.  The parameters are kept in FP32 (one flat
// vector: W1 19x64, b1, W2 64x64, b2, W3 64x64, b3, W4 64, b4; W row-major
// in x out) and rounded when staged in LDS.
//
// Features (FP64, then FP32), for root i of a merge with kept values
// 0 = d_0 < ... < d_{N-1}, z and rho = sum z^2: the interval (lo, hi) with
// width h and w2 = hi^2 - lo^2 (interior: lo = d_i, hi = d_{i+1},
// w2 = h (hi + lo); last: lo = d_{N-1}, hi = sqrt(lo^2 + rho),
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
#include "bdc_internal.h"
#include "block_util.h"

namespace bdc {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kRows = 64;     // rows (roots) per workgroup
constexpr int kF = 19;        // features
constexpr int kFP = 32;       // features padded to two k-steps of 16
constexpr int kH = 64;        // hidden width
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

// Weights of the network staged in LDS (bfloat16 bits; biases FP32).
struct MlpLds {
  unsigned short w1[kFP * kH];  // rows 19..31 zero
  unsigned short w2[kH * kH];
  unsigned short w3[kH * kH];
  unsigned short w4[kH];
  float b1[kH], b2[kH], b3[kH];
  float b4;
};

__device__ void stage_weights(const float* __restrict__ p, MlpLds& L) {
  const int t = threadIdx.x;
  for (int q = t; q < kFP * kH; q += blockDim.x) L.w1[q] = q < kF * kH ? bf16_bits(p[kOffW1 + q]) : 0;
  for (int q = t; q < kH * kH; q += blockDim.x) {
    L.w2[q] = bf16_bits(p[kOffW2 + q]);
    L.w3[q] = bf16_bits(p[kOffW3 + q]);
  }
  for (int q = t; q < kH; q += blockDim.x) {
    L.w4[q] = bf16_bits(p[kOffW4 + q]);
    L.b1[q] = p[kOffB1 + q];
    L.b2[q] = p[kOffB2 + q];
    L.b3[q] = p[kOffB3 + q];
  }
  if (t == 0) L.b4 = p[kOffB4];
}

// One 16-row strip of a product with a 64-column output on the matrix cores:
// acc[nt] (columns nt*16 .. nt*16+15) += sum_k A(r0 + row, k) B(k, col), K a
// multiple of 16.  Operand element (row, k): lane = row + 16 * (k / 4 within
// the step), 4 consecutive k per lane.  Output: lane l, register r holds
// row 4 (l / 16) + r, column l % 16 of the tile.
template <class FA, class FB>
__device__ inline void mm_strip(FA A, FB B, int r0, int K, f32x4 acc[4]) {
  const int lane = threadIdx.x & 63;
  const int rr = lane & 15, kq = (lane >> 4) * 4;
  for (int k0 = 0; k0 < K; k0 += 16) {
    bf16x4 a;
    a[0] = (short)A(r0 + rr, k0 + kq + 0);
    a[1] = (short)A(r0 + rr, k0 + kq + 1);
    a[2] = (short)A(r0 + rr, k0 + kq + 2);
    a[3] = (short)A(r0 + rr, k0 + kq + 3);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      bf16x4 b;
      b[0] = (short)B(k0 + kq + 0, nt * 16 + rr);
      b[1] = (short)B(k0 + kq + 1, nt * 16 + rr);
      b[2] = (short)B(k0 + kq + 2, nt * 16 + rr);
      b[3] = (short)B(k0 + kq + 3, nt * 16 + rr);
      acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[nt], 0, 0, 0);
    }
  }
}
__device__ inline int out_row(int r) { return 4 * ((threadIdx.x & 63) >> 4) + r; }
__device__ inline int out_col(int nt) { return nt * 16 + (threadIdx.x & 15); }

// Activations of a 64-row tile.
struct ActLds {
  unsigned short a0[kRows * kFP];  // inputs (bf16), features 19..31 zero
  unsigned short a1[kRows * kH];   // hidden activations (bf16)
  unsigned short a2[kRows * kH];
  unsigned short a3[kRows * kH];
  float out[kRows];                // logit of each row
};

// Forward pass of the tile; with pre != nullptr the FP32 pre-activations of
// the hidden layers are kept (pre[l][row * 64 + col]) for the backward pass.
__device__ void forward_tile(const MlpLds& W, ActLds& A, float (*pre)[kRows * kH]) {
  const int wv = threadIdx.x >> 6;
  const int r0 = wv * 16;
  for (int l = 0; l < 3; ++l) {
    const int K = l == 0 ? kFP : kH;
    const unsigned short* in = l == 0 ? A.a0 : (l == 1 ? A.a1 : A.a2);
    unsigned short* outl = l == 0 ? A.a1 : (l == 1 ? A.a2 : A.a3);
    const unsigned short* wl = l == 0 ? W.w1 : (l == 1 ? W.w2 : W.w3);
    const float* bl = l == 0 ? W.b1 : (l == 1 ? W.b2 : W.b3);
    f32x4 acc[4];
    for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    mm_strip([&](int r, int k) { return in[r * K + k]; }, [&](int k, int c) { return wl[k * kH + c]; }, r0, K,
             acc);
    for (int nt = 0; nt < 4; ++nt)
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + out_row(r), col = out_col(nt);
        const float v = acc[nt][r] + bl[col];
        if (pre) pre[l][row * kH + col] = v;
        outl[row * kH + col] = bf16_bits(gelu_f(v));
      }
    __syncthreads();
  }
  // 64 -> 1 on the vector units, one row per lane, FP32 in column order
  if (threadIdx.x < kRows) {
    const int row = threadIdx.x;
    float s = 0.0f;
    for (int k = 0; k < kH; ++k) s = fmaf(bf16_val(A.a3[row * kH + k]), bf16_val(W.w4[k]), s);
    A.out[row] = s + W.b4;
  }
  __syncthreads();
}

__device__ inline float logistic(float v) { return 1.0f / (1.0f + expf(-v)); }

__device__ inline float clampd(double v, double lo, double hi) { return (float)fmin(fmax(v, lo), hi); }

__device__ inline float strength(double zj, double w2) {
  const double c = (zj * zj) / w2;
  if (c == 0.0) return -2.0f;
  if (isinf(c)) return 2.0f;
  return clampd(log2(c) / 32.0, -2.0, 2.0);
}

constexpr int kMaxBlocks = 512;  // far-field blocks (B is chosen so that nb <= 512)

__device__ inline int far_block(int N) {
  int B = 4;
  while ((int64_t)B * B < N || 512 * (int64_t)B < N) B *= 2;
  return B;
}

// Far-field block moments of a secular problem, by the whole workgroup.
struct FarLds {
  double Z[kMaxBlocks];
  double D[kMaxBlocks];
};

__device__ void far_moments(const double* __restrict__ d, const double* __restrict__ z, int N, int B, FarLds& F) {
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

__device__ inline float asinh8(double x) { return (float)fmin(fmax(asinh(x) / 8.0, -4.0), 4.0); }

// Features of root i (FP64 arithmetic, FP32 results).
__device__ void root_features(const double* __restrict__ d, const double* __restrict__ z, int N, double rho, int i,
                              int B, const FarLds& FL, float* f) {
  const double lo = d[i];
  double h, w2;
  if (i < N - 1) {
    const double hi = d[i + 1];
    h = hi - lo;
    w2 = h * (hi + lo);
  } else {
    const double hi = sqrt(lo * lo + rho);
    h = rho / (lo + hi);
    w2 = rho;
  }
  for (int q = 0; q < 4; ++q) {
    int j = i - q;
    if (j >= 0) {
      f[2 * q] = (float)fmax((d[j] - lo) / h, -4.0);
      f[2 * q + 1] = strength(z[j], w2);
    } else {
      f[2 * q] = -4.0f;
      f[2 * q + 1] = -2.0f;
    }
    j = i + 1 + q;
    if (j < N) {
      f[8 + 2 * q] = (float)fmin((d[j] - lo) / h, 5.0);
      f[9 + 2 * q] = strength(z[j], w2);
    } else {
      f[8 + 2 * q] = 5.0f;
      f[9 + 2 * q] = -2.0f;
    }
  }
  f[16] = clampd(log2(rho / w2) / 32.0, -2.0, 2.0);
  // far field at the midpoint (in omega^2) of the interval
  const double lam = lo * lo + 0.5 * w2;
  double v = 1.0, sl = 0.0;
  const int nb = (N + B - 1) / B;
  for (int k = 0; k < nb; ++k) {
    const int j0 = k * B, j1 = min(N, (k + 1) * B);
    if (j1 > i - 3 && j0 <= i + 4) {
      for (int j = j0; j < j1; ++j) {
        if (j >= i - 3 && j <= i + 4) continue;
        const double den = d[j] * d[j] - lam;
        const double t = (z[j] * z[j]) / den;
        v += t;
        sl += t / den;
      }
    } else if (FL.Z[k] > 0.0) {
      const double den = FL.D[k] - lam;
      const double t = FL.Z[k] / den;
      v += t;
      sl += t / den;
    }
  }
  f[17] = asinh8(v);
  f[18] = asinh8(sl * w2);
}

// ---------------------------------------------------------------- k_start
__global__ __launch_bounds__(256) void k_start(const NodeDesc* __restrict__ nodes, Work w,
                                               const float* __restrict__ params) {
  __shared__ MlpLds W;
  __shared__ ActLds A;
  __shared__ FarLds FL;
  const NodeDesc nd = nodes[blockIdx.x];
  const int N = w.st[nd.id].N;
  if (N < 2 || (int)blockIdx.y * kRows >= N) return;  // uniform over the workgroup
  const double rho = w.st[nd.id].rho;
  const int64_t vo = nd.vec_off + nd.r0;
  const double* __restrict__ d = w.sd + vo;
  const double* __restrict__ z = w.sz + vo;
  const int B = far_block(N);
  stage_weights(params, W);
  far_moments(d, z, N, B, FL);
  __syncthreads();
  for (int base = blockIdx.y * kRows; base < N; base += gridDim.y * kRows) {
    if (threadIdx.x < kRows) {
      const int i = base + threadIdx.x;
      float f[kF];
      if (i < N) root_features(d, z, N, rho, i, B, FL, f);
      else
        for (int q = 0; q < kF; ++q) f[q] = 0.0f;
      for (int q = 0; q < kFP; ++q) A.a0[threadIdx.x * kFP + q] = q < kF ? bf16_bits(f[q]) : 0;
    }
    __syncthreads();
    forward_tile(W, A, nullptr);
    if (threadIdx.x < kRows) {
      const int i = base + threadIdx.x;
      if (i < N) w.xs[vo + i] = logistic(A.out[threadIdx.x]);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- k_harvest
__global__ __launch_bounds__(64) void k_harvest(const NodeDesc* __restrict__ nodes, Work w, Harvest hv) {
  __shared__ FarLds FL;
  const NodeDesc nd = nodes[blockIdx.x];
  const int N = w.st[nd.id].N;
  if (N < 2 || (int)blockIdx.y * kRows >= N) return;
  const double rho = w.st[nd.id].rho;
  const int64_t vo = nd.vec_off + nd.r0;
  const double* __restrict__ d = w.sd + vo;
  const double* __restrict__ z = w.sz + vo;
  const int B = far_block(N);
  far_moments(d, z, N, B, FL);
  __syncthreads();
  const int lane = threadIdx.x;
  for (int base = blockIdx.y * kRows; base < N; base += gridDim.y * kRows) {
    const int cnt = min(kRows, N - base);
    unsigned long long slot = 0;
    if (lane == 0) slot = atomicAdd(hv.count, (unsigned long long)cnt);
    slot = __shfl(slot, 0, 64);
    const int i = base + lane;
    if (i < N && slot + lane < (unsigned long long)hv.capacity) {
      const int64_t row = (int64_t)slot + lane;
      float f[kF];
      root_features(d, z, N, rho, i, B, FL, f);
      for (int q = 0; q < kF; ++q) hv.X[row * kF + q] = f[q];
      // position of the computed root in its interval
      const double tau = w.tau[vo + i];
      const int o = w.o[vo + i];
      double h;
      if (i < N - 1) h = d[i + 1] - d[i];
      else h = rho / (d[i] + sqrt(d[i] * d[i] + rho));
      double x = (o == i) ? tau / h : 1.0 + tau / h;
      hv.y[row] = clampd(x, 0.0, 1.0);
      hv.tag[3 * row + 0] = (int32_t)vo;
      hv.tag[3 * row + 1] = nd.m;
      hv.tag[3 * row + 2] = i;
    }
  }
}

// Features of one secular problem given directly (rho = sum z^2 summed in
// ascending order).
__global__ __launch_bounds__(64) void k_features(const double* __restrict__ d, const double* __restrict__ z, int N,
                                                 float* __restrict__ X) {
  __shared__ FarLds FL;
  __shared__ double s_rho;
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int j = 0; j < N; ++j) r += z[j] * z[j];
    s_rho = r;
  }
  const int B = far_block(N);
  far_moments(d, z, N, B, FL);
  __syncthreads();
  const int i = blockIdx.x * kRows + threadIdx.x;
  if (i < N) {
    float f[kF];
    root_features(d, z, N, s_rho, i, B, FL, f);
    for (int q = 0; q < kF; ++q) X[(int64_t)i * kF + q] = f[q];
  }
}

// ---------------------------------------------------------------- training
struct GradLds {
  float pre[3][kRows * kH];  // pre-activations, then the back-propagated gradients
  float g4[kRows];
  float part_loss[4];
};

// Forward (and with kGrad the backward pass) of rows [blockIdx.x * 64, +64)
// of the batch; rows are X[idx[r]] (or X[r] with idx == nullptr).
template <bool kGrad>
__global__ __launch_bounds__(256) void k_mlp(const float* __restrict__ params, const float* __restrict__ X,
                                             const float* __restrict__ y, const int32_t* __restrict__ idx,
                                             int rows, float* __restrict__ xhat, float* __restrict__ part,
                                             float* __restrict__ part_loss) {
  __shared__ MlpLds W;
  __shared__ ActLds A;
  __shared__ GradLds G;
  const int t = threadIdx.x;
  const int base = blockIdx.x * kRows;
  stage_weights(params, W);
  int src = -1;
  if (t < kRows && base + t < rows) src = idx ? idx[base + t] : base + t;
  if (t < kRows)
    for (int q = 0; q < kFP; ++q) A.a0[t * kFP + q] = (src >= 0 && q < kF) ? bf16_bits(X[(int64_t)src * kF + q]) : 0;
  __syncthreads();
  forward_tile(W, A, kGrad ? G.pre : nullptr);
  if (!kGrad) {
    if (t < kRows && src >= 0) xhat[base + t] = logistic(A.out[t]);
    return;
  }
  float* P = part + (int64_t)blockIdx.x * kParams;
  // d loss / d logit, loss = mean over the whole batch of (x_hat - y)^2
  if (t < kRows) {
    float g = 0.0f, l = 0.0f;
    if (src >= 0) {
      const float xh = logistic(A.out[t]);
      const float diff = xh - y[src];
      l = diff * diff;
      g = (2.0f / (float)rows) * diff * xh * (1.0f - xh);
    }
    G.g4[t] = g;
    float s = wave_sum(l);
    if (t == 0) G.part_loss[0] = s;
  }
  __syncthreads();
  // layer 4: dW4[k] = sum_r a3[r][k] g4[r]; db4 = sum_r g4[r]
  if (t < kH) {
    float s = 0.0f;
    for (int r = 0; r < kRows; ++r) s = fmaf(bf16_val(A.a3[r * kH + t]), bf16_val(bf16_bits(G.g4[r])), s);
    P[kOffW4 + t] = s;
  }
  if (t == 64) {
    float s = 0.0f;
    for (int r = 0; r < kRows; ++r) s += G.g4[r];
    P[kOffB4] = s;
  }
  if (t == 128) part_loss[blockIdx.x] = G.part_loss[0];
  // g3 = (g4 w4^T) * gelu'(pre3), in place of pre3
  for (int q = t; q < kRows * kH; q += blockDim.x) {
    const int r = q / kH, c = q % kH;
    const float g = bf16_val(bf16_bits(G.g4[r])) * bf16_val(W.w4[c]);
    G.pre[2][q] = g * gelu_d(G.pre[2][q]);
  }
  __syncthreads();
  const int wv = t >> 6;
  for (int l = 2; l >= 0; --l) {
    const float* Gl = G.pre[l];
    const unsigned short* al = l == 0 ? A.a0 : (l == 1 ? A.a1 : A.a2);
    const int offW = l == 0 ? kOffW1 : (l == 1 ? kOffW2 : kOffW3);
    const int offB = l == 0 ? kOffB1 : (l == 1 ? kOffB2 : kOffB3);
    const int K = l == 0 ? kFP : kH;  // input width of layer l+1
    // dW = a^T g: rows of the output are inputs, the sum runs over the 64 rows
    for (int strip = wv; strip < K / 16; strip += 4) {
      f32x4 acc[4];
      for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
      mm_strip([&](int in, int r) { return al[r * K + in]; }, [&](int r, int c) { return bf16_bits(Gl[r * kH + c]); },
               strip * 16, kRows, acc);
      for (int nt = 0; nt < 4; ++nt)
        for (int r = 0; r < 4; ++r) {
          const int in = strip * 16 + out_row(r), col = out_col(nt);
          if (l > 0 || in < kF) P[offW + in * kH + col] = acc[nt][r];
        }
    }
    if (t < kH) {
      float s = 0.0f;
      for (int r = 0; r < kRows; ++r) s += Gl[r * kH + t];
      P[offB + t] = s;
    }
    if (l > 0) {
      // g_{l-1} = (g_l W_l^T) * gelu'(pre_{l-1}), in place of pre_{l-1}
      const unsigned short* wl = l == 1 ? W.w2 : W.w3;
      float* Gp = G.pre[l - 1];
      f32x4 acc[4];
      for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
      mm_strip([&](int r, int k) { return bf16_bits(Gl[r * kH + k]); }, [&](int k, int c) { return wl[c * kH + k]; },
               wv * 16, kH, acc);
      for (int nt = 0; nt < 4; ++nt)
        for (int r = 0; r < 4; ++r) {
          const int row = wv * 16 + out_row(r), col = out_col(nt);
          Gp[row * kH + col] = acc[nt][r] * gelu_d(Gp[row * kH + col]);
        }
    }
    __syncthreads();
  }
}

// Sum of the per-workgroup gradients in workgroup order; Adam when adam_t > 0.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ params, float* __restrict__ m,
                                              float* __restrict__ v, const float* __restrict__ part, int nparts,
                                              const float* __restrict__ part_loss, float* __restrict__ grad_out,
                                              float* __restrict__ loss_out, int adam_t, float lr,
                                              float inv_rows) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0 && loss_out) {
    float s = 0.0f;
    for (int b = 0; b < nparts; ++b) s += part_loss[b];
    *loss_out = s * inv_rows;  // mean squared error of the batch
  }
  if (p >= kParams) return;
  float g = 0.0f;
  for (int b = 0; b < nparts; ++b) g += part[(int64_t)b * kParams + p];
  if (grad_out) grad_out[p] = g;
  if (adam_t > 0) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float mm = b1 * m[p] + (1.0f - b1) * g;
    const float vv = b2 * v[p] + (1.0f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float mh = mm / (1.0f - powf(b1, (float)adam_t));
    const float vh = vv / (1.0f - powf(b2, (float)adam_t));
    params[p] -= lr * mh / (sqrtf(vh) + eps);
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

void launch_start(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, const float* params,
                  hipStream_t st) {
  if (nnodes <= 0) return;
  const int gy = grid_y(nnodes, (max_m + kRows - 1) / kRows, 4096);
  hipLaunchKernelGGL(k_start, dim3(nnodes, gy), dim3(256), 0, st, nodes, w, params);
}

void launch_harvest(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, const Harvest& hv,
                    hipStream_t st) {
  if (nnodes <= 0) return;
  const int gy = grid_y(nnodes, (max_m + kRows - 1) / kRows, 4096);
  hipLaunchKernelGGL(k_harvest, dim3(nnodes, gy), dim3(64), 0, st, nodes, w, hv);
}

void launch_features(const double* d, const double* z, int N, float* X, hipStream_t st) {
  if (N < 1) return;
  hipLaunchKernelGGL(k_features, dim3((N + kRows - 1) / kRows), dim3(64), 0, st, d, z, N, X);
}

void launch_mlp_forward(const float* params, const float* X, int rows, float* xhat, hipStream_t st) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(k_mlp<false>, dim3((rows + kRows - 1) / kRows), dim3(256), 0, st, params, X, nullptr,
                     nullptr, rows, xhat, nullptr, nullptr);
}

int mlp_parts(int rows) { return (rows + kRows - 1) / kRows; }

void launch_mlp_grad(const float* params, const float* X, const float* y, const int32_t* idx, int rows,
                     float* part, float* part_loss, hipStream_t st) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(k_mlp<true>, dim3(mlp_parts(rows)), dim3(256), 0, st, params, X, y, idx, rows, nullptr,
                     part, part_loss);
}

void launch_adam(float* params, float* m, float* v, const float* part, int nparts, const float* part_loss,
                 float* grad_out, float* loss_out, int adam_t, float lr, float inv_rows, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, st, params, m, v, part, nparts, part_loss,
                     grad_out, loss_out, adam_t, lr, inv_rows);
}

}  // namespace bdc
