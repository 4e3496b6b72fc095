// Learned start of the secular iteration: a 19 -> 64 -> 64 -> 64 -> 1 MLP
// proposes each root's fractional position in its interval.
//
//   k_mlp_pack packs the parameters for inference (bfloat16, transposed);
//              the secular kernel computes features and proposals itself
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
// Features: see mlp_device.h.
#include "bdc_internal.h"
#include "block_util.h"
#include "mlp_device.h"

namespace bdc {
namespace {

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

// ---------------------------------------------------------------- k_harvest
__global__ __launch_bounds__(256) void k_harvest(const NodeDesc* __restrict__ nodes, Work w, Harvest hv) {
  __shared__ FeatLds FL;
  __shared__ unsigned long long s_slot;
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
  const int t = threadIdx.x;
  for (int base = blockIdx.y * kRows; base < N; base += gridDim.y * kRows) {
    const int cnt = min(kRows, N - base);
    if (t == 0) s_slot = atomicAdd(hv.count, (unsigned long long)cnt);
    __syncthreads();
    const unsigned long long slot = s_slot;
    const int64_t cap = hv.capacity;
    block_features(d, z, N, rho, base, B, FL, [&](int r, int q, float v) {
      if (slot + r < (unsigned long long)cap) hv.X[((int64_t)slot + r) * kF + q] = v;
    });
    const int i = base + t;
    if (t < kRows && i < N && slot + t < (unsigned long long)cap) {
      const int64_t row = (int64_t)slot + t;
      // position of the computed root in its interval
      const double tau = w.tau[vo + i];
      const int o = w.o[vo + i];
      double lo, h, w2;
      interval_of(d, N, rho, i, lo, h, w2);
      const double x = (o == i) ? tau / h : 1.0 + tau / h;
      hv.y[row] = clampd(x, 0.0, 1.0);
      hv.tag[3 * row + 0] = (int32_t)vo;
      hv.tag[3 * row + 1] = nd.m;
      hv.tag[3 * row + 2] = i;
    }
    __syncthreads();
  }
}

// Features of one secular problem given directly (rho = sum z^2 summed in
// ascending order).
__global__ __launch_bounds__(256) void k_features(const double* __restrict__ d, const double* __restrict__ z, int N,
                                                  float* __restrict__ X) {
  __shared__ FeatLds FL;
  __shared__ double s_rho;
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int j = 0; j < N; ++j) r += z[j] * z[j];
    s_rho = r;
  }
  const int B = far_block(N);
  far_moments(d, z, N, B, FL);
  __syncthreads();
  const int base = blockIdx.x * kRows;
  block_features(d, z, N, s_rho, base, B, FL,
                 [&](int r, int q, float v) { X[(int64_t)(base + r) * kF + q] = v; });
}

// Parameters -> inference layout (bfloat16 transposed weights, FP32 biases).
__global__ __launch_bounds__(256) void k_mlp_pack(const float* __restrict__ p, unsigned short* __restrict__ pk) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < kPkHalf + kPkBias; q += gridDim.x * blockDim.x) {
    if (q < kPkW2) {
      const int o = (q - kPkW1) / kFP, i = (q - kPkW1) % kFP;
      pk[q] = i < kF ? bf16_bits(p[kOffW1 + i * kH + o]) : 0;
    } else if (q < kPkW3) {
      const int o = (q - kPkW2) / kH, i = (q - kPkW2) % kH;
      pk[q] = bf16_bits(p[kOffW2 + i * kH + o]);
    } else if (q < kPkW4) {
      const int o = (q - kPkW3) / kH, i = (q - kPkW3) % kH;
      pk[q] = bf16_bits(p[kOffW3 + i * kH + o]);
    } else if (q < kPkHalf) {
      const int o = (q - kPkW4) / kH, i = (q - kPkW4) % kH;
      pk[q] = o == 0 ? bf16_bits(p[kOffW4 + i]) : 0;
    } else {
      const int b = q - kPkHalf;
      const float v = b < kH ? p[kOffB1 + b] : b < 2 * kH ? p[kOffB2 + b - kH] : b < 3 * kH ? p[kOffB3 + b - 2 * kH]
                                                                                       : p[kOffB4];
      ((float*)(pk + kPkHalf))[b] = v;
    }
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

void launch_harvest(const NodeDesc* nodes, int nnodes, int max_m, const Work& w, const Harvest& hv,
                    hipStream_t st) {
  if (nnodes <= 0) return;
  const int gy = grid_y(nnodes, (max_m + kRows - 1) / kRows, 4096);
  hipLaunchKernelGGL(k_harvest, dim3(nnodes, gy), dim3(256), 0, st, nodes, w, hv);
}

void launch_features(const double* d, const double* z, int N, float* X, hipStream_t st) {
  if (N < 1) return;
  hipLaunchKernelGGL(k_features, dim3((N + kRows - 1) / kRows), dim3(256), 0, st, d, z, N, X);
}

size_t mlp_pack_bytes() { return kPackBytes; }

void launch_mlp_pack(const float* params, unsigned short* packed, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_pack, dim3((kPkHalf + kPkBias + 255) / 256), dim3(256), 0, st, params, packed);
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
