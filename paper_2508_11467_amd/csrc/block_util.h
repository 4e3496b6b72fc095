// Workgroup-level reductions and scans for 256-thread blocks (4 wave64s).
#pragma once

#include <hip/hip_runtime.h>

namespace bdc {

constexpr int kBlock = 256;

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline double wave_maxd(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ inline double wave_prod(double v) {
  for (int off = 32; off > 0; off >>= 1) v *= __shfl_xor(v, off, 64);
  return v;
}

// All threads of the 256-thread block get the block maximum.
__device__ inline double block_max(double v, double* sh /* >= 4 */) {
  v = wave_maxd(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  return fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

__device__ inline double block_sum(double v, double* sh /* >= 4 */) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Exclusive prefix sum over the block of K counters per thread.  sh must hold
// 256*K ints.  total[] receives the block totals.
template <int K>
__device__ inline void block_exscan(int (&v)[K], int (&total)[K], int* sh) {
  const int t = threadIdx.x;
  __syncthreads();
  for (int q = 0; q < K; ++q) sh[q * kBlock + t] = v[q];
  __syncthreads();
  // Hillis-Steele inclusive scan per counter
  for (int off = 1; off < kBlock; off <<= 1) {
    int add[K];
    for (int q = 0; q < K; ++q) add[q] = t >= off ? sh[q * kBlock + t - off] : 0;
    __syncthreads();
    for (int q = 0; q < K; ++q) sh[q * kBlock + t] += add[q];
    __syncthreads();
  }
  for (int q = 0; q < K; ++q) {
    total[q] = sh[q * kBlock + kBlock - 1];
    v[q] = sh[q * kBlock + t] - v[q];
  }
  __syncthreads();
}

// The same for a block of BS threads (a multiple of 64): sh holds BS*K ints.
template <int K, int BS>
__device__ inline void block_exscan_n(int (&v)[K], int (&total)[K], int* sh) {
  const int t = threadIdx.x;
  __syncthreads();
  for (int q = 0; q < K; ++q) sh[q * BS + t] = v[q];
  __syncthreads();
  for (int off = 1; off < BS; off <<= 1) {
    int add[K];
    for (int q = 0; q < K; ++q) add[q] = t >= off ? sh[q * BS + t - off] : 0;
    __syncthreads();
    for (int q = 0; q < K; ++q) sh[q * BS + t] += add[q];
    __syncthreads();
  }
  for (int q = 0; q < K; ++q) {
    total[q] = sh[q * BS + BS - 1];
    v[q] = sh[q * BS + t] - v[q];
  }
  __syncthreads();
}

// Exclusive prefix sums of K counters over a block of BS threads (a multiple
// of 64) with wavefront shuffles: a scan inside each wavefront, then the
// wavefront totals.  sh must hold K * BS/64 ints.  Same results as
// block_exscan_n (integer sums), with two barriers.
template <int K, int BS>
__device__ inline void block_exscan_w(int (&v)[K], int (&total)[K], int* sh) {
  constexpr int NW = BS / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int inc[K];
  for (int q = 0; q < K; ++q) {
    int x = v[q];
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    inc[q] = x;
  }
  __syncthreads();
  if (lane == 63)
    for (int q = 0; q < K; ++q) sh[q * NW + wv] = inc[q];
  __syncthreads();
  for (int q = 0; q < K; ++q) {
    int before = 0, all = 0;
    for (int u = 0; u < NW; ++u) {
      const int t = sh[q * NW + u];
      if (u < wv) before += t;
      all += t;
    }
    total[q] = all;
    v[q] = before + inc[q] - v[q];
  }
  __syncthreads();
}

// Block sum for BS threads; the wave sums are added in wave order.
template <int BS>
__device__ inline double block_sum_n(double v, double* sh /* >= BS/64 */) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int q = 0; q < BS / 64; ++q) s += sh[q];
  return s;
}

// Block maximum for BS threads.
template <int BS>
__device__ inline double block_max_n(double v, double* sh /* >= BS/64 */) {
  v = wave_maxd(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double s = sh[0];
  for (int q = 1; q < BS / 64; ++q) s = fmax(s, sh[q]);
  return s;
}

}  // namespace bdc
