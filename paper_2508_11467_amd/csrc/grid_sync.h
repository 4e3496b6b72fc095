// Grid-wide barrier for cooperative launches (all workgroups resident):
// a counter and a generation number in device memory.  Every wait is
// bounded: an expired wait sets a flag and makes the barrier return false,
// so a kernel always ends.
#pragma once

#include <hip/hip_runtime.h>

namespace bdc {

constexpr unsigned kSpin = 1u << 26;

struct GridSync {
  unsigned count;
  unsigned gen;
  unsigned expired;
  unsigned pad;
};

// All workgroups of the grid meet; returns false if the wait expired.  The
// writes of every thread before the barrier are visible to every thread
// after it.  One thread per workgroup arrives: a device-scope release fence
// (the L2 write-back that makes this XCD's writes visible to the others), a
// relaxed increment of the counter, and, while the generation has not moved,
// relaxed coherent polling; then one device-scope acquire fence (the L2
// invalidate).  Acquire loads inside the poll would invalidate the XCD's L2
// on every spin and slow every workgroup on it.
__device__ inline bool grid_barrier(GridSync* s, unsigned nwg, unsigned* sh_ok) {
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned ok = 1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned g = __hip_atomic_load(&s->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__hip_atomic_fetch_add(&s->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == nwg - 1) {
      __hip_atomic_store(&s->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&s->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned it = 0;
      while (__hip_atomic_load(&s->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (++it > kSpin) {
          __hip_atomic_store(&s->expired, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *sh_ok = ok;
  }
  __syncthreads();
  return *sh_ok != 0;
}


// Totals of `cnt` values that every workgroup of the grid left in its slot
// (value q of workgroup w at base[w * stride + q]), read after a grid
// barrier: the 256 threads split the workgroups into parts (plain loads, all
// in flight together; the barrier's acquire makes them fresh), and the parts
// are added in a fixed order, so every workgroup gets the same totals.
// out[q] for q < cnt; red must hold 256 doubles.  All threads call it.
__device__ inline void sum_slots(const double* base, int stride, int G, int cnt, double* out, double* red) {
  if (cnt <= 0) return;
  const int t = threadIdx.x;
  const int parts = cnt >= 256 ? 1 : 256 / cnt;
  __syncthreads();
  if (t < parts * cnt) {
    const int q = t % cnt, p = t / cnt;
    double s = 0.0;
    for (int w = p; w < G; w += parts) s += base[(size_t)w * stride + q];
    red[p * cnt + q] = s;
  }
  __syncthreads();
  for (int q = t; q < cnt; q += 256) {
    double s = 0.0;
    for (int p = 0; p < parts; ++p) s += red[p * cnt + q];
    out[q] = s;
  }
  __syncthreads();
}

}  // namespace bdc
