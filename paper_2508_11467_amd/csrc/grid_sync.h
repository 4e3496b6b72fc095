// Grid-wide barrier and all-reduce for cooperative launches (all
// workgroups resident): counters and a generation number in device memory.
// Every wait is bounded: an expired wait sets a flag and makes the barrier
// return false, so a kernel always ends.
#pragma once

#include <hip/hip_runtime.h>

namespace bdc {

constexpr unsigned kSpin = 1u << 26;
constexpr int kGridGroup = 16;     // workgroups per group of the all-reduce
constexpr int kGridMaxGroups = 64;
constexpr int kGridMaxWg = kGridGroup * kGridMaxGroups;  // workgroups of a grid, at most

struct GridSync {
  unsigned count;
  unsigned gen;
  unsigned expired;
  unsigned pad[29];
  unsigned group[kGridMaxGroups * 16];  // one counter per 64 bytes
};

// device bytes that hold a GridSync, rounded to 256
constexpr size_t kGridSyncBytes = (sizeof(GridSync) + 255) / 256 * 256;
// doubles of the group partial sums of one all-reduce (stride doubles per group)
constexpr size_t grid_group_doubles(int stride) { return (size_t)kGridMaxGroups * stride; }

// All workgroups of the grid meet; returns false if the wait expired.  The
// writes of every thread before the barrier are visible to every thread
// after it.  The workgroup barrier orders every thread's writes before
// thread 0's device-scope release fence (the L2 write-back that makes this
// XCD's writes visible to the others; release is cumulative over what the
// workgroup barrier ordered before it); then thread 0 arrives with a relaxed
// increment of the counter and, while the generation has not moved, polls it
// with relaxed coherent loads; then one device-scope acquire fence (the L2
// invalidate).  Acquire loads inside the poll would invalidate the XCD's L2
// on every spin and slow every workgroup on it.  A release fence in every
// thread would do the same with one L2 write-back per wavefront; measured,
// it slows the bidiagonal reduction by about 9%.
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

// The state before a grid's first barrier (a workgroup of any size).
__device__ inline void grid_sync_clear(GridSync* s) {
  if (threadIdx.x == 0) {
    s->count = 0;
    s->gen = 0;
    s->expired = 0;
  }
  for (int i = threadIdx.x; i < kGridMaxGroups * 16; i += blockDim.x) s->group[i] = 0;
}

// Bounded wait (thread 0) until the generation moves past g0; then the
// device-scope acquire fence.
__device__ inline unsigned grid_wait_gen(GridSync* s, unsigned g0) {
  unsigned it = 0;
  while (__hip_atomic_load(&s->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g0) {
    if (++it > kSpin) {
      __hip_atomic_store(&s->expired, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return 0;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return 1;
}

// All-reduce of cnt (<= 256) values: every workgroup has written its values
// to slots[g * stride + q] before the call (all threads call it; a workgroup
// of at least 256 threads).  The workgroups meet in groups of kGridGroup:
// the last to arrive in a group adds the group's slots in workgroup order
// into gslots[group * stride + q] and arrives at the root counter; the last
// group to arrive moves the generation.  Then every workgroup adds the group
// sums, split into parts that are added in a fixed order, into out[q] (LDS).
// The totals are the same in every workgroup and do not depend on the order
// of arrival.  Each workgroup reads about G / kGridGroup slots instead of G.
// sh: 3 unsigned in LDS (sh[0]: this workgroup arrived last in its group,
// read by every thread; sh[2]: the wait ended in time -- a word of its own,
// so that thread 0 cannot overwrite sh[0] before a slower wavefront has read
// it); red: 256 doubles in LDS.  Consecutive calls must alternate two sets of
// slots and gslots (a workgroup may write the next call's slots while
// another still reads this call's group sums).  Returns false if a wait
// expired.
__device__ inline bool grid_allreduce(GridSync* s, const double* slots, double* gslots, int stride, int cnt,
                                      double* out, double* red, unsigned* sh) {
  const int t = threadIdx.x;
  const unsigned G = gridDim.x, g = blockIdx.x;
  const unsigned grp = g / kGridGroup, ngrp = (G + kGridGroup - 1) / kGridGroup;
  const unsigned in_grp = min((unsigned)kGridGroup, G - grp * kGridGroup);
  // the workgroup's writes (the slots, and whatever the caller publishes),
  // then thread 0's release fence, as in grid_barrier
  __syncthreads();
  if (t == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    sh[1] = __hip_atomic_load(&s->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool last = __hip_atomic_fetch_add(&s->group[grp * 16], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                      in_grp - 1;
    if (last) {
      __hip_atomic_store(&s->group[grp * 16], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    sh[0] = last;
  }
  __syncthreads();
  const bool last = sh[0] != 0;
  unsigned ok = 1;
  if (last) {
    for (int q = t; q < cnt; q += 256) {
      double a = 0.0;
      for (unsigned w = 0; w < in_grp; ++w) a += slots[(size_t)(grp * kGridGroup + w) * stride + q];
      gslots[(size_t)grp * stride + q] = a;
    }
    __syncthreads();
    if (t == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      if (__hip_atomic_fetch_add(&s->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == ngrp - 1) {
        __hip_atomic_store(&s->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&s->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      } else {
        ok = grid_wait_gen(s, sh[1]);
      }
    }
  } else if (t == 0) {
    ok = grid_wait_gen(s, sh[1]);
  }
  if (t == 0) sh[2] = ok;
  __syncthreads();
  if (sh[2] == 0) return false;
  sum_slots(gslots, stride, (int)ngrp, cnt, out, red);
  return true;
}


}  // namespace bdc
