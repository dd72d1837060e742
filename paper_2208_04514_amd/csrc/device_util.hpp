// Wave64 and grid-level helpers for gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace dawn {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Mask of lanes below the calling lane.
__device__ __forceinline__ u64 lanes_below() {
  return (1ull << lane_id()) - 1ull;
}

__device__ __forceinline__ unsigned ld_acquire(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned ld_relaxed(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u64 ld_relaxed(const u64* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_relaxed(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Agent-scope relaxed stores: written through to the point every XCD reads
// coherently (a plain store may sit in its own XCD's L2 until the kernel ends).
__device__ __forceinline__ void st_relaxed(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(unsigned* p, unsigned v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ long long ld_relaxed(const long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned atom_add(unsigned* p, unsigned v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u64 atom_add(u64* p, u64 v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u64 atom_or(u64* p, u64 v) {
  return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Inclusive prefix sum across the wave.
__device__ __forceinline__ int wave_incl_scan(int x) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    int y = __shfl_up(x, d, kWave);
    if (lane >= d) x += y;
  }
  return x;
}

__device__ __forceinline__ unsigned wave_sum(unsigned x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, kWave);
  return x;
}

__device__ __forceinline__ u64 wave_sum(u64 x) {
  unsigned lo = (unsigned)x, hi = (unsigned)(x >> 32);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    unsigned olo = __shfl_xor(lo, d, kWave), ohi = __shfl_xor(hi, d, kWave);
    unsigned nlo = lo + olo;
    hi = hi + ohi + (nlo < lo ? 1u : 0u);
    lo = nlo;
  }
  return ((u64)hi << 32) | lo;
}

__device__ __forceinline__ u64 wave_or(u64 x) {
  unsigned lo = (unsigned)x, hi = (unsigned)(x >> 32);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    lo |= __shfl_xor(lo, d, kWave);
    hi |= __shfl_xor(hi, d, kWave);
  }
  return ((u64)hi << 32) | lo;
}

// Smallest j in [0, 64) with incl[j] > x, where `incl` is the wave's
// non-decreasing inclusive scan and incl[63] > x.  Six lane permutes.
__device__ __forceinline__ int wave_owner(int incl, int x) {
  int lo = 0;
#pragma unroll
  for (int step = 32; step > 0; step >>= 1) {
    int probe = lo + step - 1;
    int v = __shfl(incl, probe, kWave);
    if (v <= x) lo = probe + 1;
  }
  return lo;
}

// Wave-aggregated append: every lane with `pred` gets a distinct slot from
// *counter; one atomic per wave.  Returns the slot, or -1 without `pred`.
__device__ __forceinline__ int wave_append(unsigned* counter, bool pred) {
  u64 mask = __ballot(pred);
  if (mask == 0) return -1;
  int leader = __ffsll((unsigned long long)mask) - 1;
  unsigned base = 0;
  if (lane_id() == leader) base = atom_add(counter, (unsigned)__popcll(mask));
  base = __shfl(base, leader, kWave);
  return pred ? (int)(base + __popcll(mask & lanes_below())) : -1;
}

// Block-wide sums, one call per counter set; every thread must call it.
template <int BLOCK>
__device__ __forceinline__ void block_sum3(unsigned& a, u64& b, u64& c) {
  __shared__ unsigned sa[BLOCK / kWave];
  __shared__ u64 sb[BLOCK / kWave], sc[BLOCK / kWave];
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if (lane_id() == 0) { sa[w] = a; sb[w] = b; sc[w] = c; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < BLOCK / kWave; ++i) { a += sa[i]; b += sb[i]; c += sc[i]; }
  }
  __syncthreads();
}

// Barrier across all workgroups of a cooperative launch.  Thread 0 of each
// workgroup arrives with a release fence and waits with an acquire fence at
// agent scope, so plain stores before the barrier are visible to plain loads
// after it on every XCD.  The last arriver resets the count and bumps the
// generation, so the state is reusable across barriers and launches.
//
// The wait is bounded: after kBarrierTimeoutTicks of the 100 MHz wall clock a
// waiter raises `abort` and leaves, and every later call returns false at
// once, so a kernel always drains even if its workgroups ever disagreed on the
// number of barriers.  Returns false on abort.
constexpr unsigned long long kBarrierTimeoutTicks = 1000000000ull;   // 10 s

__device__ __forceinline__ bool grid_sync(GridBarrier* bar) {
  __shared__ int ok;
  __syncthreads();
  if (gridDim.x == 1) return true;   // one workgroup: the workgroup barrier is enough
  if (threadIdx.x == 0) {
    ok = 1;
    const unsigned nb = gridDim.x;
    if (__hip_atomic_load(&bar->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
      ok = 0;
    } else {
      unsigned g = __hip_atomic_load(&bar->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();
      unsigned arrived = __hip_atomic_fetch_add(&bar->count, 1u, __ATOMIC_ACQ_REL,
                                                __HIP_MEMORY_SCOPE_AGENT);
      if (arrived == nb - 1) {
        __hip_atomic_store(&bar->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&bar->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        const unsigned long long t0 = wall_clock64();
        while (__hip_atomic_load(&bar->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
          if (__hip_atomic_load(&bar->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
              wall_clock64() - t0 > kBarrierTimeoutTicks) {
            __hip_atomic_store(&bar->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      __threadfence();
    }
  }
  __syncthreads();
  return ok != 0;
}

}  // namespace dawn
