// Cross-workgroup exchange through per-workgroup epoch flags (gfx950).
//
// A workgroup publishes its prior global writes by an agent-scope release
// fence in every wave, a workgroup barrier and one agent-scope release store
// of its flag; a reader polls the
// flags with relaxed loads, then acquires at agent scope and passes the
// result on with a workgroup barrier.  Every wait is bounded: a wait that
// runs out sets bit 0 of *err and returns instead of hanging (the grid must
// be co-resident for the exchange to complete; the host checks occupancy).
#pragma once

#include <hip/hip_runtime.h>

namespace cgd {
namespace {

constexpr long kSpinLimit = 1L << 25;

// Every wave releases its own global writes at agent scope (a release fence
// only waits for the issuing wave's stores), the barrier orders all of them
// before thread 0, whose release store of the flag covers what it observed.
__device__ inline void publish(unsigned* flag, unsigned value) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until flags[0..count) >> 1 >= epoch; returns the OR of the flags' low
// bits over all of them.  BS is the workgroup size.
template <int BS>
__device__ inline int wait_flags(const unsigned* flags, int count, unsigned epoch, int* err) {
  int bit = 0;
  if ((int)threadIdx.x < count) {
    for (int i = threadIdx.x; i < count; i += BS) {
      long spins = 0;
      unsigned v;
      while (((v = __hip_atomic_load(&flags[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >> 1) <
             epoch) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) {
          atomicOr(err, 1);
          break;
        }
      }
      bit |= (int)(v & 1u);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  return __syncthreads_or(bit);
}

// Start-up census of a launch whose workgroups wait for each other (the
// per-member solvers, launched without the cooperative API): every
// workgroup checks in on *word (zero before the launch); all proceed once
// the count reaches the grid size.  If it has not within `ticks` of the
// 100 MHz real-time counter (the grid is not all resident: another
// kernel holds part of the GPU), the first workgroup to give up marks the
// word abandoned, only while the count it saw is still current (so either
// every workgroup proceeds or none does), sets bit 2 of *err, and every
// workgroup returns false: the call fails promptly instead of waiting in
// its exchanges.  Thread 0 decides; the result is the workgroup's.
constexpr unsigned long long kCensusAbandoned = 1ull << 40;

// Thread 0 checks in at the start of the kernel; the count it got back is
// passed to census_wait after work that needs no other workgroup (so the
// dispatch of the rest of the grid overlaps it).
__device__ inline unsigned long long census_arrive(unsigned long long* word) {
  return __hip_atomic_fetch_add(word, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
}

__device__ inline bool census_wait(unsigned long long* word, int* err, unsigned long long ticks,
                                   unsigned long long v) {
  __shared__ int go;
  if (threadIdx.x == 0) {
    const unsigned long long grid = gridDim.x;
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    int ok = 1;
    for (;;) {
      if (v & kCensusAbandoned) {
        ok = 0;
        break;
      }
      if (v >= grid) break;
      if (__builtin_amdgcn_s_memrealtime() - t0 > ticks) {
        unsigned long long seen = v;
        if (__hip_atomic_compare_exchange_strong(word, &seen, v | kCensusAbandoned,
                                                 __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)) {
          atomicOr(err, 4);
          ok = 0;
          break;
        }
        v = seen;  // the count moved: look again
        continue;
      }
      __builtin_amdgcn_s_sleep(2);
      v = __hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    go = ok;
  }
  __syncthreads();
  return go != 0;
}

}  // namespace
}  // namespace cgd

// Diagnostic timestamp (100 MHz real-time counter), workgroup 0, thread 0.
#define CGD_TRACE(slot)                                                        \
  do {                                                                        \
    if (a.trace && blockIdx.x == 0 && threadIdx.x == 0 && (slot) < 256)       \
      a.trace[(slot)] = __builtin_amdgcn_s_memrealtime();                      \
  } while (0)
