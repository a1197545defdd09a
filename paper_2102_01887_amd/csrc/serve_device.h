// Device side of the serving ring (HIP sources only): how a wavefront of a
// persistent decision kernel claims published requests and hands back
// decisions.  The ring and its control words live in pinned host memory
// mapped into the device's address space; the claim counters in device
// memory (ServeRing).
#pragma once

#include <hip/hip_runtime.h>

#include "llama_internal.h"

namespace llama {

struct ServeClaim {
  long long first;  // first claimed sequence number
  int count;        // requests claimed (0: none published, or stop)
  bool stop;        // the host asked the kernel to exit
};

// Lane 0 of every wavefront counts it in at start (ctr[3]: wavefronts alive).
__device__ inline void serve_enter(const ServeRing& r, int lane) {
  if (lane == 0) __hip_atomic_fetch_add(r.ctr + 3, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ... and out at exit: the wavefront that takes the count to zero sets the
// exit word, after its results, so that the host can tell without asking
// the runtime that the kernel has ended (a wavefront that finds no work for
// the idle time before a sibling has even started can set it early; the host
// confirms with the launch's completion event before relaunching).
__device__ inline void serve_leave(const ServeRing& r, int lane) {
  if (lane == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    if (__hip_atomic_fetch_add(r.ctr + 3, ~0ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == 1ull)
      __hip_atomic_store(r.exited, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// Clock handshake served by a running kernel (lane 0 of one wavefront): when
// the host's probe word changes, stamp the device clock and acknowledge the
// probe, stamp first.  The host re-anchors its device-to-host time mapping
// from the round trip, so the two clocks' different rates do not accumulate
// into the latencies it reports.
__device__ inline void serve_clock(const ServeRing& r, int& answered) {
  const int p = __hip_atomic_load(r.probe, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  if (p != answered) {
    __hip_atomic_store(r.stamp, (unsigned long long)wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    __hip_atomic_store(r.ack, p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    answered = p;
  }
}

// Lane 0 reads the stop word and the published head, then claims up to
// `chunk` unclaimed requests by compare-and-swap on the device counter (each
// failed swap means another wavefront advanced it, so the loop ends within
// head - counter attempts); the claim is broadcast to the wavefront, and
// every lane's later reads of the ring are ordered after the head it saw.
// The wavefront that passes `answered` (non-null) also serves clock probes.
__device__ inline ServeClaim serve_claim(const ServeRing& r, int lane, int chunk, int* answered) {
  long long first = -1, cnt = 0;
  int stop = 0;
  if (lane == 0) {
    if (answered) serve_clock(r, *answered);
    stop = __hip_atomic_load(r.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    const long long head = __hip_atomic_load(r.head, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
    unsigned long long cur = __hip_atomic_load(r.ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (!stop && (long long)cur < head) {
      const long long k = head - (long long)cur < chunk ? head - (long long)cur : chunk;
      if (__hip_atomic_compare_exchange_strong(r.ctr, &cur, cur + (unsigned long long)k, __ATOMIC_RELAXED,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        first = (long long)cur;
        cnt = k;
        break;
      }
    }
    if (cnt > 0) {
      atomicAdd(r.ctr + 1, 1ull);
      atomicMax(r.ctr + 2, (unsigned long long)cnt);
      atomicMax(r.ctr + 4, (unsigned long long)wall_clock64());
    }
  }
  first = __shfl(first, 0, 64);
  cnt = __shfl(cnt, 0, 64);
  stop = __shfl(stop, 0, 64);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
  return ServeClaim{first, (int)cnt, stop != 0};
}

// Idle exit, kernel-wide: a wavefront that has claimed nothing for the idle
// time looks at the latest claim of any wavefront (ctr[4]) and exits only if
// that too is older, so the wavefronts (the one serving clock probes among
// them) stay while any of them has work, and leave together.
__device__ inline bool serve_idle(const ServeRing& r, unsigned long long now, unsigned long long& last) {
  if (now - last <= r.idle_ticks) return false;
  const unsigned long long g = __hip_atomic_load(r.ctr + 4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (g > last) last = g;
  return now > last && now - last > r.idle_ticks;
}

// Decision of request seq (slot = seq % cap): its device timestamp, then the
// tagged result word, ordered so that a host that sees the tag sees the time.
__device__ inline void serve_write(const ServeRing& r, long long seq, long long slot, int cfg, int flag) {
  r.ts[slot] = (unsigned long long)wall_clock64();
  const unsigned long long v = ((unsigned long long)(uint32_t)(seq + 1) << 32) |
                               ((uint32_t)(cfg + 1) & 0x7FFFFFFFu) | ((uint32_t)(flag != 0) << 31);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
  __hip_atomic_store(r.res + slot, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

}  // namespace llama
