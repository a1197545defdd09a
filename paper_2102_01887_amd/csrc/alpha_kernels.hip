// Finite-alpha Eq. 1 with per-backend queueing times (Sec. 4.3, Eq. 1 with a
// finite alpha, Alg. 1 targets with Eq. 2's queueing time per backend), by
// one search per invocation.
//
// A configuration x on backend h is feasible for an invocation with
// remaining time r0 = slo - elapsed iff L_x < floor(ref * R / W) with
// R = clamp(r0 - Q[h], 0, 2^31 - 1), that is iff r0 >= T_x + Q[h] with
// T_x = ceil((L_x + 1) * W / ref) >= 1 (never when T_x > 2^31 - 1: no clamped
// R reaches it).  So per call every configuration has one threshold
// T'_x = T_x + Q[h] on the scale of r0, and the feasible set of an
// invocation is the prefix of the op's configurations in T' order with
// T' <= r0.  r0 lies in [-(2^31 - 1), 2^31 - 1], so T' is stored clamped to
// that range and offset by 2^31 - 1, with 2^32 - 1 for "never": one uint32.  The choice is then the smaller of the prefix minimum of the
// feasible keys and the suffix minimum of the infeasible keys at that point
// (keys = rank of the objective value << 16 | local index, unique per
// configuration, so there are no ties between the two).
//
//   alpha_merge_kernel   one wavefront per op: T' of every configuration
//                        (exact integer threshold), the backends' lists
//                        (each ascending in latency, hence in T') merged by
//                        binary search in LDS, prefix and suffix minima by
//                        wavefront scans
//   alpha_queue_kernel   one thread per invocation: one binary search over
//                        the op's merged thresholds, two key loads
#include <hip/hip_runtime.h>

#include "llama_internal.h"

namespace llama {
namespace {

constexpr uint32_t T_NEVER = 0x80000000u;    // threshold T above 2^31 - 1
constexpr uint32_t TQ_NEVER = 0xFFFFFFFFu;   // stored T + Q that no r0 reaches
constexpr int64_t R0_MAX = 0x7FFFFFFFll;     // |r0| <= 2^31 - 1

// floor(a / b) for 0 <= a < 2^62, 1 <= b and a quotient below 2^53: an FP64
// estimate corrected by one remainder step.
__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b) {
  int64_t q = (int64_t)((double)a / (double)b);
  const int64_t r = a - q * b;
  if (r < 0) q -= 1;
  else if (r >= b) q += 1;
  return q;
}

// T = ceil((L + 1) * W / ref) as an exact integer, or T_NEVER above 2^31 - 1.
__device__ __forceinline__ uint32_t remaining_time_threshold(uint32_t L, int64_t W, int64_t ref) {
  const unsigned __int128 lhs = (unsigned __int128)((uint64_t)L + 1u) * (uint64_t)W;
  if (lhs > (unsigned __int128)((uint64_t)ref * 0x7FFFFFFFull)) return T_NEVER;
  return (uint32_t)floor_div((int64_t)(uint64_t)lhs + ref - 1, ref);
}

// Wavefront inclusive min scan (lane order).
__device__ __forceinline__ uint32_t wave_min_scan(uint32_t x, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x = y < x ? y : x;
  }
  return x;
}

// Wavefront inclusive min scan in reverse lane order (suffix minima).
__device__ __forceinline__ uint32_t wave_min_scan_rev(uint32_t x, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_down(x, d, 64);
    if (lane + d < 64) x = y < x ? y : x;
  }
  return x;
}

template <int NHW>
__global__ __launch_bounds__(64) void alpha_merge_kernel(DevTables t, int mode, const int64_t* queue) {
  extern __shared__ uint32_t sMem[];
  const int v = blockIdx.x;
  const int lane = threadIdx.x;
  const int a = t.cfg_off[v], n = t.cfg_off[v + 1] - a;
  uint32_t* sT = sMem;           // [n] T' (stored form) in the a_lat order
  uint32_t* sF = sMem + n;       // [n] feasible keys in merged order
  uint32_t* sI = sMem + 2 * n;   // [n] infeasible keys in merged order
  const int64_t W = t.W[(int64_t)mode * t.n_ops + v];
  const int64_t ref = t.ref[v];
  int off[NHW + 1];
  int64_t q[NHW];
#pragma unroll
  for (int h = 0; h <= NHW; ++h) off[h] = t.seg_off[(int64_t)v * NHW + h] - a;
#pragma unroll
  for (int h = 0; h < NHW; ++h) q[h] = queue[h];
  auto seg_of = [&](int j) {
    int h = 0;
#pragma unroll
    for (int g = 1; g < NHW; ++g) h += j >= off[g] ? 1 : 0;
    return h;
  };
  for (int j = lane; j < n; j += 64) {
    const uint32_t T = remaining_time_threshold((uint32_t)t.a_lat[a + j], W, ref);
    const int h = seg_of(j);
    // R = clamp(r0 - Q, 0, 2^31 - 1) >= T >= 1 iff r0 >= T + Q: above
    // 2^31 - 1 no r0 reaches it, at or below -(2^31 - 1) every r0 does
    uint32_t Tq = TQ_NEVER;
    if (T != T_NEVER) {
      const int64_t qh = q[h] < -(4 * R0_MAX) ? -(4 * R0_MAX) : q[h] > 4 * R0_MAX ? 4 * R0_MAX : q[h];
      const int64_t x = (int64_t)T + qh;
      if (x <= R0_MAX) Tq = (uint32_t)((x < -R0_MAX ? -R0_MAX : x) + R0_MAX);
    }
    sT[j] = Tq;
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  __syncthreads();
  // position in the merged order: (T', backend) ascending; within a backend
  // the list order, which is ascending in T'
  for (int j = lane; j < n; j += 64) {
    const int h = seg_of(j);
    const uint32_t Tj = sT[j];
    int pos = j - off[h];
#pragma unroll
    for (int g = 0; g < NHW; ++g) {
      if (g == h) continue;
      int lo = off[g], hi = off[g + 1];
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const bool before = sT[mid] < Tj || (sT[mid] == Tj && g < h);
        if (before) lo = mid + 1; else hi = mid;
      }
      pos += lo - off[g];
    }
    t.aq_T[a + pos] = Tj;
    sF[pos] = t.a_fk[a + j];
    sI[pos] = t.a_ik[a + j];
  }
  __syncthreads();
  // prefix minima of the feasible keys, suffix minima of the infeasible keys
  uint32_t carry = KEY_NONE;
  for (int c0 = 0; c0 < n; c0 += 64) {
    const int j = c0 + lane;
    uint32_t x = j < n ? sF[j] : KEY_NONE;
    x = wave_min_scan(x, lane);
    x = x < carry ? x : carry;
    if (j < n) t.aq_pf[a + j] = x;
    carry = __shfl(x, 63, 64);
  }
  carry = KEY_NONE;
  for (int c1 = n; c1 > 0; c1 -= 64) {
    const int j = c1 - 64 + lane;  // lane 63 holds the chunk's last entry
    uint32_t x = j >= 0 ? sI[j] : KEY_NONE;
    x = wave_min_scan_rev(x, lane);
    x = x < carry ? x : carry;
    if (j >= 0) t.aq_si[a + j] = x;
    carry = __shfl(x, 0, 64);
  }
}

__global__ __launch_bounds__(256) void alpha_queue_kernel(DevTables t, Batch b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= b.n) return;
  const int v = b.op[i], e = b.elapsed[i], s = b.slo[i];
  if ((unsigned)v >= (unsigned)t.n_ops || (e | s) < 0) {
    b.cfg[i] = -1;
    if (b.flag) b.flag[i] = 0;
    atomicOr(t.err, 1u);
    return;
  }
  const uint32_t r0 = (uint32_t)((int64_t)s - e + R0_MAX);  // r0 on the stored scale
  const int lo0 = t.cfg_off[v], end = t.cfg_off[v + 1];
  int lo = lo0, len = end - lo0;
  for (int step = 0; step < t.m_steps && len > 0; ++step) {
    const int half = len >> 1;
    if (t.aq_T[lo + half] <= r0) {
      lo += half + 1;
      len -= half + 1;
    } else {
      len = half;
    }
  }
  uint32_t best = KEY_NONE;
  uint8_t meets = 0;
  if (lo > lo0) {
    best = t.aq_pf[lo - 1];
    meets = 1;
  }
  if (lo < end) {
    const uint32_t ki = t.aq_si[lo];
    if (ki < best) {
      best = ki;
      meets = 0;
    }
  }
  b.cfg[i] = (int)(best & 0xFFFFu);
  if (b.flag) b.flag[i] = meets;
}

}  // namespace

hipError_t launch_decide_alpha_queue(const DevTables& t, const Batch& b, hipStream_t s) {
  if (b.n == 0) return hipSuccess;
  if (!b.queue || t.alpha_max_op > ALPHA_MERGE_MAX || t.n_hw < 1 || t.n_hw > MAX_HW) return hipErrorInvalidValue;
  const size_t lds = sizeof(uint32_t) * 3 * (size_t)(t.alpha_max_op > 0 ? t.alpha_max_op : 1);
  if (t.n_ops > 0) {
    switch (t.n_hw) {
#define LLAMA_MERGE(K) \
  case K: hipLaunchKernelGGL(alpha_merge_kernel<K>, dim3(t.n_ops), dim3(64), lds, s, t, b.mode, b.queue); break;
      LLAMA_MERGE(1) LLAMA_MERGE(2) LLAMA_MERGE(3) LLAMA_MERGE(4)
      LLAMA_MERGE(5) LLAMA_MERGE(6) LLAMA_MERGE(7) LLAMA_MERGE(8)
#undef LLAMA_MERGE
      default: return hipErrorInvalidValue;
    }
  }
  const int64_t blocks = (b.n + 255) / 256;
  hipLaunchKernelGGL(alpha_queue_kernel, dim3((unsigned)blocks), dim3(256), 0, s, t, b);
  return hipGetLastError();
}

}  // namespace llama
