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
//   affinity_queue_kernel  Eq. 3 the same way (the merge also records, per
//                        merged position, each backend's entries before it)
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
    int before_g[NHW];  // entries of each backend before j in the merged order
#pragma unroll
    for (int g = 0; g < NHW; ++g) {
      if (g == h) {
        before_g[g] = j - off[h];
        continue;
      }
      int lo = off[g], hi = off[g + 1];
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const bool before = sT[mid] < Tj || (sT[mid] == Tj && g < h);
        if (before) lo = mid + 1; else hi = mid;
      }
      before_g[g] = lo - off[g];
    }
    int pos = 0;
#pragma unroll
    for (int g = 0; g < NHW; ++g) pos += before_g[g];
    t.aq_T[a + pos] = Tj;
    if (t.aq_cnt) {
#pragma unroll
      for (int g = 0; g < NHW; ++g) t.aq_cnt[(int64_t)(a + pos) * NHW + g] = (uint16_t)before_g[g];
    }
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

// Eq. 3 affinity: one search in a merged order gives j, the number of the
// op's feasible configurations (QUEUE: the per-call order, T + Q <= r0;
// otherwise every backend has the same target and the static latency order
// m_lat serves, L < target); the per-backend counts at j give, for each
// backend, how many of its configurations are feasible, which is exactly
// where the per-backend search in latency order ends, so the prefix and
// suffix minima of that order (a_ps) give each backend's best key.  The rest is the per-backend kernel's: the ratio of the
// objective values of the best key on the backend and the best elsewhere
// (no configuration on the backend -> 0; none elsewhere -> infinity; a zero
// own minimum -> infinity, or 1 when the other minimum is zero too), and with
// `keys` the sort keys for the commit order.
template <int NHW, bool QUEUE>
__global__ __launch_bounds__(256) void affinity_queue_kernel(DevTables t, Batch b, double* aff, uint64_t* keys,
                                                             int32_t* iota) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= b.n) return;
  if (iota) iota[i] = (int32_t)i;
  const int v = b.op[i], e = b.elapsed[i], s = b.slo[i];
  double out[NHW];
  if ((unsigned)v >= (unsigned)t.n_ops || (e | s) < 0) {
    atomicOr(t.err, 1u);
#pragma unroll
    for (int h = 0; h < NHW; ++h) out[h] = 0.0;
  } else {
    const int lo0 = t.cfg_off[v], end = t.cfg_off[v + 1];
    int lo = lo0, len = end - lo0;
    if (QUEUE) {
      const uint32_t r0 = (uint32_t)((int64_t)s - e + R0_MAX);  // r0 on the stored scale
      for (int step = 0; step < t.m_steps && len > 0; ++step) {
        const int half = len >> 1;
        if (t.aq_T[lo + half] <= r0) {
          lo += half + 1;
          len -= half + 1;
        } else {
          len = half;
        }
      }
    } else {
      // target = floor(ref * R / W), R = clamp(r0, 0, 2^31 - 1), 0 when R = 0
      const int64_t r0 = (int64_t)s - e;
      const int64_t R = r0 < 0 ? 0 : r0;
      const int32_t target =
          R == 0 ? 0 : (int32_t)floor_div((int64_t)t.ref[v] * R, t.W[(int64_t)b.mode * t.n_ops + v]);
      for (int step = 0; step < t.m_steps && len > 0; ++step) {
        const int half = len >> 1;
        if (t.m_lat[lo + half] < target) {
          lo += half + 1;
          len -= half + 1;
        } else {
          len = half;
        }
      }
    }
    const uint16_t* cnt = QUEUE ? t.aq_cnt : t.m_cnt;
    const int32_t* so = t.seg_off + (int64_t)v * NHW;
    uint32_t best[NHW];
#pragma unroll
    for (int h = 0; h < NHW; ++h) {
      const int feas = lo < end ? (int)cnt[(int64_t)lo * NHW + h] : so[h + 1] - so[h];
      const uint2 ps = t.a_ps[(int64_t)so[h] + feas + (int64_t)v * NHW + h];
      best[h] = ps.y < ps.x ? ps.y : ps.x;
    }
    const double* val = t.a_val + 2 * (int64_t)lo0;
#pragma unroll
    for (int h = 0; h < NHW; ++h) {
      uint32_t oth = KEY_NONE;
#pragma unroll
      for (int g = 0; g < NHW; ++g)
        if (g != h && best[g] < oth) oth = best[g];
      double a;
      if (best[h] == KEY_NONE) {
        a = 0.0;
      } else if (oth == KEY_NONE) {
        a = __builtin_huge_val();
      } else {
        const double vo = val[best[h] >> 16], vt = val[oth >> 16];
        a = vo == 0.0 ? (vt == 0.0 ? 1.0 : __builtin_huge_val()) : vt / vo;
      }
      out[h] = a;
    }
  }
  double* dst = aff + i * NHW;
#pragma unroll
  for (int h = 0; h < NHW; ++h) {
    dst[h] = out[h];
    // non-negative doubles order like their bit patterns; complemented, an
    // ascending sort gives decreasing affinity
    if (keys) keys[(int64_t)h * b.n + i] = ~(uint64_t)__double_as_longlong(out[h]);
  }
}

}  // namespace

namespace {

// The per-call merged order for this call's queueing times and slack mode.
hipError_t launch_alpha_merge(const DevTables& t, const Batch& b, hipStream_t s) {
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
  return hipGetLastError();
}

}  // namespace

hipError_t launch_affinity_queue(const DevTables& t, const Batch& b, double* aff, int32_t* order, void* scratch,
                                 size_t scratch_bytes, hipStream_t s) {
  if (b.n == 0) return hipSuccess;
  hipError_t e = hipSuccess;
  if (b.queue) {
    if (!t.aq_cnt) return hipErrorInvalidValue;
    e = launch_alpha_merge(t, b, s);
    if (e != hipSuccess) return e;
  } else if (!t.m_cnt) {
    return hipErrorInvalidValue;
  }
  const int64_t n = b.n;
  uint64_t* keys = order ? static_cast<uint64_t*>(scratch) : nullptr;  // [n_hw * n]
  uint64_t* kout = keys ? keys + (int64_t)t.n_hw * n : nullptr;          // [n]
  int32_t* iota = kout ? reinterpret_cast<int32_t*>(kout + n) : nullptr; // [n]
  const unsigned blocks = (unsigned)((n + 255) / 256);
  switch (t.n_hw) {
#define LLAMA_AFF(K)                                                                                      \
  case K:                                                                                                 \
    if (b.queue)                                                                                          \
      hipLaunchKernelGGL((affinity_queue_kernel<K, true>), dim3(blocks), dim3(256), 0, s, t, b, aff, keys, iota); \
    else                                                                                                  \
      hipLaunchKernelGGL((affinity_queue_kernel<K, false>), dim3(blocks), dim3(256), 0, s, t, b, aff, keys, iota); \
    break;
    LLAMA_AFF(1) LLAMA_AFF(2) LLAMA_AFF(3) LLAMA_AFF(4)
    LLAMA_AFF(5) LLAMA_AFF(6) LLAMA_AFF(7) LLAMA_AFF(8)
#undef LLAMA_AFF
    default: return hipErrorInvalidValue;
  }
  if (!order) return hipGetLastError();
  const size_t off = ((size_t)n * (8 * (size_t)t.n_hw + 8 + 4) + 255) & ~(size_t)255;
  if (scratch_bytes < off) return hipErrorInvalidValue;
  void* tmp = static_cast<char*>(scratch) + off;
  const size_t tmp_bytes = scratch_bytes - off;
  for (int h = 0; h < t.n_hw; ++h) {
    e = sort_pairs(tmp, tmp_bytes, keys + (int64_t)h * n, kout, iota, order + (int64_t)h * n, (int)n, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t launch_decide_alpha_queue(const DevTables& t, const Batch& b, hipStream_t s) {
  if (b.n == 0) return hipSuccess;
  hipError_t e = launch_alpha_merge(t, b, s);
  if (e != hipSuccess) return e;
  const int64_t blocks = (b.n + 255) / 256;
  hipLaunchKernelGGL(alpha_queue_kernel, dim3((unsigned)blocks), dim3(256), 0, s, t, b);
  return hipGetLastError();
}

}  // namespace llama
