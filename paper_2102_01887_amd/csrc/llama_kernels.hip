// HIP kernels (gfx950) of the decision path:
//   relax_kernel            remaining worst-path latency W (Alg. 1
//                           RemainingPathLatency, min over paths) and the
//                           per-frontier-entry remaining-time thresholds
//   targets_kernel          Alg. 1 slack per invocation and backend
//   select_indexed_kernel   Eq. 1 given slacks, on the cost/latency frontiers
//   decide_indexed_kernel   Alg. 1 + Eq. 1 fused, on the threshold frontiers
//   decide_full_kernel      Alg. 1 + Eq. 1 fused, scanning every configuration
//                           with a wavefront min reduction (DPP)
//
// Everything is integer.  Exact floor division of non-negative 64-bit values
// uses an FP64 quotient estimate followed by an exact integer correction.
#include <hip/hip_runtime.h>

#include "llama_internal.h"
#include "serve_device.h"

namespace llama {
namespace {

constexpr int64_t INT32_MAX_64 = 0x7FFFFFFFll;

// floor(a / b) for 0 <= a < 2^62 and 1 <= b < 2^62 when the quotient is
// below 2^32.  The FP64 estimate is within 2^-20 of a/b (three roundings of
// relative size 2^-53 on a quotient below 2^32), so truncating it is off by
// at most one; a single signed correction step with the exact remainder
// makes it exact.
__device__ __forceinline__ int64_t div_floor_pos(int64_t a, int64_t b) {
  int64_t q = (int64_t)((double)a / (double)b);
  int64_t r = a - q * b;
  if (r < 0) {
    q -= 1;
  } else if (r >= b) {
    q += 1;
  }
  return q;
}

// Remaining time of one backend, clamped to [0, 2^31-1].
__device__ __forceinline__ int64_t remaining_time(int64_t r0, int64_t queue) {
  int64_t r = r0 - queue;
  r = r < 0 ? 0 : r;
  return r > INT32_MAX_64 ? INT32_MAX_64 : r;
}

// Smallest remaining time R for which L < floor(ref * R / W), that is
// ceil((L + 1) * W / ref); THR_NEVER when that exceeds 2^31-1 (no clamped R
// reaches it).  Exact: (L+1)*W is compared with ref*(2^31-1) in 128 bits.
__device__ __forceinline__ uint32_t remaining_threshold(uint32_t L, int64_t W, int32_t ref) {
  const unsigned __int128 lhs = (unsigned __int128)((uint64_t)L + 1u) * (uint64_t)W;
  const uint64_t lim = (uint64_t)ref * (uint64_t)INT32_MAX_64;
  if (lhs > (unsigned __int128)lim) return THR_NEVER;
  const int64_t num = (int64_t)(uint64_t)lhs + ref - 1;
  return (uint32_t)div_floor_pos(num, ref);
}

// ---------------------------------------------------------------------------
// Relaxation: one workgroup per pipeline, levels from the outputs upward.
// When a pipeline fits the LDS stage (sized at launch for the largest one),
// its reference latencies and its edges, grouped by the level of their
// source, are staged in LDS and each level is one pass with a lane per edge
// that folds the successor's W into the source's accumulator by LDS atomic
// max (max is order-free, so the result is exact); otherwise the op-parallel
// form of the same recurrence runs on global memory.  op_records_kernel then
// writes the queue-free decision records, one thread per op.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t branch_discount(uint32_t q, int64_t w) {
  return (int64_t)(((uint64_t)q * (uint64_t)w) >> 16);
}

// Exact thresholds of one (op, slack mode).  The stored threshold of an
// entry with latency L is U = T - 1, T = ceil(y), y = (L + 1) * W / ref, or
// INT32_MAX when T > 2^31 - 1 (no remaining time reaches it).
//   * T > 2^31 - 1 iff (L + 1) * W > ref * (2^31 - 1) iff L + 1 > cutoff =
//     floor(ref * (2^31 - 1) / W), computed exactly once per op.
//   * Otherwise y < 2^31 and x = fl(fl(L + 1) * fl(fl(W) / ref)) carries three
//     roundings of relative size 2^-53, so |x - y| < 2^31 * 3 * 2^-53 < 2^-20.
//     When x is at least 2^-19 away from every integer, y is not an integer
//     and floor(y) = floor(x), so U = T - 1 = floor(x).  When W / ref is an
//     integer k (every output op has W = ref), x = y = (L + 1) * k exactly
//     and U = x - 1.
//   * Near an integer, the exact path: the numerator (L + 1) * W + ref - 1 is
//     below 2^62 and the quotient below 2^31, so an FP64 estimate is off by
//     at most one and one exact remainder step corrects it.
struct OpScale {
  uint32_t cut32;   // min(cutoff, 2^32 - 1); L + 1 <= 2^31 always
  bool int_scale;   // W / ref is an integer k: then x = (L + 1) * k exactly
  int64_t W;
  int64_t ref;
  double scale;     // fl(fl(W) / ref)
  double inv_ref;   // fl(1 / ref), for the exact path's quotient estimate
};

__device__ __forceinline__ OpScale op_scale(int64_t W, int32_t ref) {
  OpScale o;
  const uint64_t lim = (uint64_t)ref * (uint64_t)INT32_MAX_64;
  const uint64_t cutoff = ((unsigned __int128)(uint64_t)W << 32) <= (unsigned __int128)lim
                              ? 0xFFFFFFFFull
                              : (uint64_t)div_floor_pos((int64_t)lim, W);
  o.cut32 = (uint32_t)(cutoff < 0xFFFFFFFFull ? cutoff : 0xFFFFFFFFull);
  o.W = W;
  o.ref = ref;
  o.scale = (double)W / (double)ref;
  o.inv_ref = 1.0 / (double)ref;
  // W < 2^53, so an integer W / ref = k is represented exactly by scale;
  // a scale that only rounds to an integer fails k * ref == W
  const double k = floor(o.scale);
  o.int_scale = k == o.scale && (int64_t)k * (int64_t)ref == W;
  return o;
}

// The quotient estimate fl(fl(num) * fl(1 / ref)) carries three roundings of
// relative size 2^-53, so for quotients below 2^31 + 1 it is off by less than
// 2^-20 and its truncation by at most one; one remainder step corrects it.
__device__ __forceinline__ uint32_t entry_threshold_exact(const OpScale& o, uint32_t l1) {
  const int64_t num = (int64_t)((uint64_t)l1 * (uint64_t)o.W) + o.ref - 1;
  int64_t q = (int64_t)(uint32_t)((double)num * o.inv_ref);  // estimate below 2^31 + 1
  const int64_t r = num - q * o.ref;
  q += r < 0 ? -1 : (r >= o.ref ? 1 : 0);
  return (uint32_t)q - 1u;  // q = T >= 1
}

// Below the cutoff y = (L + 1) * W / ref < 2^31.  With an integer scale, x = y
// is an integer and T = y; otherwise x at least 2^-19 from every integer gives
// T - 1 = floor(x), and the exact path decides the rest (rare: x falls within
// 2^-19 of an integer).
__device__ __forceinline__ uint32_t entry_threshold(const OpScale& o, uint32_t L) {
  const uint32_t l1 = L + 1u;
  if (l1 > o.cut32) return 0x7FFFFFFFu;
  const double x = (double)l1 * o.scale;
  const double fl = floor(x);
  const double fr = x - fl;
  if (o.int_scale) return (uint32_t)fl - 1u;
  if (fr >= 0x1p-19 && fr <= 1.0 - 0x1p-19) return (uint32_t)fl;
  return entry_threshold_exact(o, l1);
}

// The thresholds of N entries (latencies L[k]) as entry_threshold computes
// them, without a branch per entry: the fast path of every entry first, so
// that the entries' FP64 chains overlap, then the exact path for the entries
// that need it (x within 2^-19 of an integer; rare).
template <int N>
__device__ __forceinline__ void entry_thresholds(const OpScale& o, const uint32_t (&L)[N], uint32_t (&U)[N]) {
  uint32_t slow = 0;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const uint32_t l1 = L[k] + 1u;
    const bool never = l1 > o.cut32;
    const double x = (double)l1 * o.scale;
    const double fl = floor(fmin(x, 2147483648.0));  // below 2^31 + 1 unless never
    const double fr = x - fl;
    const bool easy = o.int_scale || (fr >= 0x1p-19 && fr <= 1.0 - 0x1p-19);
    U[k] = never ? 0x7FFFFFFFu : (uint32_t)fl - (o.int_scale ? 1u : 0u);
    slow |= (!never && !easy) ? 1u << k : 0u;
  }
  if (slow) {
#pragma unroll
    for (int k = 0; k < N; ++k)
      if (slow & (1u << k)) U[k] = entry_threshold_exact(o, L[k] + 1u);
  }
}

// Queue-free records of op v, both slack modes.  The merged frontier of an
// op (which entries survive and their order) depends only on latencies,
// because every threshold of an op is the same increasing function of L;
// ingest fixes it in mst, and only the thresholds change with W.  Record
// words are assembled in registers and written as whole 16-byte chunks;
// entries past the record go to the overflow array, ascending.
// What an op's records need besides W: its merged-frontier range, overflow
// offset, fastest configuration, the REC_SLOTS entries of largest latency and
// the first OVF_PREFETCH entries past them (static between latency updates,
// so they can be loaded ahead of W).
constexpr int OVF_PREFETCH = 8;
struct OpStatic {
  int first, n, base;
  uint32_t fastest;
  uint2 e[REC_SLOTS];
  uint2 x[OVF_PREFETCH];
};

__device__ __forceinline__ OpStatic load_op_static(const DevTables& t, int v) {
  OpStatic o;
  o.first = t.cfg_off[v];
  o.n = t.mst_n[v];
  const int32_t* hdr = t.hdr + (int64_t)v * t.hs;
  o.base = hdr[0];
  o.fastest = (uint32_t)hdr[t.n_hw + 1];
  // unconditional loads (clamped index) so that they issue together; every
  // op has at least one entry (its fastest configuration)
#pragma unroll
  for (int slot = 0; slot < REC_SLOTS; ++slot) {
    const int j = o.n - 1 - slot;
    o.e[slot] = t.mst[o.first + (j > 0 ? j : 0)];
  }
  const int last = o.n - REC_SLOTS - 1;  // last overflow entry, < 0 if none
#pragma unroll
  for (int k = 0; k < OVF_PREFETCH; ++k) o.x[k] = make_uint2(0u, 0u);
  if (last >= 0) {
#pragma unroll
    for (int k = 0; k < OVF_PREFETCH; ++k) o.x[k] = t.mst[o.first + (k < last ? k : last)];
  }
  return o;
}

// Records of op v for one slack mode (W of that mode).
__device__ __forceinline__ void write_op_records(const DevTables& t, int v, const OpStatic& st, int32_t ref,
                                                 int64_t W, int mode) {
  const int n = st.n;
  if (n <= 0) return;
  const int n_ovf = n - REC_SLOTS;
  const OpScale o = op_scale(W, ref);
  uint32_t Ls[REC_SLOTS], Us[REC_SLOTS], Lx[OVF_PREFETCH], Ux[OVF_PREFETCH];
#pragma unroll
  for (int slot = 0; slot < REC_SLOTS; ++slot) Ls[slot] = st.e[slot].x;
#pragma unroll
  for (int k = 0; k < OVF_PREFETCH; ++k) Lx[k] = st.x[k].x;
  entry_thresholds<REC_SLOTS>(o, Ls, Us);
#pragma unroll
  for (int k = 0; k < OVF_PREFETCH; ++k) Ux[k] = 0u;
  if (n_ovf > 0) entry_thresholds<OVF_PREFETCH>(o, Lx, Ux);
  uint32_t w[REC_WORDS];
#pragma unroll
  for (int k = 0; k < REC_WORDS; ++k) w[k] = 0;
  // smallest U of the frontier: its fastest entry, the last slot when the
  // frontier ends inside the record (unused slots load entry 0), else the
  // first overflow entry
  const uint32_t u_last = n > REC_SLOTS ? Ux[0] : Us[REC_SLOTS - 1];
  w[0] = st.fastest | (rec_floor_code((int32_t)u_last) << 16);
  w[REC_N_WORD] = (uint32_t)n;
#pragma unroll
  for (int slot = 0; slot < REC_SLOTS; ++slot) {
    const bool used = slot < n;
    w[rec_u_word(slot)] = used ? Us[slot] : 0x7FFFFFFFu;
    w[rec_k_word(slot)] |= (used ? st.e[slot].y & 0xFFFFu : 0u) << rec_k_shift(slot);
  }
  const int64_t r = (int64_t)mode * t.n_ops + v;
  t.rec[r] = make_uint4(w[0], w[1], w[2], w[3]);
  uint4* tl = t.rec_tail + r * REC_TAIL_VECS;
  tl[0] = make_uint4(w[4], w[5], w[6], w[7]);
  tl[1] = make_uint4(w[8], w[9], w[10], w[11]);
  if (n > REC_SLOTS_TAIL) {
    uint4* t2 = t.rec_tail2 + r * REC_TAIL2_VECS;
    t2[0] = make_uint4(w[12], w[13], w[14], w[15]);
    t2[1] = make_uint4(w[16], w[17], w[18], w[19]);
    t2[2] = make_uint4(w[20], w[21], w[22], w[23]);
    t2[3] = make_uint4(w[24], w[25], w[26], w[27]);
  }
  // entries past the record, ascending: the prefetched ones, then four
  // loads in flight at a time
  uint2* ovf = t.ovf + (int64_t)mode * t.n_front + st.base;
#pragma unroll
  for (int k = 0; k < OVF_PREFETCH; ++k)
    if (k < n_ovf) ovf[k] = make_uint2(Ux[k], st.x[k].y);
  for (int pos = OVF_PREFETCH; pos < n_ovf; pos += 4) {
    uint2 x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = t.mst[st.first + (pos + u < n_ovf ? pos + u : n_ovf - 1)];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (pos + u >= n_ovf) break;
      ovf[pos + u] = make_uint2(entry_threshold(o, x[u].x), x[u].y);
    }
  }
}

// Bytes of dynamic LDS that relax_kernel needs for the given capacities:
// accumulators, reference latencies, edges and level bounds, and with
// RECORDS each op's static record inputs (16-byte aligned).
__host__ __device__ inline size_t relax_lds_core_bytes(int ops, int edges, int lvls) {
  const size_t b = sizeof(uint64_t) * 2 * (size_t)ops + sizeof(int32_t) * ((size_t)ops + 2 * (size_t)edges + (size_t)lvls + 1);
  return (b + 15) & ~(size_t)15;
}
size_t relax_lds_bytes(const DevTables& t, bool records) {
  return relax_lds_core_bytes(t.relax_ops, t.relax_edges, t.relax_lvls) +
         (records ? sizeof(OpStatic) * (size_t)t.relax_ops : 0);
}

// One edge of a level: fold the successor's W (reference latency rd plus its
// accumulators aP, aQ) into the source's accumulators, for both slack modes.
__device__ __forceinline__ void relax_edge(uint64_t* sAccP, uint64_t* sAccQ, uint32_t pk, uint32_t q, int32_t rd,
                                           uint64_t aP, uint64_t aQ) {
  const int src = (int)(pk & 0xFFFFu);
  const uint64_t wp = (uint64_t)(rd + (int64_t)aP);
  const uint64_t wq = (uint64_t)branch_discount(q, rd + (int64_t)aQ);
  atomicMax((unsigned long long*)&sAccP[src], (unsigned long long)wp);
  atomicMax((unsigned long long*)&sAccQ[src], (unsigned long long)wq);
}

// The level passes of a staged pipeline on one wavefront, lane = edge.  The
// next level's edges (static) are read together with the current level's
// successor values, so each level costs one round of LDS reads and one of
// atomics; LDS operations of a wavefront take effect in order, so the reads
// of a level see the maxima of the one before.  SMALL: at most 64 levels,
// every level bound in registers (lane l holds the first edge of level l and
// of level l + 1); otherwise bounds past level 63 come from LDS.
template <bool SMALL>
__device__ __forceinline__ void relax_levels(uint64_t* sAccP, uint64_t* sAccQ, const int32_t* sRef,
                                             const uint32_t* sE, const uint32_t* sEq, const int32_t* sEb, int nl,
                                             int lane) {
  const int eb0 = lane <= nl ? sEb[lane] : 0;
  const int eb1 = lane + 1 <= nl ? sEb[lane + 1] : 0;
  auto lvl_lo = [&](int l) { return SMALL || l < 64 ? __builtin_amdgcn_readlane(eb0, l) : sEb[l]; };
  auto lvl_hi = [&](int l) { return SMALL || l < 64 ? __builtin_amdgcn_readlane(eb1, l) : sEb[l + 1]; };
  // level 0 (the outputs) has no outgoing edges
  int lo = lvl_lo(1), hi = lvl_hi(1);
  bool act = lo + lane < hi;
  uint32_t pk = 0, q = 0;
  if (act) {
    pk = sE[lo + lane];
    q = sEq[lo + lane];
  }
  for (int l = 1; l < nl; ++l) {
    const bool more = l + 1 < nl;
    const int lo_n = more ? lvl_lo(l + 1) : 0, hi_n = more ? lvl_hi(l + 1) : 0;
    const bool act_n = more && lo_n + lane < hi_n;
    int32_t rd = 0;
    uint64_t aP = 0, aQ = 0;
    if (act) {
      const int dst = (int)(pk >> 16);
      rd = sRef[dst];
      aP = sAccP[dst];
      aQ = sAccQ[dst];
    }
    uint32_t pk_n = 0, q_n = 0;
    if (act_n) {
      pk_n = sE[lo_n + lane];
      q_n = sEq[lo_n + lane];
    }
    if (act) relax_edge(sAccP, sAccQ, pk, q, rd, aP, aQ);
    for (int idx = lo + 64 + lane; idx < hi; idx += 64) {  // levels wider than 64 edges
      const uint32_t pk2 = sE[idx];
      const int dst = (int)(pk2 >> 16);
      relax_edge(sAccP, sAccQ, pk2, sEq[idx], sRef[dst], sAccP[dst], sAccQ[dst]);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    pk = pk_n;
    q = q_n;
    act = act_n;
    lo = lo_n;
    hi = hi_n;
  }
}

// RECORDS: every pipeline has at most 64 ops and the workgroup has two
// wavefronts; wavefront m writes the records of slack mode m (lane i: the
// pipeline's op i).  A staged pipeline is staged and relaxed by wavefront 0
// alone, one lane per edge, while wavefront 1 loads the records' static
// inputs and hands them to wavefront 0 in LDS: the level bounds sit in
// registers and the next level's edges (static) are read from LDS while the
// current level's maxima are applied; LDS operations of one wavefront take
// effect in order, so wavefront-scope fences separate staging and levels.
template <bool RECORDS>
__global__ __launch_bounds__(128) void relax_kernel(DevTables t, int modes) {
  extern __shared__ uint64_t sDyn[];
  const int cap_ops = t.relax_ops, cap_edges = t.relax_edges, cap_lvls = t.relax_lvls;
  // W[v] = ref[v] + acc[v]: acc is the largest successor term, built level by
  // level with LDS atomic max over the edges of the level (one lane per edge)
  uint64_t* sAccP = sDyn;
  uint64_t* sAccQ = sAccP + cap_ops;
  int32_t* sRef = reinterpret_cast<int32_t*>(sAccQ + cap_ops);  // cap_ops
  uint32_t* sE = reinterpret_cast<uint32_t*>(sRef + cap_ops);    // cap_edges
  uint32_t* sEq = sE + cap_edges;                                // cap_edges
  int32_t* sEb = reinterpret_cast<int32_t*>(sEq + cap_edges);     // cap_lvls + 1
  const int p = blockIdx.x;
  const int tid = threadIdx.x, bs = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int n_ops = t.n_ops;
  const int4 d0 = t.pipe_desc[2 * p], d1 = t.pipe_desc[2 * p + 1];
  const int a = d0.x, n = d0.y, e0 = d0.z, ne = d0.w;
  const int l0 = d1.x, nl = d1.y;
  int64_t* WP = t.W;
  int64_t* WQ = t.W + n_ops;
  OpStatic st;
  const bool staged = n <= cap_ops && ne <= cap_edges && nl <= cap_lvls;
  if (staged) {
    OpStatic* sSt = reinterpret_cast<OpStatic*>(reinterpret_cast<char*>(sDyn) +
                                                relax_lds_core_bytes(cap_ops, cap_edges, cap_lvls));
    if (RECORDS && wave == 1) {
      // wavefront 1 loads the static record inputs while wavefront 0 relaxes
      if (lane < n) {
        st = load_op_static(t, a + lane);
        sSt[lane] = st;
      }
    } else {
      // wavefront 0 stages the pipeline: RELAX_BATCH loads per lane in
      // flight (clamped indices, so the loads are unconditional and issue
      // together)
      constexpr int RELAX_BATCH = 8;
      for (int i0 = 0; i0 < n; i0 += RELAX_BATCH * 64) {
        int r[RELAX_BATCH];
#pragma unroll
        for (int u = 0; u < RELAX_BATCH; ++u) {
          const int i = i0 + u * 64 + lane;
          r[u] = t.ref[a + (i < n ? i : n - 1)];
        }
#pragma unroll
        for (int u = 0; u < RELAX_BATCH; ++u) {
          const int i = i0 + u * 64 + lane;
          if (i < n) {
            sRef[i] = r[u];
            sAccP[i] = 0;
            sAccQ[i] = 0;
          }
        }
      }
      for (int i0 = 0; i0 < ne; i0 += RELAX_BATCH * 64) {
        uint32_t pk[RELAX_BATCH], q[RELAX_BATCH];
#pragma unroll
        for (int u = 0; u < RELAX_BATCH; ++u) {
          const int i = i0 + u * 64 + lane;
          const int g = e0 + (i < ne ? i : ne - 1);
          pk[u] = t.lvl_edge[g];
          q[u] = t.lvl_edge_q[g];
        }
#pragma unroll
        for (int u = 0; u < RELAX_BATCH; ++u) {
          const int i = i0 + u * 64 + lane;
          if (i < ne) {
            sE[i] = pk[u];
            sEq[i] = q[u];
          }
        }
      }
      for (int i = lane; i <= nl; i += 64) sEb[i] = t.lvl_ebnd[l0 + i] - e0;
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      if (nl > 64)
        relax_levels<false>(sAccP, sAccQ, sRef, sE, sEq, sEb, nl, lane);
      else if (nl > 1)
        relax_levels<true>(sAccP, sAccQ, sRef, sE, sEq, sEb, nl, lane);
    }
    __syncthreads();
    if (RECORDS) {
      if (lane < n) {
        if (wave == 0) st = sSt[lane];
        const int64_t W = sRef[lane] + (int64_t)(wave ? sAccQ[lane] : sAccP[lane]);
        t.W[(int64_t)wave * n_ops + a + lane] = W;
        if ((modes >> wave) & 1) write_op_records(t, a + lane, st, sRef[lane], W, wave);
      }
    } else {
      for (int i = tid; i < n; i += bs) {
        WP[a + i] = sRef[i] + (int64_t)sAccP[i];
        WQ[a + i] = sRef[i] + (int64_t)sAccQ[i];
      }
    }
    return;
  }
  if (RECORDS && lane < n) st = load_op_static(t, a + lane);
  for (int l = l0; l < l0 + nl; ++l) {
    const int end = t.lvl_bnd[l + 1];
    for (int idx = t.lvl_bnd[l] + tid; idx < end; idx += bs) {
      const int v = t.lvl_ops[idx];
      int64_t mp = 0, mq = 0;
      for (int e = t.succ_off[v]; e < t.succ_off[v + 1]; ++e) {
        const int w = t.succ_ids[e];
        const int64_t wp = WP[w], wq = branch_discount(t.succ_q[e], WQ[w]);
        mp = wp > mp ? wp : mp;
        mq = wq > mq ? wq : mq;
      }
      const int64_t r = t.ref[v];
      WP[v] = r + mp;
      WQ[v] = r + mq;
    }
    __syncthreads();
  }
  if (RECORDS && lane < n && ((modes >> wave) & 1))
    write_op_records(t, a + lane, st, t.ref[a + lane], t.W[(int64_t)wave * n_ops + a + lane], wave);
}

// One thread per (op, slack mode) for both modes (modes = 3), else one
// thread per op for the one mode asked for: its records from the relaxed W.
__global__ __launch_bounds__(256) void op_records_kernel(DevTables t, int modes) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool both = modes == 3;
  if (i >= (both ? 2 : 1) * (int64_t)t.n_ops) return;
  const int v = both ? (int)(i >> 1) : (int)i;
  const int mode = both ? (int)(i & 1) : (modes >> 1);
  const OpStatic st = load_op_static(t, v);
  write_op_records(t, v, st, t.ref[v], t.W[(int64_t)mode * t.n_ops + v], mode);
}

// ---------------------------------------------------------------------------
// Decision records: one 64-lane workgroup per (op, slack mode).
//   1. every frontier entry {L, key} of backend h gets its remaining-time
//      threshold T = ceil((L+1) * W / ref) + queue[h] (lanes in parallel, LDS);
//   2. an entry survives the merge of the backends' lists iff its key is below
//      the key of every entry that precedes it in (T, key) order; within its
//      own list that always holds, and in another list the predecessors form a
//      prefix whose smallest key is its last one (binary search in LDS);
//   3. a prefix count of survivors gives each survivor its position in the
//      merged frontier, written ascending to the overflow array; the
//      REC_SLOTS largest-T entries also go to the record, descending.
// Frontiers longer than the LDS stage are merged serially by lane 0.
// ---------------------------------------------------------------------------
constexpr int REC_LDS = 512;
constexpr int BUCKET_CHUNK = 16384;  // invocations per histogram chunk
constexpr int BUCKET_LDS_OPS = 12288;  // ops countable in one LDS histogram (48 KB)
constexpr int64_t T_INF = 0x7FFFFFFFFFFFFFFFll;

// Stored form of a remaining-time threshold T: U = T - 1, clamped at
// INT32_MIN, so that "feasible iff slo - elapsed >= T" reads "U < r0" and
// U = INT32_MAX can mean "never" (no r0 exceeds it).
__device__ __forceinline__ int32_t stored_threshold(int64_t T) {
  const int64_t U = T - 1;
  return U < -INT32_MAX_64 - 1 ? (int32_t)(-INT32_MAX_64 - 1) : (int32_t)U;
}

__device__ __forceinline__ int wave_inclusive_scan(int x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

template <int NHW>
__device__ __forceinline__ void build_record(const DevTables& t, int v, int mode, const int64_t* queue,
                                             uint4* rec_hot, uint4* rec_tail, uint4* rec_tail2, int64_t rec_index, uint2* ovf,
                                             int64_t* sT, uint32_t* sK,
                                             int32_t* sC, uint32_t* sSlotT, uint32_t* sSlotK,
                                             int32_t* sN, uint32_t* sLast) {
  const int lane = threadIdx.x;
  const int32_t* hdr = t.hdr + (int64_t)v * t.hs;
  int off[NHW + 1];
#pragma unroll
  for (int h = 0; h <= NHW; ++h) off[h] = hdr[h];
  const int base = off[0], n_e = off[NHW] - base;
  const int64_t W = t.W[(int64_t)mode * t.n_ops + v];
  const int32_t ref = t.ref[v];
  int64_t Qh[NHW];
#pragma unroll
  for (int h = 0; h < NHW; ++h) Qh[h] = queue ? queue[h] : 0;
  auto threshold = [&](int j, int h) -> int64_t {  // j: absolute frontier index
    const uint32_t thr = remaining_threshold(t.front_L[j].x, W, ref);
    return thr == THR_NEVER ? T_INF : (int64_t)thr + Qh[h];
  };
  auto list_of = [&](int j) -> int {  // j: index relative to base
    int h = 0;
#pragma unroll
    for (int g = 1; g < NHW; ++g) h += (base + j >= off[g]) ? 1 : 0;
    return h;
  };

  if (n_e <= REC_LDS) {
    for (int j = lane; j < n_e; j += 64) {
      sT[j] = threshold(base + j, list_of(j));
      sK[j] = t.front_L[base + j].y;
    }
    __syncthreads();
    // number of entries of list g that precede (Tj, Kj)
    auto preceding = [&](int g, int64_t Tj, uint32_t Kj) -> int {
      int lo = off[g] - base, hi = off[g + 1] - base;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const bool before = sT[mid] < Tj || (sT[mid] == Tj && sK[mid] < Kj);
        if (before) lo = mid + 1; else hi = mid;
      }
      return lo;
    };
    for (int j = lane; j < n_e; j += 64) {
      const int h = list_of(j);
      const int64_t Tj = sT[j];
      const uint32_t Kj = sK[j];
      bool surv = Tj <= INT32_MAX_64;
      if (surv) {
#pragma unroll
        for (int g = 0; g < NHW; ++g) {
          if (g == h) continue;
          const int p = preceding(g, Tj, Kj);
          if (p > off[g] - base && sK[p - 1] < Kj) surv = false;
        }
      }
      sC[j] = surv ? 1 : 0;
    }
    __syncthreads();
    {  // inclusive prefix count of survivors, one contiguous chunk per lane
      const int c = (n_e + 63) / 64;
      const int a0 = lane * c < n_e ? lane * c : n_e;
      const int a1 = a0 + c < n_e ? a0 + c : n_e;
      int sum = 0;
      for (int j = a0; j < a1; ++j) sum += sC[j];
      int run = wave_inclusive_scan(sum) - sum;
      for (int j = a0; j < a1; ++j) {
        run += sC[j];
        sC[j] = run;
      }
    }
    __syncthreads();
    const int n = n_e > 0 ? sC[n_e - 1] : 0;
    auto count_before = [&](int idx) -> int { return idx > 0 ? sC[idx - 1] : 0; };
    for (int j = lane; j < n_e; j += 64) {
      if (sC[j] == count_before(j)) continue;  // not a survivor
      const int h = list_of(j);
      const int64_t Tj = sT[j];
      const uint32_t Kj = sK[j];
      int pos = count_before(j) - count_before(off[h] - base);
#pragma unroll
      for (int g = 0; g < NHW; ++g) {
        if (g == h) continue;
        pos += count_before(preceding(g, Tj, Kj)) - count_before(off[g] - base);
      }
      const int32_t Tc = stored_threshold(Tj);
      ovf[base + pos] = make_uint2((uint32_t)Tc, Kj);
      if (pos == 0) *sLast = (uint32_t)Tc;
      const int slot = n - 1 - pos;
      if (slot < REC_SLOTS) {
        sSlotT[slot] = (uint32_t)Tc;
        sSlotK[slot] = Kj & 0xFFFFu;
      }
    }
    if (lane == 0) *sN = n;
  } else if (lane == 0) {
    // serial merge of the backends' lists (each ascending in T)
    int pos[NHW];
    int64_t hT[NHW];
    uint32_t hK[NHW];
#pragma unroll
    for (int h = 0; h < NHW; ++h) {
      pos[h] = off[h];
      hT[h] = pos[h] < off[h + 1] ? threshold(pos[h], h) : T_INF;
      hK[h] = pos[h] < off[h + 1] ? t.front_L[pos[h]].y : KEY_NONE;
    }
    uint32_t best = KEY_NONE;
    int n = 0;
    for (;;) {
      int sel = 0;
      int64_t tmin = hT[0];
      uint32_t kmin = hK[0];
#pragma unroll
      for (int h = 1; h < NHW; ++h)
        if (hT[h] < tmin || (hT[h] == tmin && hK[h] < kmin)) {
          sel = h;
          tmin = hT[h];
          kmin = hK[h];
        }
      if (tmin > INT32_MAX_64) break;
      if (kmin < best) {
        best = kmin;
        ovf[base + n] = make_uint2((uint32_t)stored_threshold(tmin), kmin);
        ++n;
      }
#pragma unroll
      for (int h = 0; h < NHW; ++h)
        if (h == sel) {
          ++pos[h];
          hT[h] = pos[h] < off[h + 1] ? threshold(pos[h], h) : T_INF;
          hK[h] = pos[h] < off[h + 1] ? t.front_L[pos[h]].y : KEY_NONE;
        }
    }
    for (int s = 0; s < REC_SLOTS && s < n; ++s) {
      const uint2 f = ovf[base + n - 1 - s];
      sSlotT[s] = f.x;
      sSlotK[s] = f.y & 0xFFFFu;
    }
    if (n > 0) *sLast = ovf[base].x;
    *sN = n;
  }
  __syncthreads();
  if (lane < REC_WORDS) {
    const int n = *sN;
    uint32_t word = 0;
    // with no entry at all, every invocation falls back: the largest code
    const uint32_t u_last = n > 0 ? *sLast : 0x7FFFFFFFu;
    if (lane == 0) word = (uint32_t)hdr[NHW + 1] | (rec_floor_code((int32_t)u_last) << 16);
    if (lane == REC_N_WORD) word = (uint32_t)n;
#pragma unroll
    for (int slot = 0; slot < REC_SLOTS; ++slot) {
      if (lane == rec_u_word(slot)) word = slot < n ? sSlotT[slot] : 0x7FFFFFFFu;
      if (lane == rec_k_word(slot) && slot < n) word |= sSlotK[slot] << rec_k_shift(slot);
    }
    *rec_word(rec_hot, rec_tail, rec_tail2, rec_index, lane) = word;
  }
  __syncthreads();  // the LDS stage is reused by the next record
}

// One 64-lane workgroup per op; it builds the op's records for n_modes slack
// modes in turn (the frontier entries stay hot in cache between modes).
template <int NHW>
__global__ __launch_bounds__(64) void records_kernel(DevTables t, int mode0, int n_modes, const int64_t* queue,
                                                     uint4* rec_all, uint4* tail_all, uint4* tail2_all, uint2* ovf_all) {
  __shared__ int64_t sT[REC_LDS];
  __shared__ uint32_t sK[REC_LDS];
  __shared__ int32_t sC[REC_LDS];
  __shared__ uint32_t sSlotT[REC_SLOTS], sSlotK[REC_SLOTS];
  __shared__ int32_t sN;
  __shared__ uint32_t sLast;
  const int v = blockIdx.x;
  for (int m = 0; m < n_modes; ++m)
    build_record<NHW>(t, v, mode0 + m, queue, rec_all, tail_all, tail2_all, (int64_t)m * t.n_ops + v,
                      ovf_all + (int64_t)m * t.n_front, sT, sK, sC, sSlotT, sSlotK, &sN, &sLast);
}

__device__ __forceinline__ bool invalid_invocation(int v, int e, int s, int n_ops) {
  return (unsigned)v >= (unsigned)n_ops || (e | s) < 0;
}

// ---------------------------------------------------------------------------
// Targets: one invocation per lane.
// ---------------------------------------------------------------------------
template <int NHW>
__global__ __launch_bounds__(256) void targets_kernel(DevTables t, Batch b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= b.n) return;
  const int v = b.op[i], e = b.elapsed[i], s = b.slo[i];
  int32_t out[NHW];
  if (invalid_invocation(v, e, s, t.n_ops)) {
#pragma unroll
    for (int h = 0; h < NHW; ++h) out[h] = -1;
    atomicOr(t.err, 1u);
  } else {
    const int64_t r0 = (int64_t)s - e;
    const int64_t ref = t.ref[v];
    const int64_t W = t.W[(int64_t)b.mode * t.n_ops + v];
#pragma unroll
    for (int h = 0; h < NHW; ++h) {
      const int64_t R = remaining_time(r0, b.queue ? b.queue[h] : 0);
      out[h] = R == 0 ? 0 : (int32_t)div_floor_pos(ref * R, W);
    }
  }
  int32_t* dst = b.target_out + i * NHW;
#pragma unroll
  for (int h = 0; h < NHW; ++h) dst[h] = out[h];
}

// Last entry of a frontier segment [lo, hi) whose first word passes `ok`;
// returns its key or KEY_NONE.  Entries are ordered so that `ok` holds on a
// prefix.
template <typename Pred>
__device__ __forceinline__ uint32_t frontier_key(const uint2* f, int lo, int hi, Pred ok) {
  const int base = lo;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (ok(f[mid].x)) lo = mid + 1; else hi = mid;
  }
  return lo > base ? f[lo - 1].y : KEY_NONE;
}

__device__ __forceinline__ void write_choice(const Batch& b, int64_t i, uint32_t best, int fastest) {
  const bool feasible = best != KEY_NONE;
  b.cfg[i] = feasible ? (int32_t)(best & 0xFFFFu) : fastest;
  if (b.flag) b.flag[i] = feasible ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Eq. 1 given slacks: feasible iff L < target[hw]; on each (op, backend)
// frontier the feasible entries are a prefix and the last one has the
// smallest key.
// ---------------------------------------------------------------------------
template <int NHW>
__global__ __launch_bounds__(256) void select_indexed_kernel(DevTables t, Batch b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= b.n) return;
  const int v = b.op[i];
  if ((unsigned)v >= (unsigned)t.n_ops) {
    b.cfg[i] = -1;
    if (b.flag) b.flag[i] = 0;
    atomicOr(t.err, 1u);
    return;
  }
  const int32_t* hdr = t.hdr + (int64_t)v * t.hs;
  const int32_t* tg = b.target + i * NHW;
  uint32_t best = KEY_NONE;
#pragma unroll
  for (int h = 0; h < NHW; ++h) {
    const int32_t target = tg[h];
    const uint32_t k = frontier_key(t.front_L, hdr[h], hdr[h + 1],
                                    [target](uint32_t L) { return (int32_t)L < target; });
    best = k < best ? k : best;
  }
  write_choice(b, i, best, hdr[NHW + 1]);
}

// ---------------------------------------------------------------------------
// Alg. 1 + Eq. 1 fused on the decision records: a configuration is feasible
// iff slo - elapsed >= T (stored as U = T - 1 < r0), so each invocation reads its op's 64-byte record
// (four 16-byte loads of one line) and takes the first feasible slot in
// descending-T order, which is the cheapest feasible configuration; no
// division and no data-dependent branch unless the frontier continues past
// the record.
// ---------------------------------------------------------------------------

// Choice from the first tail (slots 2..6; unused slots never feasible): the
// first feasible slot in descending-T order, -1 if none; *n_out = frontier
// length.
__device__ __forceinline__ int tail_choice(const uint4& a, const uint4& bq, int32_t r0, int* n_out) {
  const uint32_t U[REC_SLOTS_TAIL - 2] = {a.w, bq.x, bq.y, bq.z, bq.w};
  const uint32_t K[REC_SLOTS_TAIL - 2] = {a.x >> 16, a.y & 0xFFFFu, a.y >> 16, a.z & 0xFFFFu, a.z >> 16};
  int sel = -1;
#pragma unroll
  for (int s = REC_SLOTS_TAIL - 3; s >= 0; --s)
    if ((int32_t)U[s] < r0) sel = (int)K[s];
  *n_out = (int)(a.x & 0xFFFFu);
  return sel;
}

// The same over the second tail (slots 7..16; n = frontier length).
__device__ __forceinline__ int record_choice2(const uint4& a, const uint4& bq, const uint4& c, const uint4& d, int n,
                                              int32_t r0) {
  const uint32_t U[REC_SLOTS - REC_SLOTS_TAIL] = {a.x, a.y, a.z, a.w, bq.x, bq.y, bq.z, bq.w, c.x, c.y};
  const uint32_t K2[(REC_SLOTS - REC_SLOTS_TAIL) / 2] = {c.z, c.w, d.x, d.y, d.z};
  int sel = -1;
#pragma unroll
  for (int s = REC_SLOTS - REC_SLOTS_TAIL - 1; s >= 0; --s) {
    const int k = (int)((K2[s >> 1] >> (16 * (s & 1))) & 0xFFFFu);
    if (REC_SLOTS_TAIL + s < n && (int32_t)U[s] < r0) sel = k;
  }
  return sel;
}

// The rest of the decision once the record's slots are known: overflow
// search when the frontier continues past the record, else the fallback.
__device__ __forceinline__ int finish_choice(const DevTables& t, const uint2* ovf, int v, int sel, int n,
                                             int32_t r0) {
  if (sel < 0 && n > REC_SLOTS) {
    // every slot needs more time: search the rest of the frontier (ascending)
    const int lo0 = t.hdr[(int64_t)v * t.hs];
    int lo = lo0, hi = lo0 + n - REC_SLOTS;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if ((int32_t)ovf[mid].x < r0) lo = mid + 1; else hi = mid;
    }
    if (lo > lo0) sel = (int)(ovf[lo - 1].y & 0xFFFFu);
  }
  return sel;
}

// Decision from the hot record words h.  The tail is read only when neither
// of the two cheapest entries is affordable and slo - elapsed exceeds the
// rounded-down smallest threshold (at or below it nothing is feasible: the
// fastest configuration, flag 0); the second tail only when no slot of the
// first is and the frontier is longer.
__device__ __forceinline__ int decide_from_record(const DevTables& t, const uint4* tail, const uint4* tail2,
                                                  const uint2* ovf, int v, const uint4& h, int32_t r0,
                                                  uint8_t* feasible) {
  int sel = -1;
  if ((int32_t)h.z < r0) sel = (int)(h.w >> 16);
  if ((int32_t)h.y < r0) sel = (int)(h.w & 0xFFFFu);
  if (sel < 0 && r0 > rec_code_value(h.x >> 16)) {
    const uint4* r = tail + (int64_t)v * REC_TAIL_VECS;
    int n;
    sel = tail_choice(r[0], r[1], r0, &n);
    if (sel < 0 && n > REC_SLOTS_TAIL) {
      const uint4* r2 = tail2 + (int64_t)v * REC_TAIL2_VECS;
      sel = record_choice2(r2[0], r2[1], r2[2], r2[3], n, r0);
      sel = finish_choice(t, ovf, v, sel, n, r0);
    }
  }
  *feasible = sel >= 0 ? 1 : 0;
  return sel >= 0 ? sel : (int)(h.x & 0xFFFFu);
}

// With NT the decision is stored with the non-temporal hint as well, so that
// the output stream need not displace decision records in L2 either.
template <bool NT = false>
__device__ __forceinline__ void store_decision(const Batch& b, int64_t i, int cfg, uint8_t feasible) {
  if (NT) {
    __builtin_nontemporal_store(cfg, b.cfg + i);
    if (b.flag) __builtin_nontemporal_store(feasible, b.flag + i);
  } else {
    b.cfg[i] = cfg;
    if (b.flag) b.flag[i] = feasible;
  }
}


// The invocation stream is read once; with NT its loads carry the
// non-temporal hint, so that they need not displace decision records in L2.
template <bool NT>
__device__ __forceinline__ void load_invocation(const Batch& b, int64_t i, int* v, int* e, int* s) {
  const bool in = i < b.n;
  if (NT) {
    *v = in ? __builtin_nontemporal_load(b.op + i) : 0;
    *e = in ? __builtin_nontemporal_load(b.elapsed + i) : 0;
    *s = in ? __builtin_nontemporal_load(b.slo + i) : 0;
  } else {
    *v = in ? b.op[i] : 0;
    *e = in ? b.elapsed[i] : 0;
    *s = in ? b.slo[i] : 0;
  }
}

// DECIDE_IPT = invocations per thread (a schedule parameter chosen by the
// autotuner): each thread decides DECIDE_IPT invocations spaced by the block
// size, so every load instruction stays coalesced, and issues all loads first.
template <int DECIDE_IPT, bool NT>
__global__ __launch_bounds__(256) void decide_indexed_kernel(DevTables t, Batch b, const uint4* rec,
                                                             const uint4* tail, const uint4* tail2,
                                                             const uint2* ovf) {
  const int64_t base = (int64_t)blockIdx.x * blockDim.x * DECIDE_IPT + threadIdx.x;
  int v[DECIDE_IPT], e[DECIDE_IPT], s[DECIDE_IPT];
#pragma unroll
  for (int u = 0; u < DECIDE_IPT; ++u) load_invocation<NT>(b, base + (int64_t)u * blockDim.x, &v[u], &e[u], &s[u]);
  uint4 h[DECIDE_IPT];
  bool ok[DECIDE_IPT];
#pragma unroll
  for (int u = 0; u < DECIDE_IPT; ++u) {
    ok[u] = !invalid_invocation(v[u], e[u], s[u], t.n_ops);
    h[u] = rec[ok[u] ? v[u] : 0];
  }
#pragma unroll
  for (int u = 0; u < DECIDE_IPT; ++u) {
    const int64_t i = base + (int64_t)u * blockDim.x;
    if (i >= b.n) continue;
    if (!ok[u]) {
      store_decision<NT>(b, i, -1, 0);
      atomicOr(t.err, 1u);
      continue;
    }
    const int32_t r0 = s[u] - e[u];  // both non-negative: no overflow
    uint8_t f;
    const int c = decide_from_record(t, tail, tail2, ovf, v[u], h[u], r0, &f);
    store_decision<NT>(b, i, c, f);
  }
}

// Persistent variant: every workgroup first stages the first 16 bytes of
// every op's record (header, the two cheapest thresholds and their
// configurations) in LDS; an invocation that can afford one of those two is
// decided from LDS, any other reads its full record from global memory.
__global__ __launch_bounds__(1024) void decide_lds_kernel(DevTables t, Batch b, const uint4* rec,
                                                         const uint4* tail, const uint4* tail2, const uint2* ovf) {
  extern __shared__ uint4 sRec[];
  for (int v = threadIdx.x; v < t.n_ops; v += blockDim.x) sRec[v] = rec[v];
  __syncthreads();
  constexpr int IPT = 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * IPT;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x * IPT + threadIdx.x; base < b.n; base += stride) {
    int v[IPT], e[IPT], s[IPT];
#pragma unroll
    for (int u = 0; u < IPT; ++u) load_invocation<false>(b, base + (int64_t)u * blockDim.x, &v[u], &e[u], &s[u]);
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      const int64_t i = base + (int64_t)u * blockDim.x;
      if (i >= b.n) continue;
      if (invalid_invocation(v[u], e[u], s[u], t.n_ops)) {
        store_decision(b, i, -1, 0);
        atomicOr(t.err, 1u);
        continue;
      }
      uint8_t f;
      const int c = decide_from_record(t, tail, tail2, ovf, v[u], sRec[v[u]], s[u] - e[u], &f);
      store_decision(b, i, c, f);
    }
  }
}

// The persistent variant for 16-byte aligned invocation arrays: each thread
// decides four consecutive invocations, read with one 16-byte load per array
// and written with one 16-byte store of configurations and one 4-byte store
// of flags, which cuts the memory instructions of the invocation stream to a
// quarter.  The last n mod 4 invocations are decided by block 0.
__global__ __launch_bounds__(1024) void decide_lds4_kernel(DevTables t, Batch b, const uint4* rec,
                                                          const uint4* tail, const uint4* tail2, const uint2* ovf) {
  extern __shared__ uint4 sRec[];
  const int64_t n4 = b.n >> 2;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int4* op4 = reinterpret_cast<const int4*>(b.op);
  const int4* el4 = reinterpret_cast<const int4*>(b.elapsed);
  const int4* slo4 = reinterpret_cast<const int4*>(b.slo);
  int4 v4 = make_int4(0, 0, 0, 0), e4 = v4, s4 = v4;
  if (q < n4) {  // the first invocations are loaded before the staging
    v4 = op4[q];
    e4 = el4[q];
    s4 = slo4[q];
  }
  for (int k = threadIdx.x; k < t.n_ops; k += blockDim.x) sRec[k] = rec[k];
  __syncthreads();
  for (; q < n4; q += stride) {
    const int v[4] = {v4.x, v4.y, v4.z, v4.w}, e[4] = {e4.x, e4.y, e4.z, e4.w};
    const int sl[4] = {s4.x, s4.y, s4.z, s4.w};
    int c[4];
    uint32_t flags = 0;
    bool bad = false;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (invalid_invocation(v[u], e[u], sl[u], t.n_ops)) {
        c[u] = -1;
        bad = true;
        continue;
      }
      uint8_t f;
      c[u] = decide_from_record(t, tail, tail2, ovf, v[u], sRec[v[u]], sl[u] - e[u], &f);
      flags |= (uint32_t)f << (8 * u);
    }
    reinterpret_cast<int4*>(b.cfg)[q] = make_int4(c[0], c[1], c[2], c[3]);
    if (b.flag) reinterpret_cast<uint32_t*>(b.flag)[q] = flags;
    if (bad) atomicOr(t.err, 1u);
    const int64_t nq = q + stride;
    if (nq < n4) {
      v4 = op4[nq];
      e4 = el4[nq];
      s4 = slo4[nq];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x < (b.n & 3)) {
    const int64_t i = (n4 << 2) + threadIdx.x;
    const int v = b.op[i], e = b.elapsed[i], sl = b.slo[i];
    if (invalid_invocation(v, e, sl, t.n_ops)) {
      store_decision(b, i, -1, 0);
      atomicOr(t.err, 1u);
    } else {
      uint8_t f;
      const int c = decide_from_record(t, tail, tail2, ovf, v, sRec[v], sl - e, &f);
      store_decision(b, i, c, f);
    }
  }
}

#define LLAMA_DISPATCH_NHW(KERNEL, GRID, BLOCK, STREAM, ...)                         \
  switch (t.n_hw) {                                                                  \
    case 1: hipLaunchKernelGGL(KERNEL<1>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); break; \
    case 2: hipLaunchKernelGGL(KERNEL<2>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); break; \
    case 3: hipLaunchKernelGGL(KERNEL<3>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); break; \
    case 4: hipLaunchKernelGGL(KERNEL<4>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); break; \
    case 5: hipLaunchKernelGGL(KERNEL<5>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); break; \
    case 6: hipLaunchKernelGGL(KERNEL<6>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); break; \
    case 7: hipLaunchKernelGGL(KERNEL<7>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); break; \
    case 8: hipLaunchKernelGGL(KERNEL<8>, GRID, BLOCK, 0, STREAM, __VA_ARGS__); break; \
    default: return hipErrorInvalidValue;                                            \
  }

inline unsigned blocks_for(int64_t n, int per_block) {
  return (unsigned)((n + per_block - 1) / per_block);
}

}  // namespace

hipError_t launch_records(const DevTables& t, int mode0, int n_modes, const int64_t* queue, uint4* rec,
                          uint4* rec_tail, uint4* rec_tail2, uint2* ovf, hipStream_t s) {
  if (t.n_ops <= 0) return hipSuccess;
  LLAMA_DISPATCH_NHW(records_kernel, dim3(t.n_ops), dim3(64), s, t, mode0, n_modes, queue, rec, rec_tail, rec_tail2,
                     ovf);
  return hipGetLastError();
}

hipError_t launch_relax(const DevTables& t, int modes, hipStream_t s) {
  if (modes < 1 || modes > 3) return hipErrorInvalidValue;
  if (t.n_pipelines <= 0) return hipSuccess;
  if (t.max_pipe_ops <= 64) {
    // one op per lane: records in the same launch
    hipLaunchKernelGGL(relax_kernel<true>, dim3(t.n_pipelines), dim3(128), relax_lds_bytes(t, true), s, t, modes);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(relax_kernel<false>, dim3(t.n_pipelines), dim3(64), relax_lds_bytes(t, false), s, t, modes);
  const int64_t threads = (modes == 3 ? 2 : 1) * (int64_t)t.n_ops;
  if (t.n_ops > 0) hipLaunchKernelGGL(op_records_kernel, dim3(blocks_for(threads, 256)), dim3(256), 0, s, t, modes);
  return hipGetLastError();
}

hipError_t launch_decide_indexed(const DevTables& t, const Batch& b, hipStream_t s) {
  if (b.n == 0) return hipSuccess;
  const uint4* rec = t.rec + (int64_t)b.mode * t.n_ops;
  const uint4* tail = t.rec_tail + (int64_t)b.mode * t.n_ops * REC_TAIL_VECS;
  const uint4* tail2 = t.rec_tail2 + (int64_t)b.mode * t.n_ops * REC_TAIL2_VECS;
  const uint2* ovf = t.ovf + (int64_t)b.mode * t.n_front;
  if (b.queue) {
    // records for this call's queueing times, in the context's own buffers
    hipError_t e = launch_records(t, b.mode, 1, b.queue, t.rec_q, t.rec_tail_q, t.rec_tail2_q, t.ovf_q, s);
    if (e != hipSuccess) return e;
    rec = t.rec_q;
    tail = t.rec_tail_q;
    tail2 = t.rec_tail2_q;
    ovf = t.ovf_q;
  }
  switch (t.decide_sched) {
    case SCHED_LDS: {
      if (t.n_ops > LDS_REC_MAX_OPS) return hipErrorInvalidValue;
      const size_t lds = sizeof(uint4) * (size_t)t.n_ops;
      const bool vec = ((reinterpret_cast<uintptr_t>(b.op) | reinterpret_cast<uintptr_t>(b.elapsed) |
                         reinterpret_cast<uintptr_t>(b.slo) | reinterpret_cast<uintptr_t>(b.cfg)) & 15u) == 0 &&
                       (reinterpret_cast<uintptr_t>(b.flag) & 3u) == 0;
      const void* fn = vec ? (const void*)decide_lds4_kernel : (const void*)decide_lds_kernel;
      hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)(sizeof(uint4) * LDS_REC_MAX_OPS));
      if (e != hipSuccess) return e;
      const int64_t per_block = 1024 * 4;
      int64_t blocks = (b.n + per_block - 1) / per_block;
      if (blocks > t.n_cu) blocks = t.n_cu;
      if (vec)
        hipLaunchKernelGGL(decide_lds4_kernel, dim3((unsigned)blocks), dim3(1024), lds, s, t, b, rec, tail, tail2, ovf);
      else
        hipLaunchKernelGGL(decide_lds_kernel, dim3((unsigned)blocks), dim3(1024), lds, s, t, b, rec, tail, tail2, ovf);
      break;
    }
#define LLAMA_DIRECT(IPT, NT) \
  hipLaunchKernelGGL((decide_indexed_kernel<IPT, NT>), dim3(blocks_for(b.n, 256 * IPT)), dim3(256), 0, s, t, b, rec, \
                     tail, tail2, ovf)
    case SCHED_DIRECT2: LLAMA_DIRECT(2, false); break;
    case SCHED_DIRECT4: LLAMA_DIRECT(4, false); break;
    case SCHED_DIRECT1_NT: LLAMA_DIRECT(1, true); break;
    case SCHED_DIRECT2_NT: LLAMA_DIRECT(2, true); break;
    case SCHED_DIRECT4_NT: LLAMA_DIRECT(4, true); break;
    default: LLAMA_DIRECT(1, false); break;
#undef LLAMA_DIRECT
  }
  return hipGetLastError();
}

// The decision path (records, relaxation, indexed decisions) ends here; the
// counter summaries of the decision kernels fingerprint the text above.
// DECISION-PATH-END

namespace {

// ---------------------------------------------------------------------------
// Full scan, the plain Eq. 1 evaluation of every configuration.
//   bucket_count / bucket_offsets / bucket_scatter: counting sort of the
//     valid invocations by op (invalid ones are answered at once);
//   scan_classes_kernel: one wavefront per op, which takes lanes = the op's
//     invocations (the table walked with wave-uniform scalar loads: one
//     compare, one select and one min per pair) or lanes = configurations
//     (wavefront min), whichever costs fewer instructions for the op's
//     bucket size and table size.
// decide_wave_kernel keeps the same evaluation with lanes = configurations
// and a DPP min reduction across the wave; it needs no scratch.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void fill_zero_kernel(int32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Invalid invocations are answered here and left out of the buckets.
__device__ __forceinline__ bool bucket_key(const DevTables& t, const Batch& b, int64_t i, int* v) {
  *v = b.op[i];
  const int e = b.elapsed[i], s = b.slo[i];
  if (invalid_invocation(*v, e, s, t.n_ops)) {
    b.cfg[i] = -1;
    if (b.flag) b.flag[i] = 0;
    atomicOr(t.err, 1u);
    return false;
  }
  return true;
}

// Sources of bucketing keys over positions 0 .. size() - 1: key() only
// loads (so that a thread's loads for several positions can be in flight
// together); visit() takes the counting pass's side effects for a position
// (answering what key() leaves out).
struct InvocationKeys {  // the batch's invocations by op; invalid ones answered at once
  DevTables t;
  Batch b;
  __device__ int64_t size() const { return b.n; }
  __device__ bool key(int64_t i, int* v) const {
    *v = b.op[i];
    return !invalid_invocation(*v, b.elapsed[i], b.slo[i], t.n_ops);
  }
  __device__ void visit(int64_t i, bool ok) const {
    if (ok) return;
    b.cfg[i] = -1;
    if (b.flag) b.flag[i] = 0;
    atomicOr(t.err, 1u);
  }
};
struct QueueKeys {  // occupied slots of the batching sub-queues, by their invocation's op
  const int32_t* op;
  const uint2* queue;
  const uint32_t* count;
  int64_t cap;
  __device__ int64_t size() const { return (int64_t)BATCH_QUEUES * cap; }
  __device__ bool key(int64_t w, int* v) const {
    const int sq = (int)(w / cap);
    if (w - (int64_t)sq * cap >= (int64_t)count[32 * sq]) return false;
    *v = op[queue[w].x];
    return true;
  }
  __device__ void visit(int64_t, bool) const {}
};
struct AffinityKeys {  // the batch's invocations by op; invalid ones get zero affinities
  DevTables t;
  Batch b;
  double* aff;
  uint64_t* keys;
  int32_t* iota;
  __device__ int64_t size() const { return b.n; }
  __device__ bool key(int64_t i, int* v) const {
    *v = b.op[i];
    return !invalid_invocation(*v, b.elapsed[i], b.slo[i], t.n_ops);
  }
  __device__ void visit(int64_t i, bool ok) const {
    if (iota) iota[i] = (int32_t)i;
    if (ok) return;
    atomicOr(t.err, 1u);
    for (int h = 0; h < t.n_hw; ++h) {
      aff[i * t.n_hw + h] = 0.0;
      if (keys) keys[(int64_t)h * b.n + i] = ~0ull;  // complemented bits of 0.0
    }
  }
};

// Positions a thread of the counting sort's chunk kernels takes at once.
constexpr int BUCKET_UNROLL = 8;

// Each workgroup counts its chunk of BUCKET_CHUNK positions in an LDS
// histogram over the keys op >> shift and writes it as one row of
// hist[chunk][key]: the ops themselves with shift = 0 (few ops), groups of
// 2^shift consecutive ops otherwise (the first level of a two-level sort).
template <class K>
__global__ __launch_bounds__(1024) void bucket_hist_kernel(K keys, int n_ops, int32_t* hist, int shift) {
  extern __shared__ int32_t sh[];
  const int n_keys = ((n_ops - 1) >> shift) + 1;
  for (int j = threadIdx.x; j < n_keys; j += blockDim.x) sh[j] = 0;
  __syncthreads();
  const int64_t n = keys.size();
  const int64_t a = (int64_t)blockIdx.x * BUCKET_CHUNK;
  const int64_t e = a + BUCKET_CHUNK < n ? a + BUCKET_CHUNK : n;
  const int64_t bs = blockDim.x;
  for (int64_t i0 = a + threadIdx.x; i0 < e; i0 += BUCKET_UNROLL * bs) {
    int v[BUCKET_UNROLL];
    bool ok[BUCKET_UNROLL];
#pragma unroll
    for (int u = 0; u < BUCKET_UNROLL; ++u) ok[u] = i0 + u * bs < e && keys.key(i0 + u * bs, &v[u]);
#pragma unroll
    for (int u = 0; u < BUCKET_UNROLL; ++u) {
      if (i0 + u * bs >= e) break;
      keys.visit(i0 + u * bs, ok[u]);
      if (ok[u]) atomicAdd(&sh[v[u] >> shift], 1);
    }
  }
  __syncthreads();
  int32_t* row = hist + (int64_t)blockIdx.x * n_keys;
  for (int j = threadIdx.x; j < n_keys; j += blockDim.x) row[j] = sh[j];
}

// Per key: exclusive prefix over chunks (in place) and the key's total.  A
// workgroup takes COL_KEYS consecutive keys with COL_PARTS threads each; part
// p of a key sums its run of chunks (loads in flight together), the parts'
// sums meet in LDS, and each part then rewrites its run as the running prefix
// from its offset.
constexpr int COL_KEYS = 32, COL_PARTS = 8;
__global__ __launch_bounds__(COL_KEYS * COL_PARTS) void bucket_columns_kernel(int32_t* hist, int n_chunks,
                                                                              int n_ops, int32_t* total) {
  __shared__ int32_t sPart[COL_PARTS][COL_KEYS];
  const int kl = threadIdx.x % COL_KEYS, part = threadIdx.x / COL_KEYS;
  const int v = blockIdx.x * COL_KEYS + kl;
  const int per = (n_chunks + COL_PARTS - 1) / COL_PARTS;
  const int c0 = part * per, c1 = c0 + per < n_chunks ? c0 + per : n_chunks;
  int sum = 0;
  if (v < n_ops) {
    for (int c = c0; c < c1; c += 32) {  // up to 32 loads in flight
      int x[32];
#pragma unroll
      for (int k = 0; k < 32; ++k) x[k] = c + k < c1 ? hist[(int64_t)(c + k) * n_ops + v] : 0;
#pragma unroll
      for (int k = 0; k < 32; ++k) sum += x[k];
    }
  }
  sPart[part][kl] = sum;
  __syncthreads();
  if (v >= n_ops) return;
  int run = 0;
  for (int q = 0; q < part; ++q) run += sPart[q][kl];
  if (part == COL_PARTS - 1) total[v] = run + sum;
  for (int c = c0; c < c1; c += 32) {
    int x[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) x[k] = c + k < c1 ? hist[(int64_t)(c + k) * n_ops + v] : 0;
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      if (c + k < c1) hist[(int64_t)(c + k) * n_ops + v] = run;
      run += x[k];
    }
  }
}

// Each chunk places its positions at start[key] + (earlier chunks' count) +
// (rank inside the chunk, from an LDS counter).  With shift = 0 the entry is
// the position; otherwise it carries the op's low shift bits above a 24-bit
// position, for the second level.
template <class K>
__global__ __launch_bounds__(1024) void bucket_place_kernel(K keys, int n_ops, const int32_t* hist,
                                                           const int32_t* start, int32_t* perm, int shift) {
  // the chunk's first position of each key (start + earlier chunks), then
  // advanced by an LDS atomic per placed position
  extern __shared__ int32_t sh[];
  const int n_keys = ((n_ops - 1) >> shift) + 1;
  const int32_t* row = hist + (int64_t)blockIdx.x * n_keys;
  for (int j = threadIdx.x; j < n_keys; j += blockDim.x) sh[j] = start[j] + row[j];
  __syncthreads();
  const int64_t n = keys.size();
  const int64_t a = (int64_t)blockIdx.x * BUCKET_CHUNK;
  const int64_t e = a + BUCKET_CHUNK < n ? a + BUCKET_CHUNK : n;
  const uint32_t low = (1u << shift) - 1u;
  const int64_t bs = blockDim.x;
  for (int64_t i0 = a + threadIdx.x; i0 < e; i0 += BUCKET_UNROLL * bs) {
    int v[BUCKET_UNROLL];
    bool ok[BUCKET_UNROLL];
#pragma unroll
    for (int u = 0; u < BUCKET_UNROLL; ++u) ok[u] = i0 + u * bs < e && keys.key(i0 + u * bs, &v[u]);
#pragma unroll
    for (int u = 0; u < BUCKET_UNROLL; ++u) {
      if (!ok[u]) continue;
      const int64_t i = i0 + u * bs;
      const int k = v[u] >> shift;
      const uint32_t entry = shift ? (((uint32_t)v[u] & low) << 24) | (uint32_t)i : (uint32_t)i;
      perm[atomicAdd(&sh[k], 1)] = (int32_t)entry;
    }
  }
}

// Second level: one workgroup per group of FINE_OPS consecutive ops sorts the
// group's packed entries (its run [cstart[g], cstart[g + 1]) of packed) by
// the op's low bits, with LDS counters, into perm, and writes the start of
// each of its ops (start[n_ops] = the end of the last group).  Entries of one
// op come out in any order.
constexpr int FINE_BITS = 8;
constexpr int FINE_OPS = 1 << FINE_BITS;
// Bucketing by op: few ops, one LDS-histogram counting sort; many ops, a
// two-level one (groups of FINE_OPS ops, then the ops of each group) while the
// groups fit one LDS histogram and a position fits 24 bits.
inline bool two_level(int64_t n, int32_t n_ops) {
  return n_ops > BUCKET_LDS_OPS && ((n_ops - 1) >> FINE_BITS) + 1 <= BUCKET_LDS_OPS && n <= (1 << 24);
}
inline int64_t round_words(int64_t w) { return (w + 63) & ~(int64_t)63; }
constexpr int FINE_THREADS = 1024;  // threads of a group's workgroup (the first FINE_OPS scan the counts)
__global__ __launch_bounds__(FINE_THREADS) void bucket_fine_kernel(const int32_t* cstart,
                                                                  const int32_t* __restrict__ packed, int n_ops,
                                                                  int32_t* start, int32_t* __restrict__ perm) {
  __shared__ int32_t cnt[FINE_OPS];
  __shared__ int32_t wsum[FINE_OPS / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int g = blockIdx.x;
  const int a = cstart[g], e = cstart[g + 1];
  if (tid < FINE_OPS) cnt[tid] = 0;
  __syncthreads();
  for (int j0 = a + tid; j0 < e; j0 += BUCKET_UNROLL * FINE_THREADS) {
    uint32_t q[BUCKET_UNROLL];
#pragma unroll
    for (int u = 0; u < BUCKET_UNROLL; ++u)
      q[u] = j0 + u * FINE_THREADS < e ? (uint32_t)packed[j0 + u * FINE_THREADS] : 0u;
#pragma unroll
    for (int u = 0; u < BUCKET_UNROLL; ++u)
      if (j0 + u * FINE_THREADS < e) atomicAdd(&cnt[q[u] >> 24], 1);
  }
  __syncthreads();
  // exclusive prefix of the FINE_OPS counts: wavefront scans, then the
  // wavefront totals
  int x = 0, incl = 0;
  if (tid < FINE_OPS) {
    x = cnt[tid];
    incl = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(incl, d, 64);
      if (lane >= d) incl += y;
    }
    if (lane == 63) wsum[wv] = incl;
  }
  __syncthreads();
  if (tid < FINE_OPS) {
    int off = a;
    for (int w = 0; w < wv; ++w) off += wsum[w];
    const int pos = off + incl - x;
    cnt[tid] = pos;  // every thread read its own count above
    const int v = g * FINE_OPS + tid;
    if (v < n_ops) start[v] = pos;
  }
  if (g == (int)gridDim.x - 1 && tid == 0) start[n_ops] = e;
  __syncthreads();
  for (int j0 = a + tid; j0 < e; j0 += BUCKET_UNROLL * FINE_THREADS) {
    uint32_t q[BUCKET_UNROLL];
#pragma unroll
    for (int u = 0; u < BUCKET_UNROLL; ++u)
      q[u] = j0 + u * FINE_THREADS < e ? (uint32_t)packed[j0 + u * FINE_THREADS] : 0u;
#pragma unroll
    for (int u = 0; u < BUCKET_UNROLL; ++u)
      if (j0 + u * FINE_THREADS < e) perm[atomicAdd(&cnt[q[u] >> 24], 1)] = (int32_t)(q[u] & 0xFFFFFFu);
  }
}

// Many ops: global atomics (few invocations share an op, so little contention).
__global__ __launch_bounds__(256) void bucket_count_kernel(DevTables t, Batch b, int32_t* cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= b.n) return;
  int v;
  if (bucket_key(t, b, i, &v)) atomicAdd(&cnt[v], 1);
}

__global__ __launch_bounds__(256) void bucket_scatter_kernel(DevTables t, Batch b, int32_t* cursor,
                                                             int32_t* perm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= b.n) return;
  const int v = b.op[i];
  if (invalid_invocation(v, b.elapsed[i], b.slo[i], t.n_ops)) return;
  perm[atomicAdd(&cursor[v], 1)] = (int32_t)i;
}

// Exclusive prefix sum of cnt[0..n) into start[0..n] and cursor[0..n), one
// workgroup of 1024 lanes walking the array in tiles of 16 K counts: each
// lane reads 16 consecutive counts with 16-byte loads, the tile is scanned
// across lanes (wavefront scans, then the 16 wavefront totals), and a carry
// links the tiles.
constexpr int OFFS_PER_LANE = 16;
__global__ __launch_bounds__(1024) void bucket_offsets_kernel(const int32_t* cnt, int32_t n,
                                                              int32_t* start, int32_t* cursor) {
  __shared__ int32_t wsum[16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int carry = 0;
  for (int64_t base = 0; base < n; base += 1024 * OFFS_PER_LANE) {
    const int64_t a = base + (int64_t)tid * OFFS_PER_LANE;
    int x[OFFS_PER_LANE];
    const bool whole = a + OFFS_PER_LANE <= n;
    if (whole) {
#pragma unroll
      for (int q = 0; q < OFFS_PER_LANE / 4; ++q) {
        const int4 v = *reinterpret_cast<const int4*>(cnt + a + 4 * q);
        x[4 * q] = v.x;
        x[4 * q + 1] = v.y;
        x[4 * q + 2] = v.z;
        x[4 * q + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int q = 0; q < OFFS_PER_LANE; ++q) x[q] = a + q < n ? cnt[a + q] : 0;
    }
    int sum = 0;
#pragma unroll
    for (int q = 0; q < OFFS_PER_LANE; ++q) sum += x[q];
    const int incl = wave_inclusive_scan(sum);
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int run = carry + incl - sum, tile = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
      run += w < wv ? wsum[w] : 0;
      tile += wsum[w];
    }
    int y[OFFS_PER_LANE];
#pragma unroll
    for (int q = 0; q < OFFS_PER_LANE; ++q) {
      y[q] = run;
      run += x[q];
    }
    if (whole) {
#pragma unroll
      for (int q = 0; q < OFFS_PER_LANE / 4; ++q) {
        const int4 v = make_int4(y[4 * q], y[4 * q + 1], y[4 * q + 2], y[4 * q + 3]);
        *reinterpret_cast<int4*>(start + a + 4 * q) = v;
        if (cursor) *reinterpret_cast<int4*>(cursor + a + 4 * q) = v;
      }
    } else {
#pragma unroll
      for (int q = 0; q < OFFS_PER_LANE; ++q)
        if (a + q < n) {
          start[a + q] = y[q];
          if (cursor) cursor[a + q] = y[q];
        }
    }
    carry += tile;
    __syncthreads();  // wsum is rewritten by the next tile
  }
  if (tid == 0) start[n] = carry;
}

// Configurations read as scalar operands: the table through the constant
// address space (s_load into SGPRs), two configurations per 16 bytes.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) u32x4 const_u32x4;

// DPP controls (GFX9 encoding).
constexpr int DPP_QUAD_XOR1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_XOR2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int DPP_ROW_HALF_MIRROR = 0x141;
constexpr int DPP_ROW_MIRROR = 0x140;
constexpr int DPP_ROW_BCAST15 = 0x142;
constexpr int DPP_ROW_BCAST31 = 0x143;

__device__ __forceinline__ uint32_t umin32(uint32_t a, uint32_t b) { return a < b ? a : b; }

// Minimum over the 64 lanes, returned to every lane.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  v = umin32(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, DPP_QUAD_XOR1, 0xF, 0xF, false));
  v = umin32(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, DPP_QUAD_XOR2, 0xF, 0xF, false));
  v = umin32(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, DPP_ROW_HALF_MIRROR, 0xF, 0xF, false));
  v = umin32(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, DPP_ROW_MIRROR, 0xF, 0xF, false));
  // every lane of a 16-lane row now holds the row minimum
  v = umin32(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, DPP_ROW_BCAST15, 0xA, 0xF, false));
  v = umin32(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, DPP_ROW_BCAST31, 0xC, 0xF, false));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

template <int NHW>
__global__ __launch_bounds__(256) void decide_wave_kernel(DevTables t, Batch b) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = wave; i < b.n; i += n_waves) {
    const int v = b.op[i], e = b.elapsed[i], s = b.slo[i];
    if (invalid_invocation(v, e, s, t.n_ops)) {
      if (lane == 0) {
        b.cfg[i] = -1;
        if (b.flag) b.flag[i] = 0;
        atomicOr(t.err, 1u);
      }
      continue;
    }
    const int64_t r0 = (int64_t)s - e;
    const int64_t ref = t.ref[v];
    const int64_t W = t.W[(int64_t)b.mode * t.n_ops + v];
    const int32_t* seg = t.seg_off + (int64_t)v * NHW;
    uint32_t best = KEY_NONE;
#pragma unroll
    for (int h = 0; h < NHW; ++h) {
      const int64_t R = remaining_time(r0, b.queue ? b.queue[h] : 0);
      const int32_t target = R == 0 ? 0 : (int32_t)div_floor_pos(ref * R, W);
      // eight configurations per lane at a time, their loads issued together
      for (int x0 = seg[h] + lane; x0 < seg[h + 1]; x0 += 8 * 64) {
        uint2 c[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) c[u] = x0 + 64 * u < seg[h + 1] ? t.tab[x0 + 64 * u] : make_uint2(0x7FFFFFFFu, KEY_NONE);
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if ((int32_t)c[u].x < target) best = umin32(best, c[u].y);
      }
    }
    // any lane feasible?  otherwise skip the reduction and fall back
    const uint64_t any = __builtin_amdgcn_ballot_w64(best != KEY_NONE);
    if (any) best = wave_min_u32(best);
    if (lane == 0) write_choice(b, i, best, t.hdr[(int64_t)v * t.hs + NHW + 1]);
  }
}

// ---------------------------------------------------------------------------
// Full scan with schedule classes: one wavefront per op, which evaluates its
// op's bucket of k invocations against the op's c configurations in the
// cheaper of two layouts (wavefront instructions, from counting loop trips):
//   lanes = invocations: ceil(k / 64) passes over the table, each
//     configuration a scalar operand (compare, select, min):  ~3 c per pass;
//   lanes = configurations: groups of S = 16, 32 or 64 lanes (the smallest
//     that covers c, so 64 / S invocations share a pass), each lane walking
//     every S-th configuration, then a min over the group:
//     ~ceil(k / (64 / S)) (5 ceil(c / S) + 14).  With S = 64 the table is
//     held in registers instead, in pieces of at most CFG_REG_SLOTS slots of
//     64 per backend (one round of loads per piece instead of one per pass),
//     and the invocations take their turns: each lane computes one
//     invocation's targets, which the wavefront then reads lane by lane:
//     ~ceil(k / 64) 24 NHW + k sum over pieces of (NHW (1 + 3 rs) + 10), rs
//     = the slots of the piece.
// The first is taken when its count times the crossover's den is at most the
// second's times its num; the crossover is the schedule table entry the
// autotuner picks on the caller's batch (llama_autotune_full).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t group_min_u32(uint32_t v, int S) {
  v = umin32(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, DPP_QUAD_XOR1, 0xF, 0xF, false));
  v = umin32(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, DPP_QUAD_XOR2, 0xF, 0xF, false));
  v = umin32(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, DPP_ROW_HALF_MIRROR, 0xF, 0xF, false));
  v = umin32(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, DPP_ROW_MIRROR, 0xF, 0xF, false));
  // every lane of a 16-lane row holds the row minimum
  if (S >= 32) v = umin32(v, (uint32_t)__shfl_xor((int)v, 16, 64));
  if (S >= 64) v = umin32(v, (uint32_t)__shfl_xor((int)v, 32, 64));
  return v;
}

constexpr int CFG_REG_SLOTS = 4;  // register slots of 64 configurations per backend run and piece
// Minimum over the 64 lanes, returned to every lane; the identity as the
// DPP "old" value lets each step fuse into one v_min_u32 with a DPP source.
__device__ __forceinline__ uint32_t wave_min_u32_fused(uint32_t v) {
  const int I = (int)KEY_NONE;
  v = umin32(v, (uint32_t)__builtin_amdgcn_update_dpp(I, (int)v, DPP_QUAD_XOR1, 0xF, 0xF, false));
  v = umin32(v, (uint32_t)__builtin_amdgcn_update_dpp(I, (int)v, DPP_QUAD_XOR2, 0xF, 0xF, false));
  v = umin32(v, (uint32_t)__builtin_amdgcn_update_dpp(I, (int)v, DPP_ROW_HALF_MIRROR, 0xF, 0xF, false));
  v = umin32(v, (uint32_t)__builtin_amdgcn_update_dpp(I, (int)v, DPP_ROW_MIRROR, 0xF, 0xF, false));
  v = umin32(v, (uint32_t)__builtin_amdgcn_update_dpp(I, (int)v, DPP_ROW_BCAST15, 0xA, 0xF, false));
  v = umin32(v, (uint32_t)__builtin_amdgcn_update_dpp(I, (int)v, DPP_ROW_BCAST31, 0xC, 0xF, false));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Lanes = configurations held in registers, one piece of every backend's run
// at a time: slot u of backend h holds configuration seg[h] + base + lane +
// 64 u (never feasible past the run), RS <= CFG_REG_SLOTS slots per backend.
// The piece is read in one round of loads; the wavefront then takes the
// batch's cnt invocations in turn, reading each one's targets (tgv, one
// invocation per lane) lane by lane, and folds the piece's minimum into the
// invocation's lane of res.
// With MASK, configurations whose batch (batch_a[k], k = the key's low 16
// bits) exceeds limit are never feasible either.
template <int NHW, int RS, bool MASK = false>
__device__ __forceinline__ void scan_cfg_piece(const DevTables& t, const int (&seg)[NHW + 1], int base,
                                               const int32_t (&tgv)[NHW], int cnt, uint32_t& res,
                                               const int32_t* batch_a = nullptr, int32_t limit = 0) {
  const int lane = threadIdx.x & 63;
  uint32_t cL[NHW][RS], cK[NHW][RS];
#pragma unroll
  for (int h = 0; h < NHW; ++h)
#pragma unroll
    for (int u = 0; u < RS; ++u) {
      const int x = seg[h] + base + lane + 64 * u;
      uint2 q = x < seg[h + 1] ? t.tab[x] : make_uint2(0x7FFFFFFFu, KEY_NONE);
      if (MASK && q.y != KEY_NONE && batch_a[q.y & 0xFFFFu] > limit) q = make_uint2(0x7FFFFFFFu, KEY_NONE);
      cL[h][u] = q.x;
      cK[h][u] = q.y;
    }
  for (int j = 0; j < cnt; ++j) {
    // every slot's candidate on its own, then a tree of minima (no chain
    // through one accumulator)
    uint32_t cand[NHW * RS];
#pragma unroll
    for (int h = 0; h < NHW; ++h) {
      const int32_t tg = __builtin_amdgcn_readlane(tgv[h], j);
#pragma unroll
      for (int u = 0; u < RS; ++u) cand[h * RS + u] = (int32_t)cL[h][u] < tg ? cK[h][u] : KEY_NONE;
    }
#pragma unroll
    for (int w = 1; w < NHW * RS; w *= 2)
#pragma unroll
      for (int q = 0; q + w < NHW * RS; q += 2 * w) cand[q] = umin32(cand[q], cand[q + w]);
    const uint32_t best = wave_min_u32_fused(cand[0]);
    res = lane == j && best < res ? best : res;
  }
}

template <int NHW>
__device__ __forceinline__ void scan_cfg_regs(const DevTables& t, const Batch& b, const int32_t* perm, int p0,
                                              int p1, const int (&seg)[NHW + 1], int longest, int64_t ref,
                                              int64_t W, int fastest) {
  const int lane = threadIdx.x & 63;
  for (int pb = p0; pb < p1; pb += 64) {
    const int p = pb + lane;
    const bool live = p < p1;
    const int64_t i = live ? perm[p] : 0;
    const int64_t r0 = live ? (int64_t)b.slo[i] - b.elapsed[i] : 0;
    int32_t tgv[NHW];
#pragma unroll
    for (int h = 0; h < NHW; ++h) {
      const int64_t R = remaining_time(r0, b.queue ? b.queue[h] : 0);
      tgv[h] = R == 0 ? 0 : (int32_t)div_floor_pos(ref * R, W);
    }
    uint32_t res = KEY_NONE;
    const int cnt = p1 - pb < 64 ? p1 - pb : 64;
    for (int base = 0; base < longest; base += 64 * CFG_REG_SLOTS) {
      const int rest = longest - base;
      switch (rest <= 64 ? 1 : rest <= 128 ? 2 : rest <= 192 ? 3 : 4) {
        case 1: scan_cfg_piece<NHW, 1>(t, seg, base, tgv, cnt, res); break;
        case 2: scan_cfg_piece<NHW, 2>(t, seg, base, tgv, cnt, res); break;
        case 3: scan_cfg_piece<NHW, 3>(t, seg, base, tgv, cnt, res); break;
        default: scan_cfg_piece<NHW, 4>(t, seg, base, tgv, cnt, res); break;
      }
    }
    if (live) write_choice(b, i, res, fastest);
  }
}

template <int NHW>
__global__ __launch_bounds__(256) void scan_classes_kernel(DevTables t, Batch b, const int32_t* start,
                                                           const int32_t* perm, int32_t cross_num,
                                                           int32_t cross_den) {
  const int lane = threadIdx.x & 63;
  // the op is the same for the whole wavefront: keep it (and what is loaded
  // from it) in scalar registers
  const int v = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
  if (v >= t.n_ops) return;
  const int p0 = start[v], p1 = start[v + 1];
  const int k = p1 - p0;
  if (k == 0) return;
  int seg[NHW + 1];
#pragma unroll
  for (int h = 0; h <= NHW; ++h) seg[h] = t.seg_off[(int64_t)v * NHW + h];
  const int c = seg[NHW] - seg[0];
  const int64_t ref = t.ref[v];
  const int64_t W = t.W[(int64_t)b.mode * t.n_ops + v];
  const int fastest = t.hdr[(int64_t)v * t.hs + NHW + 1];
  const int S = c <= 16 ? 16 : c <= 32 ? 32 : 64;
  const int per = 64 / S;
  int longest = 0;
#pragma unroll
  for (int h = 0; h < NHW; ++h) longest = seg[h + 1] - seg[h] > longest ? seg[h + 1] - seg[h] : longest;
  // register pieces: full ones of CFG_REG_SLOTS slots, then the rest
  const int full = longest / (64 * CFG_REG_SLOTS), rest = longest % (64 * CFG_REG_SLOTS);
  const int per_inv = full * (NHW * (1 + 3 * CFG_REG_SLOTS) + 10) + (rest ? NHW * (1 + 3 * ((rest + 63) >> 6)) + 10 : 0);
  const int64_t cost_inv = (int64_t)((k + 63) / 64) * c * 3;
  const int64_t cost_cfg = S == 64 ? (int64_t)((k + 63) / 64) * 24 * NHW + (int64_t)k * per_inv
                                   : (int64_t)((k + per - 1) / per) * (5 * ((c + S - 1) / S) + 14);
  if (cost_inv * cross_den <= cost_cfg * cross_num) {
    // lanes = invocations; the table as scalar operands, two configurations per 16 bytes
    const_u32x4* tab2 = (const_u32x4*)(const void*)t.tab;
    for (int pb = p0; pb < p1; pb += 64) {
      const int p = pb + lane;
      const bool live = p < p1;
      const int64_t i = live ? perm[p] : 0;
      const int64_t r0 = live ? (int64_t)b.slo[i] - b.elapsed[i] : 0;
      uint32_t best = KEY_NONE;
#pragma unroll
      for (int h = 0; h < NHW; ++h) {
        const int64_t R = remaining_time(r0, b.queue ? b.queue[h] : 0);
        const int32_t tg = R == 0 ? 0 : (int32_t)div_floor_pos(ref * R, W);
        int x = seg[h];
        const int x1 = seg[h + 1];
        if (x < x1 && (x & 1)) {  // align to a pair
          const uint2 q = t.tab[x];
          best = umin32(best, (int32_t)q.x < tg ? q.y : KEY_NONE);
          ++x;
        }
        for (; x + 8 <= x1; x += 8) {
          const u32x4 q0 = tab2[x >> 1], q1 = tab2[(x >> 1) + 1], q2 = tab2[(x >> 1) + 2], q3 = tab2[(x >> 1) + 3];
          uint32_t m0 = umin32((int32_t)q0.x < tg ? q0.y : KEY_NONE, (int32_t)q0.z < tg ? q0.w : KEY_NONE);
          uint32_t m1 = umin32((int32_t)q1.x < tg ? q1.y : KEY_NONE, (int32_t)q1.z < tg ? q1.w : KEY_NONE);
          uint32_t m2 = umin32((int32_t)q2.x < tg ? q2.y : KEY_NONE, (int32_t)q2.z < tg ? q2.w : KEY_NONE);
          uint32_t m3 = umin32((int32_t)q3.x < tg ? q3.y : KEY_NONE, (int32_t)q3.z < tg ? q3.w : KEY_NONE);
          best = umin32(best, umin32(umin32(m0, m1), umin32(m2, m3)));
        }
        for (; x < x1; ++x) {
          const uint2 q = t.tab[x];
          best = umin32(best, (int32_t)q.x < tg ? q.y : KEY_NONE);
        }
      }
      if (live) write_choice(b, i, best, fastest);
    }
    return;
  }
  if (S == 64) {
    scan_cfg_regs<NHW>(t, b, perm, p0, p1, seg, longest, ref, W, fastest);
    return;
  }
  // lanes = configurations, 64 / S invocations per pass
  const int g = lane / S, l = lane % S;
  for (int pb = p0; pb < p1; pb += per) {
    const int p = pb + g;
    const bool live = p < p1;
    const int64_t i = live ? perm[p] : 0;
    const int64_t r0 = live ? (int64_t)b.slo[i] - b.elapsed[i] : 0;
    uint32_t best = KEY_NONE;
#pragma unroll
    for (int h = 0; h < NHW; ++h) {
      const int64_t R = remaining_time(r0, b.queue ? b.queue[h] : 0);
      const int32_t tg = R == 0 ? 0 : (int32_t)div_floor_pos(ref * R, W);
      for (int x0 = seg[h] + l; x0 < seg[h + 1]; x0 += 4 * S) {  // four loads in flight per lane
        uint2 q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) q[u] = x0 + S * u < seg[h + 1] ? t.tab[x0 + S * u] : make_uint2(0x7FFFFFFFu, KEY_NONE);
#pragma unroll
        for (int u = 0; u < 4; ++u) best = umin32(best, (int32_t)q[u].x < tg ? q[u].y : KEY_NONE);
      }
    }
    best = group_min_u32(best, S);
    if (live && l == 0) write_choice(b, i, best, fastest);
  }
}

// Eq. 1 given targets and a latency per (invocation, configuration): one
// wavefront per invocation, lanes over the op's configurations (caller order),
// wavefront min reductions for the cheapest feasible key and the fastest.
template <int NHW>
__global__ __launch_bounds__(256) void select_rows_kernel(DevTables t, Batch b, const int32_t* lat,
                                                          int64_t stride) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = wave; i < b.n; i += n_waves) {
    const int v = b.op[i];
    if ((unsigned)v >= (unsigned)t.n_ops || t.cfg_off[v + 1] - t.cfg_off[v] > stride) {
      if (lane == 0) {
        b.cfg[i] = -1;
        if (b.flag) b.flag[i] = 0;
        atomicOr(t.err, 1u);
      }
      continue;
    }
    int32_t tg[NHW];
#pragma unroll
    for (int h = 0; h < NHW; ++h) tg[h] = b.target[i * NHW + h];
    const int a0 = t.cfg_off[v], n_c = t.cfg_off[v + 1] - a0;
    uint32_t best = KEY_NONE;
    uint64_t fast = ~0ull;
    for (int k = lane; k < n_c; k += 64) {
      const int32_t L = lat[i * stride + k];
      const int h = t.cfg_hw[a0 + k];
      int32_t target = tg[0];
#pragma unroll
      for (int hh = 1; hh < NHW; ++hh) target = h == hh ? tg[hh] : target;
      const uint32_t key = t.cfg_key[a0 + k];
      if (L < target) best = umin32(best, key);
      const uint64_t fk = ((uint64_t)(uint32_t)L << 16) | (uint64_t)k;
      fast = fk < fast ? fk : fast;
    }
    best = wave_min_u32(best);
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint64_t o = __shfl_xor(fast, d, 64);
      fast = o < fast ? o : fast;
    }
    if (lane == 0) {
      b.cfg[i] = best != KEY_NONE ? (int32_t)(best & 0xFFFFu) : (int32_t)(fast & 0xFFFFu);
      if (b.flag) b.flag[i] = best != KEY_NONE ? 1 : 0;
    }
  }
}

// ---------------------------------------------------------------------------
// Eq. 2: queueing time per backend.  Each thread sums L * R of its queued
// entries per backend in 128 bits; a wavefront reduction (two 64-bit halves)
// and an LDS step leave one partial per workgroup and backend in scratch;
// queue_finalize_kernel adds the partials (again in 128 bits) and divides.
// No atomics: the result does not depend on the order of the additions.
// ---------------------------------------------------------------------------
constexpr int QUEUE_BATCH = 4;

__device__ __forceinline__ unsigned __int128 wave_sum_u128(unsigned __int128 x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long lo = __shfl_xor((unsigned long long)x, off, 64);
    const unsigned long long hi = __shfl_xor((unsigned long long)(x >> 64), off, 64);
    x += ((unsigned __int128)hi << 64) | lo;
  }
  return x;
}

template <int NHW>
__global__ __launch_bounds__(256) void queue_accumulate_kernel(DevTables t, int64_t n, const int32_t* q_op,
                                                               const int32_t* q_cfg, unsigned long long* part) {
  __shared__ unsigned long long sPart[4][NHW][2];
  unsigned __int128 sum[NHW];
#pragma unroll
  for (int h = 0; h < NHW; ++h) sum[h] = 0;
  bool bad = false;
  // QUEUE_BATCH entries per thread and pass, their loads issued together
  // (out-of-range entries read entry 0 of op 0 and contribute nothing)
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * QUEUE_BATCH;
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x * QUEUE_BATCH + threadIdx.x; i0 < n; i0 += stride) {
    int v[QUEUE_BATCH], k[QUEUE_BATCH], x[QUEUE_BATCH];
    bool ok[QUEUE_BATCH];
#pragma unroll
    for (int u = 0; u < QUEUE_BATCH; ++u) {
      const int64_t i = i0 + (int64_t)u * blockDim.x;
      v[u] = i < n ? q_op[i] : 0;
      k[u] = i < n ? q_cfg[i] : 0;
      ok[u] = i < n && (unsigned)v[u] < (unsigned)t.n_ops;
      bad |= i < n && !ok[u];
    }
#pragma unroll
    for (int u = 0; u < QUEUE_BATCH; ++u) {
      const int a = t.cfg_off[ok[u] ? v[u] : 0];
      const int e = t.cfg_off[(ok[u] ? v[u] : 0) + 1];
      const bool in = ok[u] && (unsigned)k[u] < (unsigned)(e - a);
      bad |= ok[u] && !in;
      ok[u] = in;
      x[u] = in ? a + k[u] : 0;
    }
#pragma unroll
    for (int u = 0; u < QUEUE_BATCH; ++u) {
      const uint4 q = t.cfg_q[x[u]];  // {L, R, hw, 0}
      const uint64_t p = ok[u] ? (uint64_t)q.x * (uint64_t)q.y : 0ull;
#pragma unroll
      for (int h = 0; h < NHW; ++h) sum[h] += h == (int)q.z ? p : 0ull;
    }
  }
  if (bad) atomicOr(t.err, DEVERR_QUEUE_ENTRY);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int h = 0; h < NHW; ++h) {
    const unsigned __int128 w = wave_sum_u128(sum[h]);
    if (lane == 0) {
      sPart[wave][h][0] = (unsigned long long)w;
      sPart[wave][h][1] = (unsigned long long)(w >> 64);
    }
  }
  __syncthreads();
  if (threadIdx.x < NHW) {
    const int h = threadIdx.x;
    unsigned __int128 tot = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) tot += ((unsigned __int128)sPart[w][h][1] << 64) | sPart[w][h][0];
    unsigned long long* dst = part + ((int64_t)blockIdx.x * MAX_HW + h) * 2;
    dst[0] = (unsigned long long)tot;
    dst[1] = (unsigned long long)(tot >> 64);
  }
}

// Q[h] = min(floor(total[h] / R_total[h]), 2^62): 1024 threads add the
// n_part partials of every backend (wavefront sums, then LDS), then thread h
// divides (a 128-bit total by a divisor below 2^41, 16 bits at a time).
__global__ __launch_bounds__(1024) void queue_finalize_kernel(const unsigned long long* part, int n_part, ResTotals rt,
                                                              int n_hw, int64_t* out) {
  __shared__ unsigned long long sRed[16][MAX_HW][2];
  __shared__ unsigned long long sTot[MAX_HW][2];
  const int tid = threadIdx.x, wave = tid >> 6;
  unsigned __int128 x[MAX_HW];
#pragma unroll
  for (int h = 0; h < MAX_HW; ++h) x[h] = 0;
  if (tid < n_part) {  // n_part <= QUEUE_PARTS = blockDim.x: one partial per thread
    const uint4* p = reinterpret_cast<const uint4*>(part) + (int64_t)tid * MAX_HW;
#pragma unroll
    for (int h = 0; h < MAX_HW; ++h) {
      if (h >= n_hw) break;
      const uint4 v = p[h];  // {low 64 bits, high 64 bits} as four 32-bit words
      x[h] = ((unsigned __int128)(((uint64_t)v.w << 32) | v.z) << 64) | (((uint64_t)v.y << 32) | v.x);
    }
  }
#pragma unroll
  for (int h = 0; h < MAX_HW; ++h) {
    if (h >= n_hw) break;
    const unsigned __int128 w = wave_sum_u128(x[h]);
    if ((tid & 63) == 0) {
      sRed[wave][h][0] = (unsigned long long)w;
      sRed[wave][h][1] = (unsigned long long)(w >> 64);
    }
  }
  __syncthreads();
  if (tid < n_hw) {
    unsigned __int128 tot = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += ((unsigned __int128)sRed[w][tid][1] << 64) | sRed[w][tid][0];
    sTot[tid][0] = (unsigned long long)tot;
    sTot[tid][1] = (unsigned long long)(tot >> 64);
  }
  __syncthreads();
  const int lane = tid;
  if (lane >= n_hw) return;
  const unsigned __int128 s = ((unsigned __int128)sTot[lane][1] << 64) | sTot[lane][0];
  const unsigned __int128 d = (unsigned __int128)(uint64_t)rt.r[lane];
  if (s >= d << 62) {  // d < 2^41, so d * 2^62 < 2^103 does not overflow
    out[lane] = (int64_t)1 << 62;
    return;
  }
  // s < d * 2^62, so the quotient has at most 62 bits: long division by
  // 16-bit digits of s, the running remainder (< d < 2^41) times 2^16 plus a
  // digit staying below 2^57
  const uint64_t dd = (uint64_t)d;
  uint64_t rem = 0, q = 0;
  for (int dig = 7; dig >= 0; --dig) {
    const uint64_t cur = (rem << 16) | (uint64_t)((s >> (16 * dig)) & 0xFFFFu);
    const uint64_t qd = cur / dd;
    rem = cur - qd * dd;
    q = (q << 16) | qd;  // qd < 2^16; bits shifted out are zero as q < 2^62
  }
  out[lane] = (int64_t)q;
}

// ---------------------------------------------------------------------------
// Finite-alpha Eq. 1: per backend, j = number of configurations faster than
// the target (a two-level count over the latency-sorted run); the backend's
// best key is min(prefix-min feasible key before j, suffix-min infeasible key
// from j); the smallest key over backends wins.
// ---------------------------------------------------------------------------
// Entries of the ascending run lat[0 .. len) below target.  smp holds the
// last entry of each block of ALPHA_BLOCK (16-byte aligned, padded with
// INT32_MAX): the samples below target count the blocks entirely below it,
// and the next block is counted entry by entry.  Two dependent rounds of a
// line or two each, where a binary search takes one dependent random load per
// halving.
__device__ __forceinline__ int count_below(const int32_t* lat, int len, const int32_t* smp, int32_t target) {
  const int nb = (len + ALPHA_BLOCK - 1) / ALPHA_BLOCK;
  int m = 0;
  for (int q0 = 0; q0 < nb; q0 += 32) {  // up to eight 16-byte sample loads in flight
    int4 sv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      sv[k] = q0 + 4 * k < nb ? *reinterpret_cast<const int4*>(smp + q0 + 4 * k)
                              : make_int4(INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX);
#pragma unroll
    for (int k = 0; k < 8; ++k)
      m += (sv[k].x < target) + (sv[k].y < target) + (sv[k].z < target) + (sv[k].w < target);
  }
  if (m >= nb) return len;
  const int b0 = m * ALPHA_BLOCK;
  const int bl = len - b0 < ALPHA_BLOCK ? len - b0 : ALPHA_BLOCK;
  int c = 0;
#pragma unroll
  for (int i = 0; i < ALPHA_BLOCK; ++i) c += (i < bl && lat[b0 + i] < target) ? 1 : 0;
  return b0 + c;
}

template <int NHW>
__global__ __launch_bounds__(256) void decide_alpha_kernel(DevTables t, Batch b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= b.n) return;
  const int v = b.op[i], e = b.elapsed[i], s = b.slo[i];
  if (invalid_invocation(v, e, s, t.n_ops)) {
    b.cfg[i] = -1;
    if (b.flag) b.flag[i] = 0;
    atomicOr(t.err, 1u);
    return;
  }
  const int64_t r0 = (int64_t)s - e;
  const int64_t ref = t.ref[v];
  const int64_t W = t.W[(int64_t)b.mode * t.n_ops + v];
  const int32_t* so = t.seg_off + (int64_t)v * NHW;
  int base[NHW];
  const int32_t* smp = t.a_smp + t.a_soff[v];
#pragma unroll
  for (int h = 0; h < NHW; ++h) {
    const int lo = so[h], len = so[h + 1] - lo;
    const int64_t R = remaining_time(r0, b.queue ? b.queue[h] : 0);
    const int32_t target = R == 0 ? 0 : (int32_t)div_floor_pos(ref * R, W);
    base[h] = lo + count_below(t.a_lat + lo, len, smp, target);
    smp += ((len + ALPHA_BLOCK - 1) / ALPHA_BLOCK + 3) & ~3;
  }
  uint32_t best = KEY_NONE;
  uint8_t meets = 0;
  uint2 ps[NHW];
#pragma unroll
  for (int h = 0; h < NHW; ++h) ps[h] = t.a_ps[(int64_t)base[h] + (int64_t)v * NHW + h];
#pragma unroll
  for (int h = 0; h < NHW; ++h) {
    // keys of the segment's entries below and from the first with L >= target
    if (ps[h].x < best) {
      best = ps[h].x;
      meets = 1;
    }
    if (ps[h].y < best) {
      best = ps[h].y;
      meets = 0;
    }
  }
  b.cfg[i] = (int)(best & 0xFFFFu);
  if (b.flag) b.flag[i] = meets;
}

// Eq. 3 from each backend's best key: the ratio of the objective values of
// the best key elsewhere and the best key on the backend (no configuration
// on the backend -> 0; none elsewhere -> infinity; a zero own value ->
// infinity, or 1 when the other is zero too).
template <int NHW>
__device__ __forceinline__ void affinities_from_best(const DevTables& t, int v, const uint32_t (&best)[NHW],
                                                     double (&out)[NHW]) {
  const double* val = t.a_val + 2 * (int64_t)t.cfg_off[v];
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

// An invocation's affinities, and with keys the commit order's sort keys:
// non-negative doubles order like their bit patterns; complemented, an
// ascending sort gives decreasing affinity.
template <int NHW>
__device__ __forceinline__ void store_affinities(const Batch& b, int64_t i, const double (&out)[NHW], double* aff,
                                                 uint64_t* keys) {
  double* dst = aff + i * NHW;
#pragma unroll
  for (int h = 0; h < NHW; ++h) {
    dst[h] = out[h];
    if (keys) keys[(int64_t)h * b.n + i] = ~(uint64_t)__double_as_longlong(out[h]);
  }
}

// Finite-alpha Eq. 1 (with queueing times) and Eq. 3 (with or without),
// grouped by op: one wavefront per op with invocations (perm[start[v] ..
// start[v + 1])).  Each backend's latency run is held in registers in pieces
// of up to CFG_REG_SLOTS slots of 64 (padded with INT32_MAX); each
// invocation's count of entries below its target is the population count of
// the wavefront's compares, invocation by invocation with the targets read
// lane by lane, and each lane then reads its invocation's pair of key minima
// at that count: the decision, or with AFF the affinities.
template <int R, int RS>
__device__ __forceinline__ void alpha_count_piece(const int32_t* lat, const int (&lo)[R], const int (&hi)[R],
                                                  int base, const int32_t (&tgv)[R], int cnt, int (&cntv)[R]) {
  const int lane = threadIdx.x & 63;
  int32_t L[R][RS];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int u = 0; u < RS; ++u) {
      const int x = lo[r] + base + lane + 64 * u;
      L[r][u] = x < hi[r] ? lat[x] : INT32_MAX;
    }
  for (int j = 0; j < cnt; ++j) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int32_t tg = __builtin_amdgcn_readlane(tgv[r], j);
      int c = 0;
#pragma unroll
      for (int u = 0; u < RS; ++u) c += __popcll(__builtin_amdgcn_ballot_w64(L[r][u] < tg));
      cntv[r] += lane == j ? c : 0;
    }
  }
}

template <int NHW, bool AFF>
__device__ __forceinline__ void alpha_ops(const DevTables& t, const Batch& b, const int32_t* start,
                                          const int32_t* perm, double* aff, uint64_t* keys) {
  const int lane = threadIdx.x & 63;
  const int v = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
  if (v >= t.n_ops) return;
  const int p0 = start[v], p1 = start[v + 1];
  if (p0 == p1) return;
  int lo[NHW], hi[NHW];
  int longest = 0;
#pragma unroll
  for (int h = 0; h < NHW; ++h) {
    lo[h] = t.seg_off[(int64_t)v * NHW + h];
    hi[h] = t.seg_off[(int64_t)v * NHW + h + 1];
    longest = hi[h] - lo[h] > longest ? hi[h] - lo[h] : longest;
  }
  const int64_t ref = t.ref[v];
  const int64_t W = t.W[(int64_t)b.mode * t.n_ops + v];
  for (int pb = p0; pb < p1; pb += 64) {
    const int p = pb + lane;
    const bool live = p < p1;
    const int64_t i = live ? perm[p] : 0;
    const int64_t r0 = live ? (int64_t)b.slo[i] - b.elapsed[i] : 0;
    int32_t tgv[NHW];
    int cntv[NHW];
#pragma unroll
    for (int h = 0; h < NHW; ++h) {
      const int64_t R = remaining_time(r0, b.queue ? b.queue[h] : 0);
      tgv[h] = R == 0 ? 0 : (int32_t)div_floor_pos(ref * R, W);
      cntv[h] = 0;
    }
    const int cnt = p1 - pb < 64 ? p1 - pb : 64;
    for (int base = 0; base < longest; base += 64 * CFG_REG_SLOTS) {
      const int rest = longest - base;
      switch (rest <= 64 ? 1 : rest <= 128 ? 2 : rest <= 192 ? 3 : 4) {
        case 1: alpha_count_piece<NHW, 1>(t.a_lat, lo, hi, base, tgv, cnt, cntv); break;
        case 2: alpha_count_piece<NHW, 2>(t.a_lat, lo, hi, base, tgv, cnt, cntv); break;
        case 3: alpha_count_piece<NHW, 3>(t.a_lat, lo, hi, base, tgv, cnt, cntv); break;
        default: alpha_count_piece<NHW, 4>(t.a_lat, lo, hi, base, tgv, cnt, cntv); break;
      }
    }
    if (!live) continue;
    uint2 ps[NHW];
#pragma unroll
    for (int h = 0; h < NHW; ++h) ps[h] = t.a_ps[(int64_t)lo[h] + cntv[h] + (int64_t)v * NHW + h];
    if (AFF) {
      uint32_t best[NHW];
      double out[NHW];
#pragma unroll
      for (int h = 0; h < NHW; ++h) best[h] = ps[h].y < ps[h].x ? ps[h].y : ps[h].x;
      affinities_from_best<NHW>(t, v, best, out);
      store_affinities<NHW>(b, i, out, aff, keys);
      continue;
    }
    uint32_t best = KEY_NONE;
    uint8_t meets = 0;
#pragma unroll
    for (int h = 0; h < NHW; ++h) {
      if (ps[h].x < best) {
        best = ps[h].x;
        meets = 1;
      }
      if (ps[h].y < best) {
        best = ps[h].y;
        meets = 0;
      }
    }
    b.cfg[i] = (int)(best & 0xFFFFu);
    if (b.flag) b.flag[i] = meets;
  }
}

template <int NHW>
__global__ __launch_bounds__(256) void decide_alpha_ops_kernel(DevTables t, Batch b, const int32_t* start,
                                                               const int32_t* perm) {
  alpha_ops<NHW, false>(t, b, start, perm, nullptr, nullptr);
}

template <int NHW>
__global__ __launch_bounds__(256) void affinity_ops_kernel(DevTables t, Batch b, const int32_t* start,
                                                           const int32_t* perm, double* aff, uint64_t* keys) {
  alpha_ops<NHW, true>(t, b, start, perm, aff, keys);
}

// Without queueing times every backend's target is the same, so one search
// over the op's configurations of all backends (latency order) suffices.
__global__ __launch_bounds__(256) void decide_alpha_merged_kernel(DevTables t, Batch b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= b.n) return;
  const int v = b.op[i], e = b.elapsed[i], s = b.slo[i];
  if (invalid_invocation(v, e, s, t.n_ops)) {
    b.cfg[i] = -1;
    if (b.flag) b.flag[i] = 0;
    atomicOr(t.err, 1u);
    return;
  }
  const int64_t R = remaining_time((int64_t)s - e, 0);
  const int32_t target =
      R == 0 ? 0 : (int32_t)div_floor_pos((int64_t)t.ref[v] * R, t.W[(int64_t)b.mode * t.n_ops + v]);
  const int lo = t.cfg_off[v], end = t.cfg_off[v + 1];
  // one search per invocation: a binary search (an op's run is long and its
  // upper levels are shared by the op's invocations in L2) measured faster
  // here than the two-level count
  int base = lo, len = end - lo;
  for (int step = 0; step < t.m_steps && len > 0; ++step) {
    const int half = len >> 1;
    if (t.m_lat[base + half] < target) {
      base += half + 1;
      len -= half + 1;
    } else {
      len = half;
    }
  }
  uint32_t best = KEY_NONE;
  uint8_t meets = 0;
  if (base > lo) {
    best = t.m_pf[base - 1];
    meets = 1;
  }
  if (base < end) {
    const uint32_t ki = t.m_si[base];
    if (ki < best) {
      best = ki;
      meets = 0;
    }
  }
  b.cfg[i] = (int)(best & 0xFFFFu);
  if (b.flag) b.flag[i] = meets;
}

// ---------------------------------------------------------------------------
// Feedback (exponential smoothing of the profile, then the table rebuild).
//   feedback_accumulate_kernel  count and sum of each configuration's
//                               observations (atomics into zeroed scratch)
//   feedback_apply_kernel       one smoothing step per observed configuration,
//                               taken by the observation that finds the count
//                               non-zero (and resets count and sum to zero)
//   retable_kernel              per op with an observation (one wavefront):
//                               merged and per-backend frontiers by running
//                               minima in the static key order (no sort);
//                               header, fastest, reference, the full table's
//                               latencies
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void feedback_accumulate_kernel(DevTables t, FeedbackArgs f, int64_t n,
                                                                  const int32_t* op, const int32_t* cfg,
                                                                  const int32_t* obs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int v = op[i], k = cfg[i], o = obs[i];
  if ((unsigned)v >= (unsigned)t.n_ops || o < 1 || (unsigned)k >= (unsigned)(t.cfg_off[v + 1] - t.cfg_off[v])) {
    atomicOr(t.err, DEVERR_OBSERVATION);
    return;
  }
  const int x = t.cfg_off[v] + k;
  atomicAdd(&f.count[x], 1u);
  atomicAdd(&f.sum[x], (unsigned long long)o);
  if (f.dirty[v] == 0u) f.dirty[v] = 1u;  // racing writers all store 1
}

// L' = L + floor(beta * (S - m L) / (2^16 m)), clamped to [1, 2^31 - 1], in
// 64-bit integers: with D = S - m L = m t1 + r (0 <= r < m) and
// beta t1 = 2^16 a + b (0 <= b < 2^16), the step is
// a + [b m + beta r >= 2^16 m] (the bracket's left side is below 2^17 m).
__global__ __launch_bounds__(256) void feedback_apply_kernel(DevTables t, FeedbackArgs f, int64_t n, const int32_t* op,
                                                             const int32_t* cfg, const int32_t* obs, uint32_t beta) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int v = op[i], k = cfg[i], o = obs[i];
  if ((unsigned)v >= (unsigned)t.n_ops || o < 1 || (unsigned)k >= (unsigned)(t.cfg_off[v + 1] - t.cfg_off[v])) return;
  const int x = t.cfg_off[v] + k;
  const uint32_t m = atomicExch(&f.count[x], 0u);
  if (m == 0) return;  // another observation of x applied the step
  const int64_t S = (int64_t)atomicExch(&f.sum[x], 0ull);
  const int64_t L = f.lat[x];
  const int64_t mm = m;
  const int64_t D = S - mm * L;
  int64_t t1 = D / mm, r = D - t1 * mm;
  if (r < 0) {
    t1 -= 1;
    r += mm;
  }
  const int64_t u = (int64_t)beta * t1;
  int64_t a = u >> 16;  // floor division by 2^16 (arithmetic shift)
  const int64_t b = u - (a << 16);
  if (b * mm + (int64_t)beta * r >= (mm << 16)) a += 1;
  int64_t nl = L + a;
  nl = nl < 1 ? 1 : (nl > INT32_MAX_64 ? INT32_MAX_64 : nl);
  f.lat[x] = (int32_t)nl;
}

// Exclusive prefix minimum over the wavefront (lane order) of x, continued
// from `carry` (the minimum of everything before lane 0); returns the
// exclusive value of this lane and updates carry to the chunk's total.
// min(x, x of the lane the DPP control names); lanes it names none (or that
// the row or bank mask leaves out) take the identity 0xFFFFFFFF
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ uint32_t dpp_min(uint32_t x) {
  return umin32(x, (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFFu, (int)x, CTRL, ROW_MASK, BANK_MASK, false));
}
constexpr int DPP_ROW_SHR1 = 0x111, DPP_ROW_SHR2 = 0x112, DPP_ROW_SHR4 = 0x114, DPP_ROW_SHR8 = 0x118;
constexpr int DPP_WAVE_SHR1 = 0x138;

// Exclusive running minimum over the wavefront's lanes, continuing from
// carry (updated to the minimum through lane 63): the inclusive minimum by
// doubling shifts within each 16-lane row, then the rows' last lanes carried
// into the rows after them; shifted one lane, with carry in lane 0.
__device__ __forceinline__ uint32_t wave_excl_min(uint32_t x, uint32_t& carry) {
  uint32_t incl = dpp_min<DPP_ROW_SHR1, 0xF, 0xF>(x);
  incl = dpp_min<DPP_ROW_SHR2, 0xF, 0xF>(incl);
  incl = dpp_min<DPP_ROW_SHR4, 0xF, 0xF>(incl);
  incl = dpp_min<DPP_ROW_SHR8, 0xF, 0xF>(incl);
  incl = dpp_min<DPP_ROW_BCAST15, 0xA, 0xF>(incl);
  incl = dpp_min<DPP_ROW_BCAST31, 0xC, 0xF>(incl);
  incl = umin32(incl, carry);
  const uint32_t excl = (uint32_t)__builtin_amdgcn_update_dpp((int)carry, (int)incl, DPP_WAVE_SHR1, 0xF, 0xF, false);
  carry = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
  return excl;
}

// Frontiers without sorting.  Along an op's frontier (latency ascending,
// every entry cheaper than all faster ones) a configuration survives iff it
// is strictly faster than every cheaper configuration: L_x < min{L_y : key_y
// < key_x} (ties in L go to the cheaper key, as in the sorted construction).
// Keys do not change with latencies, so the op's configurations are visited
// in the static key order and one running minimum of L per list decides;
// survivors come out in key order, which is descending latency, and are
// written from the back.  The backend lists use the same test restricted to
// their backend.  Two passes: counts, then writes.
template <int NHW>
__global__ __launch_bounds__(64) void retable_kernel(DevTables t, FeedbackArgs f) {
  const int v = blockIdx.x, lane = threadIdx.x;
  // only ops with an observed configuration changed; the flag is cleared
  // here for the next call (every lane has read it before the barrier)
  const bool changed = f.dirty[v] != 0u;
  __syncthreads();
  if (!changed) return;
  if (lane == 0) f.dirty[v] = 0u;
  const int a = t.cfg_off[v], n = t.cfg_off[v + 1] - a;
  const int rk = f.ref_k[v];
  uint64_t fast = ~0ull;
  for (int i = lane; i < n; i += 64) {
    const int x = a + i;
    const uint32_t L = (uint32_t)f.lat[x];
    const uint64_t c = ((uint64_t)L << 16) | (uint32_t)i;  // fastest: smallest L, lowest index
    fast = c < fast ? c : fast;
    if (i == rk) f.ref[v] = (int32_t)L;
    if (f.cfg_q) f.cfg_q[x].x = L;
    f.tab[x].x = (uint32_t)f.lat[f.tab_src[x]];  // the full table's row at position x
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(fast, off, 64);
    fast = o < fast ? o : fast;
  }
  constexpr uint32_t INF = 0xFFFFFFFFu;
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  int tot_m = 0, tot_h[NHW];
#pragma unroll
  for (int h = 0; h < NHW; ++h) tot_h[h] = 0;
  for (int pass = 0; pass < 2; ++pass) {
    uint32_t carry_m = INF, carry_h[NHW];
#pragma unroll
    for (int h = 0; h < NHW; ++h) carry_h[h] = INF;
    int seen_m = 0, seen_h[NHW], start_h[NHW];
    int pos = a;
#pragma unroll
    for (int h = 0; h < NHW; ++h) {
      seen_h[h] = 0;
      start_h[h] = pos;
      pos += tot_h[h];
    }
    for (int c0 = 0; c0 < n; c0 += 64) {
      const int p = c0 + lane;
      const bool valid = p < n;
      const int x = valid ? f.ksrc[a + p] : a;
      const uint32_t L = valid ? (uint32_t)f.lat[x] : INF;
      const int hw = valid ? t.cfg_hw[x] : NHW;
      const uint32_t em = wave_excl_min(L, carry_m);
      const bool sm = valid && L < em;
      const uint64_t bm = __ballot(sm);
      if (pass == 1 && sm) {
        const int r = seen_m + __popcll(bm & below);
        f.mst[a + tot_m - 1 - r] = make_uint2(L, t.cfg_key[x]);
      }
      seen_m += __popcll(bm);
#pragma unroll
      for (int h = 0; h < NHW; ++h) {
        const uint32_t eh = wave_excl_min(hw == h ? L : INF, carry_h[h]);
        const bool sh = valid && hw == h && L < eh;
        const uint64_t bh = __ballot(sh);
        if (pass == 1 && sh) {
          const int r = seen_h[h] + __popcll(bh & below);
          f.front[start_h[h] + tot_h[h] - 1 - r] = make_uint2(L, t.cfg_key[x]);
        }
        seen_h[h] += __popcll(bh);
      }
    }
    if (pass == 0) {
      tot_m = seen_m;
#pragma unroll
      for (int h = 0; h < NHW; ++h) tot_h[h] = seen_h[h];
    } else if (lane == 0) {
      int32_t* hd = f.hdr + (int64_t)v * t.hs;
#pragma unroll
      for (int h = 0; h < NHW; ++h) hd[h] = start_h[h];
      hd[NHW] = pos;
      hd[NHW + 1] = (int32_t)(fast & 0xFFFFu);
      f.mst_n[v] = tot_m;
    }
  }
}

// ---------------------------------------------------------------------------
// Eq. 3 affinity: per backend the best key among its configurations (the
// finite-alpha search of decide_alpha_kernel) and among the others; the
// ratio of their objective values (per-rank table).  Readings: no
// configuration on the backend -> 0; none elsewhere -> infinity; a zero own
// minimum -> infinity, or 1 when the other minimum is zero too.  With `keys`,
// also the sort keys for the commit order (descending affinity).
// ---------------------------------------------------------------------------
template <int NHW>
__global__ __launch_bounds__(256) void affinity_kernel(DevTables t, Batch b, double* aff, uint64_t* keys,
                                                       int32_t* iota) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= b.n) return;
  if (iota) iota[i] = (int32_t)i;
  const int v = b.op[i], e = b.elapsed[i], s = b.slo[i];
  double out[NHW];
  if (invalid_invocation(v, e, s, t.n_ops)) {
    atomicOr(t.err, 1u);
#pragma unroll
    for (int h = 0; h < NHW; ++h) out[h] = 0.0;
  } else {
    const int64_t r0 = (int64_t)s - e;
    const int64_t ref = t.ref[v];
    const int64_t W = t.W[(int64_t)b.mode * t.n_ops + v];
    const int32_t* so = t.seg_off + (int64_t)v * NHW;
    int base[NHW], len[NHW];
    int32_t target[NHW];
#pragma unroll
    for (int h = 0; h < NHW; ++h) {
      base[h] = so[h];
      len[h] = so[h + 1] - so[h];
      const int64_t R = remaining_time(r0, b.queue ? b.queue[h] : 0);
      target[h] = R == 0 ? 0 : (int32_t)div_floor_pos(ref * R, W);
    }
    for (int step = 0; step < t.a_steps; ++step) {
#pragma unroll
      for (int h = 0; h < NHW; ++h) {
        if (len[h] > 0) {
          const int half = len[h] >> 1;
          if (t.a_lat[base[h] + half] < target[h]) {
            base[h] += half + 1;
            len[h] -= half + 1;
          } else {
            len[h] = half;
          }
        }
      }
    }
    uint32_t best[NHW];
#pragma unroll
    for (int h = 0; h < NHW; ++h) {
      const uint2 ps = t.a_ps[(int64_t)base[h] + (int64_t)v * NHW + h];
      best[h] = ps.y < ps.x ? ps.y : ps.x;
    }
    affinities_from_best<NHW>(t, v, best, out);
  }
  store_affinities<NHW>(b, i, out, aff, keys);
}

// ---------------------------------------------------------------------------
// Safe delayed batching, two kernels.
//   batching_commit_kernel  one thread per invocation: x*, the Eq. 1 choice
//                           over every configuration, from the op's decision
//                           record (with queueing times the records are
//                           rebuilt for the call); commit x* when its batch
//                           is available, wait when it meets its slack and
//                           the batch arrives in time; any other invocation
//                           joins its workgroup's sub-queue (one atomic per
//                           wavefront, 64 sub-queues)
//   batching_scan_kernel    one wavefront per sub-queue slot (those past their
//                           sub-queue's length exit at once): lanes over the
//                           op's configurations (caller order, coalesced),
//                           the cheapest feasible key and the fastest
//                           (L << 16 | k) among those whose batch fits
//                           max(available, 1); x* if none fits
// ---------------------------------------------------------------------------
template <int NHW>
__device__ __forceinline__ int32_t backend_target(const DevTables& t, const Batch& b, int v, int64_t r0, int h) {
  const int64_t R = remaining_time(r0, b.queue ? b.queue[h] : 0);
  return R == 0 ? 0 : (int32_t)div_floor_pos((int64_t)t.ref[v] * R, t.W[(int64_t)b.mode * t.n_ops + v]);
}

template <int NHW>
__global__ __launch_bounds__(BATCH_BLOCK) void batching_commit_kernel(DevTables t, Batch b, BatchingArgs ba,
                                                                      const uint4* rec, const uint4* tail,
                                                                      const uint4* tail2, const uint2* ovf,
                                                                      int64_t cap) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool push = false;
  int xs = 0;
  uint8_t meets = 0;
  if (i < b.n) {
    const int v = b.op[i], e = b.elapsed[i], s = b.slo[i];
    if (invalid_invocation(v, e, s, t.n_ops)) {
      b.cfg[i] = -1;
      if (b.flag) b.flag[i] = 0;
      atomicOr(t.err, 1u);
    } else {
      xs = decide_from_record(t, tail, tail2, ovf, v, rec[v], s - e, &meets);
      const int a = t.cfg_off[v];
      const int32_t av = ba.available[v];
      const int32_t Bx = t.cfg_batch[a + xs];
      int c = xs;
      uint8_t f = meets;
      if (Bx > av) {
        bool wait = false;
        if (meets && (int64_t)av + ba.upstream[v] >= Bx) {
          const int32_t tx = backend_target<NHW>(t, b, v, (int64_t)s - e, t.cfg_hw[a + xs]);
          wait = (int64_t)ba.wait_us[v] + t.cfg_lat[a + xs] < tx;
        }
        if (wait) {
          c = CFG_WAIT;
          f = 1;
        } else {
          push = true;
        }
      }
      if (!push) {
        b.cfg[i] = c;
        if (b.flag) b.flag[i] = f;
      }
    }
  }
  // wavefront-aggregated append to this workgroup's sub-queue
  const uint64_t mask = __ballot(push);
  if (mask == 0) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)mask) - 1;
  const int sq = (int)(blockIdx.x % BATCH_QUEUES);
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(ba.count + 32 * sq, (uint32_t)__popcll(mask));
  base = __shfl(base, leader, 64);
  if (push) {
    const uint32_t rank = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
    ba.queue[(int64_t)sq * cap + base + rank] = make_uint2((uint32_t)i, (uint32_t)xs | ((uint32_t)meets << 16));
  }
}

template <int NHW>
__global__ __launch_bounds__(256) void batching_scan_kernel(DevTables t, Batch b, BatchingArgs ba, int64_t cap) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int sq = (int)(w / cap);
  const int64_t q = w - (int64_t)sq * cap;
  // the counts are final: the commit kernel ran before on this stream
  if (sq < BATCH_QUEUES && q < (int64_t)ba.count[32 * sq]) {  // uniform per wavefront
    const uint2 ent = ba.queue[w];
    const int64_t i = ent.x;
    const int v = b.op[i];
    const int64_t r0 = (int64_t)b.slo[i] - b.elapsed[i];
    int32_t target[NHW];
#pragma unroll
    for (int h = 0; h < NHW; ++h) target[h] = backend_target<NHW>(t, b, v, r0, h);
    const int a = t.cfg_off[v], end = t.cfg_off[v + 1];
    const int32_t av = ba.available[v];
    const int64_t limit = av > 1 ? av : 1;
    uint32_t kFr = KEY_NONE;
    uint64_t fR = ~0ull;
    // eight configurations per lane at a time, their loads issued together
    for (int x0 = a + lane; x0 < end; x0 += 8 * 64) {
      int32_t Bv[8], Lv[8], Hv[8];
      uint32_t Kv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int x = x0 + 64 * u;
        const bool in = x < end;
        Bv[u] = in ? t.cfg_batch[x] : INT32_MAX;
        Lv[u] = in ? t.cfg_lat[x] : 0;
        Kv[u] = in ? t.cfg_key[x] : KEY_NONE;
        Hv[u] = in ? t.cfg_hw[x] : 0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (Bv[u] > limit) continue;
        int32_t tg = target[0];
#pragma unroll
        for (int h = 1; h < NHW; ++h) tg = Hv[u] == h ? target[h] : tg;
        const uint64_t fk = ((uint64_t)(uint32_t)Lv[u] << 16) | (uint32_t)(x0 + 64 * u - a);
        if (Lv[u] < tg && Kv[u] < kFr) kFr = Kv[u];
        if (fk < fR) fR = fk;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const uint32_t o2 = __shfl_xor(kFr, off, 64);
      const uint64_t o4 = __shfl_xor(fR, off, 64);
      kFr = o2 < kFr ? o2 : kFr;
      fR = o4 < fR ? o4 : fR;
    }
    if (lane == 0) {
      int c = (int)(ent.y & 0xFFFFu);
      uint8_t f = (uint8_t)(ent.y >> 16);
      if (fR != ~0ull) {  // otherwise no configuration fits: x* stands
        const bool mr = kFr != KEY_NONE;
        c = (int)((mr ? (uint64_t)kFr : fR) & 0xFFFFu);
        f = mr ? 1 : 0;
      }
      b.cfg[i] = c;
      if (b.flag) b.flag[i] = f;
    }
  }
}


// The batch-limited scan grouped by op: one wavefront per op with queued
// invocations (perm[start[v] .. start[v + 1]) are their sub-queue slots).
// The op's configurations whose batch fits max(available, 1) are scanned
// from registers in pieces as in the full scan, the others never feasible;
// the fastest of them (L << 16 | k) is found once for the op.
template <int NHW>
__global__ __launch_bounds__(256) void batching_ops_kernel(DevTables t, Batch b, BatchingArgs ba,
                                                           const int32_t* start, const int32_t* perm) {
  const int lane = threadIdx.x & 63;
  const int v = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
  if (v >= t.n_ops) return;
  const int p0 = start[v], p1 = start[v + 1];
  if (p0 == p1) return;
  int seg[NHW + 1];
#pragma unroll
  for (int h = 0; h <= NHW; ++h) seg[h] = t.seg_off[(int64_t)v * NHW + h];
  int longest = 0;
#pragma unroll
  for (int h = 0; h < NHW; ++h) longest = seg[h + 1] - seg[h] > longest ? seg[h + 1] - seg[h] : longest;
  const int32_t* batch_a = t.cfg_batch + t.cfg_off[v];
  const int32_t av = ba.available[v];
  const int32_t limit = av > 1 ? av : 1;
  uint64_t fR = ~0ull;
  for (int x = seg[0] + lane; x < seg[NHW]; x += 64) {
    const uint2 q = t.tab[x];
    const uint32_t k = q.y & 0xFFFFu;
    const uint64_t fk = ((uint64_t)q.x << 16) | k;
    if (batch_a[k] <= limit && fk < fR) fR = fk;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(fR, off, 64);
    fR = o < fR ? o : fR;
  }
  for (int pb = p0; pb < p1; pb += 64) {
    const int p = pb + lane;
    const bool live = p < p1;
    const uint2 ent = live ? ba.queue[perm[p]] : make_uint2(0u, 0u);
    const int64_t i = ent.x;
    const int64_t r0 = live ? (int64_t)b.slo[i] - b.elapsed[i] : 0;
    int32_t tgv[NHW];
#pragma unroll
    for (int h = 0; h < NHW; ++h) tgv[h] = backend_target<NHW>(t, b, v, r0, h);
    uint32_t res = KEY_NONE;
    const int cnt = p1 - pb < 64 ? p1 - pb : 64;
    if (fR != ~0ull) {  // otherwise no configuration fits and every x* stands
      for (int base = 0; base < longest; base += 64 * CFG_REG_SLOTS) {
        const int rest = longest - base;
        switch (rest <= 64 ? 1 : rest <= 128 ? 2 : rest <= 192 ? 3 : 4) {
          case 1: scan_cfg_piece<NHW, 1, true>(t, seg, base, tgv, cnt, res, batch_a, limit); break;
          case 2: scan_cfg_piece<NHW, 2, true>(t, seg, base, tgv, cnt, res, batch_a, limit); break;
          case 3: scan_cfg_piece<NHW, 3, true>(t, seg, base, tgv, cnt, res, batch_a, limit); break;
          default: scan_cfg_piece<NHW, 4, true>(t, seg, base, tgv, cnt, res, batch_a, limit); break;
        }
      }
    }
    if (live) {
      int c = (int)(ent.y & 0xFFFFu);
      uint8_t f = (uint8_t)(ent.y >> 16);
      if (fR != ~0ull) {
        const bool mr = res != KEY_NONE;
        c = (int)((mr ? (uint64_t)res : fR) & 0xFFFFu);
        f = mr ? 1 : 0;
      }
      b.cfg[i] = c;
      if (b.flag) b.flag[i] = f;
    }
  }
}


// ---------------------------------------------------------------------------
// Serving: persistent plain decisions.  Each wavefront claims up to r.chunk
// published requests (lanes = requests), decides them from the records and
// writes result and device time into the ring; it exits when the host sets
// stop, once no wavefront has claimed anything for idle_ticks, or once it has
// run life_ticks (it never exits holding a claim).  The host relaunches the kernel whenever it
// has exited with requests outstanding.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void serve_plain_kernel(DevTables t, ServeRing r) {
  const int lane = threadIdx.x & 63;
  const uint4* rec = t.rec + (int64_t)r.mode * t.n_ops;
  const uint4* tail = t.rec_tail + (int64_t)r.mode * t.n_ops * REC_TAIL_VECS;
  const uint4* tail2 = t.rec_tail2 + (int64_t)r.mode * t.n_ops * REC_TAIL2_VECS;
  const uint2* ovf = t.ovf + (int64_t)r.mode * t.n_front;
  int answered = 0;
  int* clock = blockIdx.x == 0 && threadIdx.x < 64 ? &answered : nullptr;
  serve_enter(r, lane);
  const unsigned long long start = (unsigned long long)wall_clock64();
  unsigned long long last = start;
  for (;;) {
    const unsigned long long now = (unsigned long long)wall_clock64();
    if (now - start > r.life_ticks) break;
    const ServeClaim c = serve_claim(r, lane, r.chunk, clock);
    if (c.stop) break;
    if (c.count == 0) {
      if (serve_idle(r, now, last)) break;
      __builtin_amdgcn_s_sleep(8);
      continue;
    }
    last = now;
    if (lane < c.count) {
      const long long seq = c.first + lane;
      const long long slot = seq % r.cap;
      const int4 q = r.req[slot];
      int cfg = -1;
      uint8_t f = 0;
      if (invalid_invocation(q.x, q.y, q.z, t.n_ops))
        atomicOr(t.err, 1u);
      else
        cfg = decide_from_record(t, tail, tail2, ovf, q.x, rec[q.x], q.z - q.y, &f);
      serve_write(r, seq, slot, cfg, f);
    }
  }
  serve_leave(r, lane);
}

// Host/device clock handshake (one thread): see launch_clock_probe.
__global__ void clock_probe_kernel(const int* flag, int* ack, unsigned long long* stamp, int rounds,
                                   unsigned long long timeout_ticks) {
  if (threadIdx.x != 0) return;
  const unsigned long long start = (unsigned long long)wall_clock64();
  for (int k = 0; k < rounds; ++k) {
    while (__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM) != k + 1) {
      if ((unsigned long long)wall_clock64() - start > timeout_ticks) return;
      __builtin_amdgcn_s_sleep(1);
    }
    stamp[k] = (unsigned long long)wall_clock64();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    __hip_atomic_store(ack, k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

}  // namespace

hipError_t launch_targets(const DevTables& t, const Batch& b, hipStream_t s) {
  if (b.n == 0) return hipSuccess;
  LLAMA_DISPATCH_NHW(targets_kernel, dim3(blocks_for(b.n, 256)), dim3(256), s, t, b);
  return hipGetLastError();
}

hipError_t launch_select_indexed(const DevTables& t, const Batch& b, hipStream_t s) {
  if (b.n == 0) return hipSuccess;
  LLAMA_DISPATCH_NHW(select_indexed_kernel, dim3(blocks_for(b.n, 256)), dim3(256), s, t, b);
  return hipGetLastError();
}

hipError_t launch_queue_time(const DevTables& t, int64_t n, const int32_t* q_op, const int32_t* q_cfg,
                             unsigned long long* part, const ResTotals& rt, int64_t* out, hipStream_t s) {
  int64_t blocks = (n + 256 * QUEUE_BATCH - 1) / (256 * QUEUE_BATCH);
  if (blocks > QUEUE_PARTS) blocks = QUEUE_PARTS;
  if (blocks > 0)
    LLAMA_DISPATCH_NHW(queue_accumulate_kernel, dim3((unsigned)blocks), dim3(256), s, t, n, q_op, q_cfg, part);
  hipLaunchKernelGGL(queue_finalize_kernel, dim3(1), dim3(1024), 0, s, (const unsigned long long*)part, (int)blocks,
                     rt, t.n_hw, out);
  return hipGetLastError();
}

hipError_t launch_feedback(const DevTables& t, const FeedbackArgs& f, int64_t n, const int32_t* obs_op,
                           const int32_t* obs_cfg, const int32_t* obs_lat, uint32_t beta_q16, hipStream_t s) {
  if (n > 0) {
    hipLaunchKernelGGL(feedback_accumulate_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, t, f, n, obs_op,
                       obs_cfg, obs_lat);
    hipLaunchKernelGGL(feedback_apply_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, t, f, n, obs_op, obs_cfg,
                       obs_lat, beta_q16);
  }
  switch (t.n_hw) {
#define LLAMA_RETABLE(NH) \
  case NH: hipLaunchKernelGGL(retable_kernel<NH>, dim3(t.n_ops), dim3(64), 0, s, t, f); break;
    LLAMA_RETABLE(1) LLAMA_RETABLE(2) LLAMA_RETABLE(3) LLAMA_RETABLE(4)
    LLAMA_RETABLE(5) LLAMA_RETABLE(6) LLAMA_RETABLE(7) LLAMA_RETABLE(8)
#undef LLAMA_RETABLE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Counting sort of positions 0 .. n - 1 of `keys` by op into perm, with
// start[v] .. start[v + 1] the positions of op v: one LDS-histogram pass for
// few ops, two levels for many (two_level).  cnt and cursor are scratch of
// n_ops + 1 words, hist of full_scan_hist_words(n, n_ops).  Returns false,
// launching nothing, when neither applies.
template <class K>
bool launch_counting_sort(const K& keys, int64_t n, int n_ops, int32_t* cnt, int32_t* start, int32_t* cursor,
                          int32_t* perm, int32_t* hist, hipStream_t s) {
  const int n_chunks = (int)((n + BUCKET_CHUNK - 1) / BUCKET_CHUNK);
  if (n_ops <= BUCKET_LDS_OPS) {
    const size_t lds = sizeof(int32_t) * (size_t)n_ops;
    hipLaunchKernelGGL(bucket_hist_kernel<K>, dim3(n_chunks), dim3(1024), lds, s, keys, n_ops, hist, 0);
    hipLaunchKernelGGL(bucket_columns_kernel, dim3(blocks_for(n_ops, COL_KEYS)), dim3(COL_KEYS * COL_PARTS), 0, s,
                       hist, n_chunks, n_ops, cnt);
    hipLaunchKernelGGL(bucket_offsets_kernel, dim3(1), dim3(1024), 0, s, cnt, n_ops, start, (int32_t*)nullptr);
    hipLaunchKernelGGL(bucket_place_kernel<K>, dim3(n_chunks), dim3(1024), lds, s, keys, n_ops, hist, start, perm, 0);
    return true;
  }
  if (!two_level(n, n_ops)) return false;
  // groups of FINE_OPS ops: counts in cnt, group starts in cursor (n_ops >
  // groups + 1 words), packed entries after the group histograms
  const int n_groups = ((n_ops - 1) >> FINE_BITS) + 1;
  const size_t lds = sizeof(int32_t) * (size_t)n_groups;
  int32_t* packed = hist + round_words((int64_t)n_chunks * n_groups);
  hipLaunchKernelGGL(bucket_hist_kernel<K>, dim3(n_chunks), dim3(1024), lds, s, keys, n_ops, hist, FINE_BITS);
  hipLaunchKernelGGL(bucket_columns_kernel, dim3(blocks_for(n_groups, COL_KEYS)), dim3(COL_KEYS * COL_PARTS), 0, s,
                     hist, n_chunks, n_groups, cnt);
  hipLaunchKernelGGL(bucket_offsets_kernel, dim3(1), dim3(1024), 0, s, cnt, n_groups, cursor, (int32_t*)nullptr);
  hipLaunchKernelGGL(bucket_place_kernel<K>, dim3(n_chunks), dim3(1024), lds, s, keys, n_ops, hist, cursor, packed,
                     FINE_BITS);
  hipLaunchKernelGGL(bucket_fine_kernel, dim3(n_groups), dim3(FINE_THREADS), 0, s, cursor, packed, n_ops, start,
                     perm);
  return true;
}

hipError_t launch_decide_batching(const DevTables& t, const Batch& b, const BatchingArgs& a, hipStream_t s) {
  if (b.n == 0) return hipSuccess;
  const uint4* rec = t.rec + (int64_t)b.mode * t.n_ops;
  const uint4* tail = t.rec_tail + (int64_t)b.mode * t.n_ops * REC_TAIL_VECS;
  const uint4* tail2 = t.rec_tail2 + (int64_t)b.mode * t.n_ops * REC_TAIL2_VECS;
  const uint2* ovf = t.ovf + (int64_t)b.mode * t.n_front;
  if (b.queue) {
    // records for this call's queueing times, in the context's own buffers
    hipError_t e = launch_records(t, b.mode, 1, b.queue, t.rec_q, t.rec_tail_q, t.rec_tail2_q, t.ovf_q, s);
    if (e != hipSuccess) return e;
    rec = t.rec_q;
    tail = t.rec_tail_q;
    tail2 = t.rec_tail2_q;
    ovf = t.ovf_q;
  }
  const int64_t cap = batch_queue_capacity(b.n);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks_for(32 * BATCH_QUEUES, 256)), dim3(256), 0, s,
                     reinterpret_cast<int32_t*>(a.count), (int64_t)32 * BATCH_QUEUES);
  LLAMA_DISPATCH_NHW(batching_commit_kernel, dim3(blocks_for(b.n, BATCH_BLOCK)), dim3(BATCH_BLOCK), s, t, b, a, rec,
                     tail, tail2, ovf, cap);
  const int64_t n_slots = (int64_t)BATCH_QUEUES * cap;
  // the queued invocations grouped by op (counting sort of the occupied
  // slots), then one wavefront per op
  if (launch_counting_sort(QueueKeys{b.op, a.queue, a.count, cap}, n_slots, t.n_ops, a.op_cnt, a.op_start,
                           a.op_cursor, a.perm, a.hist, s)) {
    LLAMA_DISPATCH_NHW(batching_ops_kernel, dim3((unsigned)t.n_ops), dim3(64), s, t, b, a, a.op_start,
                       a.perm);
    return hipGetLastError();
  }
  // one wavefront per sub-queue slot; those past their sub-queue's count exit at once
  LLAMA_DISPATCH_NHW(batching_scan_kernel, dim3(blocks_for(n_slots, 4)), dim3(256), s, t, b, a, cap);
  return hipGetLastError();
}

hipError_t launch_affinity(const DevTables& t, const Batch& b, double* aff, int32_t* order, void* scratch,
                           size_t scratch_bytes, const FullScratch* w, hipStream_t s) {
  if (b.n == 0) return hipSuccess;
  const int64_t n = b.n;
  uint64_t* keys = order ? static_cast<uint64_t*>(scratch) : nullptr;  // [n_hw * n]
  uint64_t* kout = keys ? keys + (int64_t)t.n_hw * n : nullptr;          // [n]
  int32_t* iota = kout ? reinterpret_cast<int32_t*>(kout + n) : nullptr; // [n]
  if (w && launch_counting_sort(AffinityKeys{t, b, aff, keys, iota}, n, t.n_ops, w->cnt, w->start, w->cursor, w->perm,
                                w->hist, s)) {
    LLAMA_DISPATCH_NHW(affinity_ops_kernel, dim3((unsigned)t.n_ops), dim3(64), s, t, b, w->start,
                       w->perm, aff, keys);
  } else {
    LLAMA_DISPATCH_NHW(affinity_kernel, dim3(blocks_for(n, 256)), dim3(256), s, t, b, aff, keys, iota);
  }
  if (!order) return hipGetLastError();
  const size_t off = ((size_t)n * (8 * (size_t)t.n_hw + 8 + 4) + 255) & ~(size_t)255;
  if (scratch_bytes < off) return hipErrorInvalidValue;
  void* tmp = static_cast<char*>(scratch) + off;
  const size_t tmp_bytes = scratch_bytes - off;
  for (int h = 0; h < t.n_hw; ++h) {
    hipError_t e = sort_pairs(tmp, tmp_bytes, keys + (int64_t)h * n, kout, iota, order + (int64_t)h * n, (int)n, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t launch_decide_alpha(const DevTables& t, const Batch& b, const FullScratch* w, hipStream_t s) {
  if (b.n == 0) return hipSuccess;
  // grouped by op only with queueing times: without them one binary search
  // per invocation over the op's merged run is as fast (0.60 against
  // 0.62 ms with grouping on 4 M invocations over 81 M configurations), the
  // run's upper levels being shared in L2 by the op's invocations
  if (b.queue && w &&
      launch_counting_sort(InvocationKeys{t, b}, b.n, t.n_ops, w->cnt, w->start, w->cursor, w->perm, w->hist, s)) {
    LLAMA_DISPATCH_NHW(decide_alpha_ops_kernel, dim3((unsigned)t.n_ops), dim3(64), s, t, b, w->start,
                       w->perm);
    return hipGetLastError();
  }
  if (b.queue) {
    LLAMA_DISPATCH_NHW(decide_alpha_kernel, dim3(blocks_for(b.n, 256)), dim3(256), s, t, b);
  } else {
    hipLaunchKernelGGL(decide_alpha_merged_kernel, dim3(blocks_for(b.n, 256)), dim3(256), 0, s, t, b);
  }
  return hipGetLastError();
}

hipError_t launch_serve_plain(const DevTables& t, const ServeRing& r, int workgroups, hipStream_t s) {
  if (workgroups < 1 || r.cap < 1 || r.chunk < 1 || r.chunk > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(serve_plain_kernel, dim3(workgroups), dim3(256), 0, s, t, r);
  return hipGetLastError();
}

hipError_t launch_clock_probe(const int* flag, int* ack, unsigned long long* stamp, int rounds,
                              uint64_t timeout_ticks, hipStream_t s) {
  hipLaunchKernelGGL(clock_probe_kernel, dim3(1), dim3(64), 0, s, flag, ack, stamp, rounds,
                     (unsigned long long)timeout_ticks);
  return hipGetLastError();
}

// Few ops and two-level bucketing as two_level() tells; else global atomics.
int64_t full_scan_hist_words(int64_t n_inv, int32_t n_ops) {
  const int64_t n_chunks = (n_inv + BUCKET_CHUNK - 1) / BUCKET_CHUNK;
  if (n_ops <= BUCKET_LDS_OPS) return n_chunks * (int64_t)n_ops;
  // group histograms, then the packed entries of the first level
  if (two_level(n_inv, n_ops)) return round_words(n_chunks * (int64_t)(((n_ops - 1) >> FINE_BITS) + 1)) + n_inv;
  return 0;
}

hipError_t launch_decide_full(const DevTables& t, const Batch& b, const FullScratch& w, hipStream_t s) {
  if (b.n == 0) return hipSuccess;
  if (!launch_counting_sort(InvocationKeys{t, b}, b.n, t.n_ops, w.cnt, w.start, w.cursor, w.perm, w.hist, s)) {
    const unsigned g = blocks_for(b.n, 256);
    hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks_for(t.n_ops + 1, 256)), dim3(256), 0, s, w.cnt,
                       (int64_t)t.n_ops + 1);
    hipLaunchKernelGGL(bucket_count_kernel, dim3(g), dim3(256), 0, s, t, b, w.cnt);
    hipLaunchKernelGGL(bucket_offsets_kernel, dim3(1), dim3(1024), 0, s, w.cnt, t.n_ops, w.start, w.cursor);
    hipLaunchKernelGGL(bucket_scatter_kernel, dim3(g), dim3(256), 0, s, t, b, w.cursor, w.perm);
  }
  LLAMA_DISPATCH_NHW(scan_classes_kernel, dim3((unsigned)t.n_ops), dim3(64), s, t, b, w.start, w.perm,
                     t.full_cross_num, t.full_cross_den);
  return hipGetLastError();
}

hipError_t launch_select_rows(const DevTables& t, const Batch& b, const int32_t* lat, int64_t stride,
                              hipStream_t s) {
  if (b.n == 0) return hipSuccess;
  const int64_t waves = b.n < (int64_t)256 * 4 * 16 ? b.n : (int64_t)256 * 4 * 16;
  LLAMA_DISPATCH_NHW(select_rows_kernel, dim3(blocks_for(waves, 4)), dim3(256), s, t, b, lat, stride);
  return hipGetLastError();
}

hipError_t launch_decide_wave(const DevTables& t, const Batch& b, hipStream_t s) {
  if (b.n == 0) return hipSuccess;
  // 4 waves per block; enough blocks for every CU several times over, each
  // wave then walks its invocations with a grid stride.
  const int64_t waves = b.n < (int64_t)256 * 4 * 16 ? b.n : (int64_t)256 * 4 * 16;
  LLAMA_DISPATCH_NHW(decide_wave_kernel, dim3(blocks_for(waves, 4)), dim3(256), s, t, b);
  return hipGetLastError();
}

}  // namespace llama
