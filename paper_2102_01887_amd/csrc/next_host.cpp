// Host side of the queueing-time estimate (Eq. 2) and the finite-alpha form
// of the Eq. 1 objective: argument checks, the alpha tables built at set-up,
// and the launches.  Implements llama_queue_time, llama_set_alpha and
// llama_decide_alpha of include/llama.h.
//
// Finite-alpha tables.  For configuration x of op v the objective takes one
// of two values, independent of the invocation:
//     feasible   F(x) = C/B
//     infeasible I(x) = (C * R_total * a_den + a_num * L * R) / (B * R_total * a_den)
// (R_total of x's backend).  Every op's 2n values are ranked exactly (dense
// ranks, compared by 256-bit cross-multiplication), so the decision compares
// 32-bit keys rank << 16 | k.  Feasibility on backend h is a latency prefix
// of that backend's configurations (L < target_h), so per (op, backend) the
// configurations are stored in latency order with the prefix minimum of the
// feasible keys and the suffix minimum of the infeasible keys: the best
// choice on backend h is min(prefix_min_F[j - 1], suffix_min_I[j]) with j the
// number of configurations faster than the target.  Without queueing times
// every backend has the same target, and one list per op over all backends
// (same minima) needs a single search.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "llama.h"
#include "llama_ctx.h"
#include "llama_internal.h"

namespace {

// A non-negative fraction with 128-bit numerator and denominator.
struct Frac {
  unsigned __int128 num, den;
};

// 128 x 128 -> 256-bit product as four 64-bit limbs, least significant first,
// by schoolbook multiplication of 32-bit digits into 64-bit columns.
void mul_256(unsigned __int128 a, unsigned __int128 b, uint64_t out[4]) {
  uint32_t x[4], y[4];
  for (int i = 0; i < 4; ++i) {
    x[i] = (uint32_t)(a >> (32 * i));
    y[i] = (uint32_t)(b >> (32 * i));
  }
  uint32_t digit[8];
  uint64_t carry = 0;
  for (int k = 0; k < 8; ++k) {
    // sum of x[i]*y[k-i]: at most four products below 2^64 each, so split
    // every product into 32-bit halves to keep the column sum exact
    uint64_t lo = carry, hi = 0;
    for (int i = 0; i < 4; ++i) {
      const int j = k - i;
      if (j < 0 || j > 3) continue;
      const uint64_t p = (uint64_t)x[i] * y[j];
      lo += (uint32_t)p;
      hi += p >> 32;
    }
    digit[k] = (uint32_t)lo;
    carry = (lo >> 32) + hi;
  }
  for (int i = 0; i < 4; ++i) out[i] = (uint64_t)digit[2 * i] | ((uint64_t)digit[2 * i + 1] << 32);
}

// a < b exactly.
bool frac_less(const Frac& a, const Frac& b) {
  uint64_t l[4], r[4];
  mul_256(a.num, b.den, l);
  mul_256(b.num, a.den, r);
  for (int i = 3; i >= 0; --i)
    if (l[i] != r[i]) return l[i] < r[i];
  return false;
}

}  // namespace

namespace llama {

int build_alpha_tables(llama_ctx* c) {
  const int n_ops = c->n_ops, n_hw = c->n_hw;
  const int64_t n_cfg = c->n_cfg;
  std::vector<int32_t> a_lat(n_cfg), m_lat(n_cfg);
  std::vector<double> a_val(2 * (size_t)n_cfg, 0.0);
  std::vector<uint32_t> a_pf(n_cfg), a_si(n_cfg), m_pf(n_cfg), m_si(n_cfg), a_fk(n_cfg), a_ik(n_cfg);
  std::vector<uint16_t> m_cnt((size_t)n_cfg * n_hw);
  int max_seg = 0, max_op = 0;
  bool too_many = false;
#pragma omp parallel for schedule(dynamic, 64) reduction(max : max_seg, max_op) reduction(|| : too_many)
  for (int v = 0; v < n_ops; ++v) {
    const int a = c->cfg_off[v], b = c->cfg_off[v + 1], n = b - a;
    if (n > LLAMA_ALPHA_MAX_CFG_PER_OP) {
      too_many = true;
      continue;
    }
    // the op's 2n objective values: index 2j = F of config j, 2j+1 = I
    std::vector<Frac> val(2 * (size_t)n);
    for (int j = 0; j < n; ++j) {
      const int x = a + j;
      const unsigned __int128 rt = (unsigned __int128)(uint64_t)c->res_total[c->hw[x]];
      val[2 * j] = Frac{(unsigned __int128)(uint64_t)c->cost[x], (unsigned __int128)(uint32_t)c->batch[x]};
      val[2 * j + 1] = Frac{(unsigned __int128)(uint64_t)c->cost[x] * rt * c->alpha_den +
                                (unsigned __int128)c->alpha_num * (uint32_t)c->lat[x] * (uint32_t)c->res[x],
                            (unsigned __int128)(uint32_t)c->batch[x] * rt * c->alpha_den};
    }
    std::vector<int32_t> ord(2 * (size_t)n);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int32_t p, int32_t q) { return frac_less(val[p], val[q]); });
    std::vector<uint32_t> rank(2 * (size_t)n);
    uint32_t r = 0;
    for (size_t i = 0; i < ord.size(); ++i) {
      if (i > 0 && frac_less(val[ord[i - 1]], val[ord[i]])) ++r;
      rank[ord[i]] = r;
      // the objective value of each rank, for Eq. 3's ratios (three roundings)
      a_val[2 * (size_t)a + r] = (double)val[ord[i]].num / (double)val[ord[i]].den;
    }
    // per backend: configurations in latency order (caller index among equal
    // latencies), prefix minima of feasible keys, suffix minima of infeasible keys
    std::vector<int32_t> cnt(n_hw + 1, 0);
    for (int x = a; x < b; ++x) cnt[c->hw[x] + 1]++;
    for (int h = 0; h < n_hw; ++h) cnt[h + 1] += cnt[h];
    std::vector<int32_t> seg(n);
    {
      std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
      for (int x = a; x < b; ++x) seg[fill[c->hw[x]]++] = x - a;
    }
    for (int h = 0; h < n_hw; ++h) {
      const int s0 = cnt[h], s1 = cnt[h + 1];
      max_seg = std::max(max_seg, s1 - s0);
      std::sort(seg.begin() + s0, seg.begin() + s1, [&](int32_t p, int32_t q) {
        return c->lat[a + p] != c->lat[a + q] ? c->lat[a + p] < c->lat[a + q] : p < q;
      });
      uint32_t m = KEY_NONE;
      for (int i = s0; i < s1; ++i) {
        const int j = seg[i];
        a_lat[a + i] = c->lat[a + j];
        a_fk[a + i] = (rank[2 * j] << 16) | (uint32_t)j;
        a_ik[a + i] = (rank[2 * j + 1] << 16) | (uint32_t)j;
        m = std::min(m, a_fk[a + i]);
        a_pf[a + i] = m;
      }
      m = KEY_NONE;
      for (int i = s1 - 1; i >= s0; --i) {
        const int j = seg[i];
        m = std::min(m, (rank[2 * j + 1] << 16) | (uint32_t)j);
        a_si[a + i] = m;
      }
    }
    // the same over all backends together, for calls without queueing times
    // (every backend then has the same target)
    max_op = std::max(max_op, n);
    std::vector<int32_t> all(n);
    std::iota(all.begin(), all.end(), 0);
    std::sort(all.begin(), all.end(), [&](int32_t p, int32_t q) {
      return c->lat[a + p] != c->lat[a + q] ? c->lat[a + p] < c->lat[a + q] : p < q;
    });
    uint32_t m = KEY_NONE;
    std::vector<uint16_t> seen(n_hw, 0);  // per backend, entries before position i
    for (int i = 0; i < n; ++i) {
      for (int h = 0; h < n_hw; ++h) m_cnt[(size_t)(a + i) * n_hw + h] = seen[h];
      ++seen[c->hw[a + all[i]]];
      m_lat[a + i] = c->lat[a + all[i]];
      m = std::min(m, (rank[2 * all[i]] << 16) | (uint32_t)all[i]);
      m_pf[a + i] = m;
    }
    m = KEY_NONE;
    for (int i = n - 1; i >= 0; --i) {
      m = std::min(m, (rank[2 * all[i] + 1] << 16) | (uint32_t)all[i]);
      m_si[a + i] = m;
    }
  }
  if (too_many)
    return fail(c, LLAMA_E_RANGE, "set_alpha: an op has more than %d configurations", LLAMA_ALPHA_MAX_CFG_PER_OP);
  // block samples of every (op, backend) run of a_lat
  auto padded_blocks = [](int len) { return ((len + ALPHA_BLOCK - 1) / ALPHA_BLOCK + 3) & ~3; };
  auto backend_counts = [&](int v, std::vector<int32_t>& cnt) {  // run h = [a + cnt[h], a + cnt[h + 1])
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int x = c->cfg_off[v]; x < c->cfg_off[v + 1]; ++x) cnt[c->hw[x] + 1]++;
    for (int h = 0; h < n_hw; ++h) cnt[h + 1] += cnt[h];
  };
  std::vector<int32_t> a_soff(n_ops + 1, 0);
  {
    std::vector<int32_t> cnt(n_hw + 1);
    for (int v = 0; v < n_ops; ++v) {
      backend_counts(v, cnt);
      int na = 0;
      for (int h = 0; h < n_hw; ++h) na += padded_blocks(cnt[h + 1] - cnt[h]);
      a_soff[v + 1] = a_soff[v] + na;
    }
  }
  std::vector<int32_t> a_smp(std::max(a_soff[n_ops], 4), INT32_MAX);
#pragma omp parallel
  {
    std::vector<int32_t> cnt(n_hw + 1);
#pragma omp for schedule(dynamic, 256)
    for (int v = 0; v < n_ops; ++v) {
      const int a = c->cfg_off[v];
      backend_counts(v, cnt);
      int o = a_soff[v];
      for (int h = 0; h < n_hw; ++h) {
        const int s0 = a + cnt[h], len = cnt[h + 1] - cnt[h];
        for (int b = 0; b * ALPHA_BLOCK < len; ++b)
          a_smp[o + b] = a_lat[s0 + std::min(len - 1, b * ALPHA_BLOCK + ALPHA_BLOCK - 1)];
        o += padded_blocks(len);
      }
    }
  }
  // per backend run of len entries, len + 1 pairs {min feasible key over its
  // first j entries, min infeasible key over entries j..}: run h of op v
  // starts at seg_off + v * n_hw + h, one extra pair per earlier run
  std::vector<uint2> a_ps((size_t)n_cfg + (size_t)n_ops * n_hw);
#pragma omp parallel
  {
    std::vector<int32_t> cnt(n_hw + 1);
#pragma omp for schedule(dynamic, 256)
    for (int v = 0; v < n_ops; ++v) {
      const int a = c->cfg_off[v];
      backend_counts(v, cnt);
      for (int h = 0; h < n_hw; ++h) {
        const int s0 = a + cnt[h], len = cnt[h + 1] - cnt[h];
        uint2* ps = a_ps.data() + (size_t)s0 + (size_t)v * n_hw + h;
        for (int j = 0; j <= len; ++j)
          ps[j] = make_uint2(j > 0 ? a_pf[s0 + j - 1] : KEY_NONE, j < len ? a_si[s0 + j] : KEY_NONE);
      }
    }
  }
  int steps = 0, msteps = 0;
  while ((1 << steps) <= max_seg) ++steps;
  while ((1 << msteps) <= max_op) ++msteps;
  int rc;
  if ((rc = upload(c, c->d_a_lat, a_lat.data(), a_lat.size() * 4, "alpha latencies")) ||
      (rc = upload(c, c->d_a_ps, a_ps.data(), a_ps.size() * sizeof(uint2), "alpha prefix and suffix keys")) ||
      (rc = upload(c, c->d_m_lat, m_lat.data(), m_lat.size() * 4, "alpha merged latencies")) ||
      (rc = upload(c, c->d_m_pf, m_pf.data(), m_pf.size() * 4, "alpha merged prefix keys")) ||
      (rc = upload(c, c->d_m_si, m_si.data(), m_si.size() * 4, "alpha merged suffix keys")) ||
      (rc = upload(c, c->d_a_val, a_val.data(), a_val.size() * 8, "alpha objective values")) ||
      (rc = upload(c, c->d_a_fk, a_fk.data(), a_fk.size() * 4, "alpha feasible keys")) ||
      (rc = upload(c, c->d_a_ik, a_ik.data(), a_ik.size() * 4, "alpha infeasible keys")) ||
      (rc = upload(c, c->d_m_cnt, m_cnt.data(), m_cnt.size() * 2, "alpha merged backend counts")) ||
      (rc = upload(c, c->d_a_smp, a_smp.data(), a_smp.size() * 4, "alpha latency samples")) ||
      (rc = upload(c, c->d_a_soff, a_soff.data(), a_soff.size() * 4, "alpha sample offsets")))
    return rc;
  if (max_op <= ALPHA_MERGE_MAX) {
    // per-call merged order for calls with queueing times
    if ((rc = upload(c, c->d_aq_T, nullptr, (size_t)n_cfg * 4, "alpha merged thresholds")) ||
        (rc = upload(c, c->d_aq_pf, nullptr, (size_t)n_cfg * 4, "alpha merged prefix keys")) ||
        (rc = upload(c, c->d_aq_si, nullptr, (size_t)n_cfg * 4, "alpha merged suffix keys")) ||
        (rc = upload(c, c->d_aq_cnt, nullptr, (size_t)n_cfg * n_hw * 2, "alpha merged backend counts")))
      return rc;
  }
  if ((rc = sync_ctx(c, "alpha tables"))) return rc;
  c->alpha_steps = steps;
  c->alpha_msteps = msteps;
  c->alpha_max_op = max_op;
  return LLAMA_OK;
}

}  // namespace llama

extern "C" {

int llama_queue_time(llama_ctx* c, int64_t n, const int32_t* q_op, const int32_t* q_cfg, int64_t* out,
                     void* stream) {
  int rc = llama::enter(c);
  if (rc) return rc;
  if (!c->has_prof) return llama::fail(c, LLAMA_E_STATE, "queue_time: no profiles");
  if ((int)c->res_total.size() != c->n_hw)
    return llama::fail(c, LLAMA_E_STATE, "queue_time: the profiles carry no hw_res_total");
  if (n < 0) return llama::fail(c, LLAMA_E_ARG, "queue_time: n_queued < 0");
  if (!out || (n > 0 && (!q_op || !q_cfg))) return llama::fail(c, LLAMA_E_ARG, "queue_time: null pointer");
  if (!c->d_qacc.p) return llama::fail(c, LLAMA_E_STATE, "queue_time: no accumulators");
  llama::ResTotals rt{};
  for (int h = 0; h < c->n_hw; ++h) rt.r[h] = c->res_total[h];
  hipError_t e = llama::launch_queue_time(c->tables(), n, q_op, q_cfg, c->d_qacc.as<unsigned long long>(), rt,
                                          out, (hipStream_t)stream);
  if (e != hipSuccess) return llama::hip_fail(c, e, "queue_time launch");
  return LLAMA_OK;
}

int llama_set_alpha(llama_ctx* c, uint32_t alpha_num, uint32_t alpha_den) {
  int rc = llama::enter(c);
  if (rc) return rc;
  if (!c->has_prof) return llama::fail(c, LLAMA_E_STATE, "set_alpha: no profiles");
  if ((int)c->res_total.size() != c->n_hw)
    return llama::fail(c, LLAMA_E_STATE, "set_alpha: the profiles carry no hw_res_total");
  if (alpha_den < 1) return llama::fail(c, LLAMA_E_ARG, "set_alpha: alpha_den must be >= 1");
  if ((rc = llama::pull_profiles(c))) return rc;
  c->has_alpha = false;
  c->alpha_num = alpha_num;
  c->alpha_den = alpha_den;
  if ((rc = llama::build_alpha_tables(c))) return rc;
  c->has_alpha = true;
  return LLAMA_OK;
}

namespace {

// With queueing times the per-call merge rebuilds every op's merged order
// (work in proportion to the configurations: NHW - 1 binary searches per
// configuration), while one search per backend costs work in proportion to
// the invocations (NHW searches each); the merge pays only when each
// configuration serves enough invocations.  Measured on the MI355X: the
// merge wins at 1 M invocations over 1.86 M configurations (256 pipelines of
// 10-40 ops) and loses by about 4x at 4 M over 81 M (4,096 pipelines of
// 3-200 ops), so it is used when 8 n_inv >= n_cfg.
bool merge_pays(const llama_ctx* c, int64_t n) { return 8 * n >= c->n_cfg; }

}  // namespace

int llama_decide_alpha(llama_ctx* c, int64_t n, const int32_t* op, const int32_t* elapsed, const int32_t* slo,
                       const int64_t* queue, int32_t mode, int32_t* cfg, uint8_t* flag, void* stream) {
  int rc = llama::enter(c);
  if (rc) return rc;
  if (!c->has_prof) return llama::fail(c, LLAMA_E_STATE, "decide_alpha: no profiles");
  if (!c->has_alpha) return llama::fail(c, LLAMA_E_STATE, "decide_alpha: call llama_set_alpha first");
  if (n < 0) return llama::fail(c, LLAMA_E_ARG, "decide_alpha: n_inv < 0");
  if (n > 0 && (!op || !elapsed || !slo || !cfg)) return llama::fail(c, LLAMA_E_ARG, "decide_alpha: null pointer");
  if (mode != LLAMA_SLACK_PAPER && mode != LLAMA_SLACK_PROB)
    return llama::fail(c, LLAMA_E_ARG, "decide_alpha: bad slack_mode %d", mode);
  llama::Batch b{};
  b.n = n; b.op = op; b.elapsed = elapsed; b.slo = slo; b.queue = queue; b.cfg = cfg; b.flag = flag; b.mode = mode;
  // with queueing times, one search per invocation in the op's per-call
  // merged order when every op fits the merge and the merge pays; else one
  // search per backend
  hipError_t e;
  if (queue && c->alpha_max_op <= llama::ALPHA_MERGE_MAX && c->d_aq_T.p && merge_pays(c, n)) {
    e = llama::launch_decide_alpha_queue(c->tables(), b, (hipStream_t)stream);
  } else {
    // with queueing times, grouped by op in the full scan's scratch when it
    // holds n invocations (grown here, except while the stream is being
    // captured)
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const bool capturing = stream && hipStreamIsCapturing((hipStream_t)stream, &cs) == hipSuccess &&
                           cs != hipStreamCaptureStatusNone;
    const bool grouped = queue && n > 0 &&
                         (n <= c->perm_cap || (!capturing && reserve_perm(c, n, (hipStream_t)stream) == LLAMA_OK));
    llama::FullScratch w{c->d_cnt.as<int32_t>(), c->d_start.as<int32_t>(), c->d_cursor.as<int32_t>(),
                         c->d_perm.as<int32_t>(), c->d_hist.as<int32_t>()};
    e = llama::launch_decide_alpha(c->tables(), b, grouped ? &w : nullptr, (hipStream_t)stream);
  }
  if (e != hipSuccess) return llama::hip_fail(c, e, "decide_alpha launch");
  return LLAMA_OK;
}

int llama_decide_batching(llama_ctx* c, int64_t n, const int32_t* op, const int32_t* elapsed, const int32_t* slo,
                          const int64_t* queue, int32_t mode, const int32_t* available, const int32_t* upstream,
                          const int32_t* wait_us, int32_t* cfg, uint8_t* flag, void* stream) {
  int rc = llama::enter(c);
  if (rc) return rc;
  if (!c->has_prof) return llama::fail(c, LLAMA_E_STATE, "decide_batching: no profiles");
  if (n < 0) return llama::fail(c, LLAMA_E_ARG, "decide_batching: n_inv < 0");
  if (n > 0 && (!op || !elapsed || !slo || !cfg || !available || !upstream || !wait_us))
    return llama::fail(c, LLAMA_E_ARG, "decide_batching: null pointer");
  if (mode != LLAMA_SLACK_PAPER && mode != LLAMA_SLACK_PROB)
    return llama::fail(c, LLAMA_E_ARG, "decide_batching: bad slack_mode %d", mode);
  if (n > INT32_MAX) return llama::fail(c, LLAMA_E_RANGE, "decide_batching: n_inv out of range");
  if (!queue && !llama::records_current(c, mode))
    return llama::fail(c, LLAMA_E_STATE, "decide_batching: the last relaxation left out the records of slack mode %d", mode);
  if (n == 0) return LLAMA_OK;
  hipStream_t s = (hipStream_t)stream;
  // scratch: sub-queue counters and the sub-queues (grows; not while the
  // stream is being captured)
  const size_t need = llama::batch_scratch_bytes(n, c->n_ops);
  if (need > c->d_batch_scratch.bytes) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (s && hipStreamIsCapturing(s, &cs) != hipSuccess)
      return llama::fail(c, LLAMA_E_DEVICE, "decide_batching: capture status");
    if (cs != hipStreamCaptureStatusNone)
      return llama::fail(c, LLAMA_E_STATE, "decide_batching: scratch must grow; call once before capturing");
    if (s && hipStreamSynchronize(s) != hipSuccess) return llama::fail(c, LLAMA_E_DEVICE, "decide_batching: sync");
    if ((rc = llama::upload(c, c->d_batch_scratch, nullptr, need, "batching scratch"))) return rc;
    if ((rc = llama::sync_ctx(c, "batching scratch"))) return rc;
  }
  llama::Batch b{};
  b.n = n; b.op = op; b.elapsed = elapsed; b.slo = slo; b.queue = queue; b.cfg = cfg; b.flag = flag; b.mode = mode;
  char* scratch = static_cast<char*>(c->d_batch_scratch.p);
  const int64_t slots = (int64_t)llama::BATCH_QUEUES * llama::batch_queue_capacity(n);
  int32_t* g = reinterpret_cast<int32_t*>(scratch + sizeof(uint32_t) * 32 * llama::BATCH_QUEUES +
                                          sizeof(uint2) * (size_t)slots);
  const int64_t ow = llama::batch_words64((int64_t)c->n_ops + 1);
  llama::BatchingArgs a{available, upstream, wait_us,
                        reinterpret_cast<uint2*>(scratch + sizeof(uint32_t) * 32 * llama::BATCH_QUEUES),
                        reinterpret_cast<uint32_t*>(scratch),
                        g, g + ow, g + 2 * ow, g + 3 * ow, g + 3 * ow + llama::batch_words64(slots)};
  hipError_t e = llama::launch_decide_batching(c->tables(), b, a, s);
  if (e != hipSuccess) return llama::hip_fail(c, e, "decide_batching launch");
  return LLAMA_OK;
}

int llama_affinity(llama_ctx* c, int64_t n, const int32_t* op, const int32_t* elapsed, const int32_t* slo,
                   const int64_t* queue, int32_t mode, double* aff, int32_t* order, void* stream) {
  int rc = llama::enter(c);
  if (rc) return rc;
  if (!c->has_prof) return llama::fail(c, LLAMA_E_STATE, "affinity: no profiles");
  if (!c->has_alpha) return llama::fail(c, LLAMA_E_STATE, "affinity: call llama_set_alpha first");
  if (n < 0 || n > INT32_MAX) return llama::fail(c, LLAMA_E_RANGE, "affinity: n_inv out of range");
  if (n > 0 && (!op || !elapsed || !slo || !aff)) return llama::fail(c, LLAMA_E_ARG, "affinity: null pointer");
  if (mode != LLAMA_SLACK_PAPER && mode != LLAMA_SLACK_PROB)
    return llama::fail(c, LLAMA_E_ARG, "affinity: bad slack_mode %d", mode);
  if (n == 0) return LLAMA_OK;
  hipStream_t s = (hipStream_t)stream;
  if (order) {
    // sort scratch (grows; not while the stream is being captured)
    size_t tmp = 0;
    hipError_t e = llama::sort_pairs_bytes((int)n, &tmp);
    if (e != hipSuccess) return llama::hip_fail(c, e, "affinity sort size");
    const size_t need = (((size_t)n * (8 * (size_t)c->n_hw + 8 + 4) + 255) & ~(size_t)255) + tmp;
    if (need > c->d_aff_scratch.bytes) {
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      if (s && hipStreamIsCapturing(s, &cs) != hipSuccess) return llama::fail(c, LLAMA_E_DEVICE, "affinity: capture status");
      if (cs != hipStreamCaptureStatusNone)
        return llama::fail(c, LLAMA_E_STATE, "affinity: scratch must grow; call once before capturing");
      if (s && hipStreamSynchronize(s) != hipSuccess) return llama::fail(c, LLAMA_E_DEVICE, "affinity: sync");
      if ((rc = llama::upload(c, c->d_aff_scratch, nullptr, need, "affinity scratch"))) return rc;
      if ((rc = llama::sync_ctx(c, "affinity scratch"))) return rc;
    }
  }
  llama::Batch b{};
  b.n = n; b.op = op; b.elapsed = elapsed; b.slo = slo; b.queue = queue; b.mode = mode;
  // with queueing times, one search per invocation in the per-call merged
  // order when every op fits the merge and the merge pays; else the
  // invocations grouped by op in the full scan's scratch when it holds n
  // (grown here, except while the stream is being captured), counted per
  // backend; else one thread per invocation (without queueing times, one
  // search in the static merged order)
  hipError_t e;
  if (queue && c->alpha_max_op <= llama::ALPHA_MERGE_MAX && c->d_aq_cnt.p && merge_pays(c, n)) {
    e = llama::launch_affinity_queue(c->tables(), b, aff, order, c->d_aff_scratch.p, c->d_aff_scratch.bytes, s);
  } else {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const bool capturing = s && hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
    const bool grouped = n <= c->perm_cap || (!capturing && reserve_perm(c, n, s) == LLAMA_OK);
    llama::FullScratch w{c->d_cnt.as<int32_t>(), c->d_start.as<int32_t>(), c->d_cursor.as<int32_t>(),
                         c->d_perm.as<int32_t>(), c->d_hist.as<int32_t>()};
    if (!grouped && !queue && c->d_m_cnt.p)
      e = llama::launch_affinity_queue(c->tables(), b, aff, order, c->d_aff_scratch.p, c->d_aff_scratch.bytes, s);
    else
      e = llama::launch_affinity(c->tables(), b, aff, order, c->d_aff_scratch.p, c->d_aff_scratch.bytes,
                                 grouped ? &w : nullptr, s);
  }
  if (e != hipSuccess) return llama::hip_fail(c, e, "affinity launch");
  return LLAMA_OK;
}

}  // extern "C"
