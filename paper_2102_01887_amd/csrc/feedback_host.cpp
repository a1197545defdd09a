// Host side of the feedback step (Sec. 3.3, Manager: the profile is updated
// from observed latencies by exponential smoothing): argument checks, the
// static helper arrays of the device rebuild, and the launches.  Implements
// llama_feedback of include/llama.h.
//
// After the smoothing, every latency-derived table of the ops that had an
// observation is rebuilt on the device
// (reference latencies, fastest configurations, per-backend and merged
// frontiers, the full table's latencies) and the relaxation runs, so that the
// next decision uses the new profile.  The host copy of the latencies is
// refreshed lazily, only when a host-side function needs it.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "llama.h"
#include "llama_ctx.h"
#include "llama_internal.h"

namespace llama {

// Static arrays of the rebuild and the zeroed accumulators (first call).
int prepare_feedback(llama_ctx* c) {
  if (c->fb_ready) return LLAMA_OK;
  const int n_ops = c->n_ops, n_hw = c->n_hw;
  const int64_t n_cfg = c->n_cfg;
  std::vector<int32_t> ksrc(n_cfg);
  std::vector<int32_t> tab_src(n_cfg);
  for (int v = 0; v < n_ops; ++v) {
    const int a = c->cfg_off[v], b = c->cfg_off[v + 1];
    std::iota(ksrc.begin() + a, ksrc.begin() + b, a);
    std::sort(ksrc.begin() + a, ksrc.begin() + b, [&](int32_t p, int32_t q) { return c->key[p] < c->key[q]; });
    // the full table's order: grouped by backend, caller order inside
    std::vector<int32_t> cnt(n_hw + 1, 0);
    for (int x = a; x < b; ++x) cnt[c->hw[x] + 1]++;
    for (int h = 0; h < n_hw; ++h) cnt[h + 1] += cnt[h];
    for (int x = a; x < b; ++x) tab_src[a + cnt[c->hw[x]]++] = x;
  }
  int rc;
  if ((rc = upload(c, c->d_fb_ksrc, ksrc.data(), ksrc.size() * 4, "feedback key order")) ||
      (rc = upload(c, c->d_fb_tab_src, tab_src.data(), tab_src.size() * 4, "feedback table order")) ||
      (rc = upload(c, c->d_fb_ref_k, c->ref_k.data(), c->ref_k.size() * 4, "feedback reference configs")) ||
      (rc = upload(c, c->d_fb_count, nullptr, 4 * (size_t)n_cfg, "feedback counts")) ||
      (rc = upload(c, c->d_fb_sum, nullptr, 8 * (size_t)n_cfg, "feedback sums")) ||
      (rc = upload(c, c->d_fb_dirty, nullptr, 4 * (size_t)n_ops, "feedback op flags")))
    return rc;
  hipError_t e = hipMemsetAsync(c->d_fb_count.p, 0, 4 * (size_t)n_cfg, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->d_fb_sum.p, 0, 8 * (size_t)n_cfg, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->d_fb_dirty.p, 0, 4 * (size_t)n_ops, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "feedback scratch");
  if ((rc = sync_ctx(c, "feedback set-up"))) return rc;
  c->fb_ready = true;
  return LLAMA_OK;
}

// Host copies of the latencies, reference latencies and fastest
// configurations after device-side feedback.
int pull_profiles(llama_ctx* c) {
  if (!c->host_stale) return LLAMA_OK;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(c->lat.data(), c->d_cfg_lat.p, 4 * (size_t)c->n_cfg, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, "pull latencies");
  for (int v = 0; v < c->n_ops; ++v) {
    const int a = c->cfg_off[v], b = c->cfg_off[v + 1];
    c->ref[v] = c->lat[a + c->ref_k[v]];
    int f = a;
    for (int x = a + 1; x < b; ++x)
      if (c->lat[x] < c->lat[f]) f = x;
    c->fastest[v] = f - a;
  }
  c->host_stale = false;
  return LLAMA_OK;
}

}  // namespace llama

extern "C" {

int llama_feedback(llama_ctx* c, int64_t n, const int32_t* obs_op, const int32_t* obs_cfg, const int32_t* obs_lat,
                   uint32_t beta_q16, void* stream) {
  int rc = llama::enter(c);
  if (rc) return rc;
  if (!c->has_prof) return llama::fail(c, LLAMA_E_STATE, "feedback: no profiles");
  if (n < 0) return llama::fail(c, LLAMA_E_ARG, "feedback: n_obs < 0");
  if (n > 0 && (!obs_op || !obs_cfg || !obs_lat)) return llama::fail(c, LLAMA_E_ARG, "feedback: null pointer");
  if (beta_q16 > 65536u) return llama::fail(c, LLAMA_E_ARG, "feedback: beta_q16 above 65536");
  if (n > INT32_MAX) return llama::fail(c, LLAMA_E_RANGE, "feedback: more than 2^31-1 observations");
  if (c->max_pipe_ops >= (1 << 15))
    return llama::fail(c, LLAMA_E_RANGE, "feedback: a pipeline has 2^15 or more ops");
  if ((rc = llama::prepare_feedback(c))) return rc;
  llama::DevTables t = c->tables();
  llama::FeedbackArgs f{};
  f.lat = c->d_cfg_lat.as<int32_t>();
  f.count = c->d_fb_count.as<uint32_t>();
  f.sum = c->d_fb_sum.as<unsigned long long>();
  f.dirty = c->d_fb_dirty.as<uint32_t>();
  f.ksrc = c->d_fb_ksrc.as<int32_t>();
  f.ref_k = c->d_fb_ref_k.as<int32_t>();
  f.tab_src = c->d_fb_tab_src.as<int32_t>();
  f.ref = c->d_ref.as<int32_t>();
  f.hdr = c->d_hdr.as<int32_t>();
  f.front = c->d_front_L.as<uint2>();
  f.mst = c->d_mst.as<uint2>();
  f.mst_n = c->d_mst_n.as<int32_t>();
  f.tab = c->d_tab.as<uint2>();
  f.cfg_q = c->d_cfg_q.p ? c->d_cfg_q.as<uint4>() : nullptr;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = llama::launch_feedback(t, f, n, obs_op, obs_cfg, obs_lat, beta_q16, s);
  if (e == hipSuccess) e = llama::relax_next(c, s);
  if (e != hipSuccess) return llama::hip_fail(c, e, "feedback launch");
  c->host_stale = true;
  c->has_alpha = false;  // the finite-alpha tables follow the latencies: llama_set_alpha again
  return LLAMA_OK;
}

}  // extern "C"
