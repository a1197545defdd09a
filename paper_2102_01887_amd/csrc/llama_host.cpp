// Host side of libllama: argument validation, ingest of the pipeline DAGs
// and configuration tables into device-resident layouts, and the launches of
// the decision kernels.  Implements include/llama.h.
//
// Ingest (once per llama_set_dag / llama_set_profiles, not per decision):
//   * heights of every op above the outputs (reverse Kahn order), used by the
//     level-synchronous relaxation on the GPU; a cycle is rejected;
//   * the reference latency of each op (Sec. 3.2: smallest CPU configuration,
//     1 core and batch 1, unless the caller names one);
//   * the dense rank of each configuration's cost per item C/B within its op
//     (equal rationals share a rank), packed with the caller index as
//     key = rank << 16 | k, so that the smallest key is the cheapest
//     configuration with the lowest index among equals (Eq. 1 tie rule);
//   * the fastest configuration of each op (smallest L, lowest index);
//   * per (op, backend), the cost/latency frontier: configurations of that
//     backend sorted by latency, keeping each one whose key is smaller than
//     every faster one's.  The feasible set for any slack is a latency prefix,
//     so its cheapest member is the last frontier entry inside the prefix;
//   * the full table grouped by (op, backend) for the scan that visits every
//     configuration.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "llama.h"
#include "llama_ctx.h"
#include "llama_internal.h"

using llama::DevTables;
using llama::fail;
using llama::hip_fail;
using llama::upload;
using llama::enter;
using llama::sync_ctx;

namespace llama {

int fail(llama_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  c->err = buf;
  return code;
}

int hip_fail(llama_ctx* c, hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory)
    return fail(c, LLAMA_E_NOMEM, "%s: %s", what, hipGetErrorString(e));
  return fail(c, LLAMA_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Allocate `buf` for `bytes` and copy `src` into it (src may be null).
int upload(llama_ctx* c, DevBuf& buf, const void* src, size_t bytes, const char* what) {
  buf.release();
  size_t n = bytes ? bytes : 4;
  hipError_t e = hipMalloc(&buf.p, n);
  if (e != hipSuccess) {
    buf.p = nullptr;
    return hip_fail(c, e, what);
  }
  buf.bytes = n;
  if (src && bytes) {
    e = hipMemcpyAsync(buf.p, src, bytes, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, what);
  }
  return LLAMA_OK;
}

int enter(llama_ctx* c) {
  if (!c) return LLAMA_E_ARG;
  c->err.clear();
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  return LLAMA_OK;
}

int sync_ctx(llama_ctx* c, const char* what) {
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, what);
  return LLAMA_OK;
}

hipError_t relax_next(llama_ctx* c, hipStream_t s, int modes) {
  const int set = 1 - c->rec_cur;
  hipError_t e = launch_relax(c->tables_for(set), modes, s);
  if (e == hipSuccess) {
    c->rec_cur = set;
    c->rec_modes[set] = modes;
  }
  return e;
}

}  // namespace llama

namespace {

template <typename T>
int upload_vec(llama_ctx* c, DevBuf& buf, const std::vector<T>& v, const char* what) {
  return upload(c, buf, v.data(), v.size() * sizeof(T), what);
}

// C/B of x is smaller than C/B of y (exact: C <= 2^40, B <= 2^16).
inline bool per_item_less(const llama_ctx* c, int64_t x, int64_t y) {
  return c->cost[x] * (int64_t)c->batch[y] < c->cost[y] * (int64_t)c->batch[x];
}

int build_tables(llama_ctx* c);

}  // namespace

extern "C" {

int llama_create(llama_ctx** out, int32_t device) {
  if (!out) return LLAMA_E_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return LLAMA_E_DEVICE;
  llama_ctx* c = new (std::nothrow) llama_ctx();
  if (!c) return LLAMA_E_NOMEM;
  c->device = device;
  {
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cu > 0) c->n_cu = cu;
  }
  if (hipSetDevice(device) != hipSuccess || llama::noalloc_attach(device) != hipSuccess ||
      hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return LLAMA_E_DEVICE;
  }
  if (upload(c, c->d_err, nullptr, sizeof(uint32_t), "error word") != LLAMA_OK ||
      hipMemsetAsync(c->d_err.p, 0, sizeof(uint32_t), c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    (void)hipStreamDestroy(c->stream);
    delete c;
    return LLAMA_E_DEVICE;
  }
  *out = c;
  return LLAMA_OK;
}

void llama_destroy(llama_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* llama_last_error(const llama_ctx* c) { return c ? c->err.c_str() : "null context"; }

int llama_set_dag(llama_ctx* c, int32_t n_pipelines, const int32_t* pipe_off,
                  const int32_t* succ_off, const int32_t* succ_ids, const uint32_t* succ_q) {
  int rc = enter(c);
  if (rc) return rc;
  if (n_pipelines < 1 || !pipe_off || !succ_off)
    return fail(c, LLAMA_E_ARG, "set_dag: need n_pipelines >= 1, pipe_op_offsets and succ_offsets");
  if (pipe_off[0] != 0) return fail(c, LLAMA_E_RANGE, "set_dag: pipe_op_offsets[0] must be 0");
  for (int p = 0; p < n_pipelines; ++p)
    if (pipe_off[p + 1] < pipe_off[p])
      return fail(c, LLAMA_E_RANGE, "set_dag: pipe_op_offsets decreases at pipeline %d", p);
  const int32_t n_ops = pipe_off[n_pipelines];
  if (n_ops < 1) return fail(c, LLAMA_E_RANGE, "set_dag: no operations");
  if (succ_off[0] != 0) return fail(c, LLAMA_E_RANGE, "set_dag: succ_offsets[0] must be 0");
  for (int v = 0; v < n_ops; ++v)
    if (succ_off[v + 1] < succ_off[v])
      return fail(c, LLAMA_E_RANGE, "set_dag: succ_offsets decreases at op %d", v);
  const int64_t n_edges = succ_off[n_ops];
  if (n_edges > 0 && !succ_ids) return fail(c, LLAMA_E_ARG, "set_dag: succ_ids is null");

  c->has_dag = false;
  c->has_prof = false;
  std::vector<int32_t> pipe_of(n_ops);
  for (int p = 0; p < n_pipelines; ++p)
    for (int v = pipe_off[p]; v < pipe_off[p + 1]; ++v) pipe_of[v] = p;
  for (int v = 0; v < n_ops; ++v)
    for (int e = succ_off[v]; e < succ_off[v + 1]; ++e) {
      const int w = succ_ids[e];
      if (w < 0 || w >= n_ops) return fail(c, LLAMA_E_RANGE, "set_dag: edge %d -> %d out of range", v, w);
      if (w == v) return fail(c, LLAMA_E_CYCLE, "set_dag: self-loop at op %d", v);
      if (pipe_of[w] != pipe_of[v])
        return fail(c, LLAMA_E_RANGE, "set_dag: edge %d -> %d crosses pipelines", v, w);
      if (succ_q && (succ_q[e] < 1 || succ_q[e] > (uint32_t)LLAMA_Q_ONE))
        return fail(c, LLAMA_E_RANGE, "set_dag: branch probability %u of edge %d -> %d not in [1, 65536]",
                    succ_q[e], v, w);
    }

  // Heights above the outputs by reverse Kahn order: an op is final once all
  // of its successors are; height = 1 + max height of the successors.
  std::vector<int32_t> pred_cnt(n_ops + 1, 0), pred_off, preds(n_edges);
  for (int64_t e = 0; e < n_edges; ++e) pred_cnt[succ_ids[e] + 1]++;
  pred_off.assign(n_ops + 1, 0);
  for (int v = 0; v < n_ops; ++v) pred_off[v + 1] = pred_off[v] + pred_cnt[v + 1];
  {
    std::vector<int32_t> fill(pred_off.begin(), pred_off.end() - 1);
    for (int v = 0; v < n_ops; ++v)
      for (int e = succ_off[v]; e < succ_off[v + 1]; ++e) preds[fill[succ_ids[e]]++] = v;
  }
  std::vector<int32_t> outdeg(n_ops), height(n_ops, 0), queue;
  queue.reserve(n_ops);
  for (int v = 0; v < n_ops; ++v) {
    outdeg[v] = succ_off[v + 1] - succ_off[v];
    if (!outdeg[v]) queue.push_back(v);
  }
  for (size_t h = 0; h < queue.size(); ++h) {
    const int w = queue[h];
    for (int e = pred_off[w]; e < pred_off[w + 1]; ++e) {
      const int u = preds[e];
      height[u] = std::max(height[u], height[w] + 1);
      if (--outdeg[u] == 0) queue.push_back(u);
    }
  }
  if ((int64_t)queue.size() != n_ops) return fail(c, LLAMA_E_CYCLE, "set_dag: the successor lists contain a cycle");

  // Ops of each pipeline grouped by height (outputs first).
  std::vector<int32_t> pipe_lvl(n_pipelines + 1, 0), lvl_bnd, lvl_ops(n_ops);
  int32_t max_depth = 0, max_ops = 0, max_edges = 0;
  for (int p = 0; p < n_pipelines; ++p) {
    const int a = pipe_off[p], b = pipe_off[p + 1];
    int hmax = -1;
    for (int v = a; v < b; ++v) hmax = std::max(hmax, height[v]);
    std::vector<int32_t> cnt(hmax + 2, 0);
    for (int v = a; v < b; ++v) cnt[height[v] + 1]++;
    for (int l = 0; l <= hmax; ++l) cnt[l + 1] += cnt[l];
    for (int l = 0; l <= hmax; ++l) lvl_bnd.push_back(a + cnt[l]);
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (int v = a; v < b; ++v) lvl_ops[a + fill[height[v]]++] = v;
    pipe_lvl[p + 1] = pipe_lvl[p] + (hmax + 1);
    max_depth = std::max(max_depth, hmax + 1);
    max_ops = std::max(max_ops, b - a);
    max_edges = std::max(max_edges, succ_off[b] - succ_off[a]);
  }
  lvl_bnd.push_back(n_ops);
  std::vector<int32_t> pipe_desc((size_t)8 * n_pipelines, 0);
  for (int p = 0; p < n_pipelines; ++p) {
    int32_t* d = &pipe_desc[(size_t)8 * p];
    const int a = pipe_off[p], b = pipe_off[p + 1];
    d[0] = a;
    d[1] = b - a;
    d[2] = succ_off[a];
    d[3] = succ_off[b] - succ_off[a];
    d[4] = pipe_lvl[p];
    d[5] = pipe_lvl[p + 1] - pipe_lvl[p];
  }

  c->n_pipelines = n_pipelines;
  c->n_ops = n_ops;
  c->n_edges = n_edges;
  c->max_depth = max_depth;
  c->max_pipe_ops = max_ops;
  c->max_pipe_edges = max_edges;
  c->pipe_off.assign(pipe_off, pipe_off + n_pipelines + 1);
  c->succ_off.assign(succ_off, succ_off + n_ops + 1);
  c->succ_ids.assign(succ_ids ? succ_ids : succ_off, succ_ids ? succ_ids + n_edges : succ_off);
  if (succ_q) c->succ_q.assign(succ_q, succ_q + n_edges);
  else c->succ_q.assign(n_edges, (uint32_t)LLAMA_Q_ONE);
  c->pipe_of.swap(pipe_of);

  // Edges of each pipeline grouped by the height of their source (outputs
  // first), endpoints as pipeline-local indices packed src | dst << 16 (read
  // only for pipelines small enough to be relaxed in LDS), and the first edge
  // of each level.
  std::vector<uint32_t> lvl_edge(n_edges), lvl_edge_q(n_edges);
  std::vector<int32_t> lvl_ebnd;
  lvl_ebnd.reserve(lvl_bnd.size());
  {
    int64_t pos = 0;
    for (int p = 0; p < n_pipelines; ++p) {
      const int a = pipe_off[p];
      for (int l = pipe_lvl[p]; l < pipe_lvl[p + 1]; ++l) {
        lvl_ebnd.push_back((int32_t)pos);
        for (int idx = lvl_bnd[l]; idx < lvl_bnd[l + 1]; ++idx) {
          const int v = lvl_ops[idx];
          for (int e = succ_off[v]; e < succ_off[v + 1]; ++e) {
            lvl_edge[pos] = ((uint32_t)(v - a) & 0xFFFFu) | (((uint32_t)(succ_ids[e] - a) & 0xFFFFu) << 16);
            lvl_edge_q[pos] = c->succ_q[e];
            ++pos;
          }
        }
      }
    }
    lvl_ebnd.push_back((int32_t)pos);
  }

  if ((rc = upload_vec(c, c->d_pipe_off, c->pipe_off, "pipe_off")) ||
      (rc = upload_vec(c, c->d_lvl_edge, lvl_edge, "level edges")) ||
      (rc = upload_vec(c, c->d_lvl_edge_q, lvl_edge_q, "level edge probabilities")) ||
      (rc = upload_vec(c, c->d_lvl_ebnd, lvl_ebnd, "level edge bounds")) ||
      (rc = upload_vec(c, c->d_pipe_desc, pipe_desc, "pipeline descriptors")) ||
      (rc = upload_vec(c, c->d_lvl_bnd, lvl_bnd, "lvl_bnd")) ||
      (rc = upload_vec(c, c->d_lvl_ops, lvl_ops, "lvl_ops")) ||
      (rc = upload_vec(c, c->d_succ_off, c->succ_off, "succ_off")) ||
      (rc = upload_vec(c, c->d_succ_ids, c->succ_ids, "succ_ids")) ||
      (rc = upload_vec(c, c->d_succ_q, c->succ_q, "succ_q")))
    return rc;
  if ((rc = sync_ctx(c, "set_dag upload"))) return rc;
  c->has_dag = true;
  return LLAMA_OK;
}

int llama_set_profiles(llama_ctx* c, int32_t n_ops, int32_t n_hw, const int32_t* cfg_off,
                       const int32_t* hw, const int32_t* batch, const int32_t* res,
                       const int32_t* lat, const int64_t* cost, const int32_t* ref_cfg,
                       const int64_t* hw_res_total) {
  int rc = enter(c);
  if (rc) return rc;
  if (!c->has_dag) return fail(c, LLAMA_E_STATE, "set_profiles: call llama_set_dag first");
  if (n_ops != c->n_ops) return fail(c, LLAMA_E_STATE, "set_profiles: n_ops %d != DAG's %d", n_ops, c->n_ops);
  if (n_hw < 1 || n_hw > LLAMA_MAX_HW) return fail(c, LLAMA_E_RANGE, "set_profiles: n_hw %d not in [1, %d]", n_hw, LLAMA_MAX_HW);
  if (!cfg_off || !hw || !batch || !res || !lat || !cost)
    return fail(c, LLAMA_E_ARG, "set_profiles: null table pointer");
  if (cfg_off[0] != 0) return fail(c, LLAMA_E_RANGE, "set_profiles: cfg_offsets[0] must be 0");
  for (int v = 0; v < n_ops; ++v) {
    const int64_t k = (int64_t)cfg_off[v + 1] - cfg_off[v];
    if (k < 1 || k > LLAMA_MAX_CFG_PER_OP)
      return fail(c, LLAMA_E_RANGE, "set_profiles: op %d has %lld configurations (need 1..%d)", v,
                  (long long)k, LLAMA_MAX_CFG_PER_OP);
  }
  const int64_t n_cfg = cfg_off[n_ops];
  for (int64_t x = 0; x < n_cfg; ++x) {
    if (hw[x] < 0 || hw[x] >= n_hw) return fail(c, LLAMA_E_RANGE, "set_profiles: cfg %lld hw %d not in [0, %d)", (long long)x, hw[x], n_hw);
    if (batch[x] < 1 || batch[x] > LLAMA_MAX_BATCH) return fail(c, LLAMA_E_RANGE, "set_profiles: cfg %lld batch %d", (long long)x, batch[x]);
    if (res[x] < 1) return fail(c, LLAMA_E_RANGE, "set_profiles: cfg %lld resource %d < 1", (long long)x, res[x]);
    if (lat[x] < 1) return fail(c, LLAMA_E_RANGE, "set_profiles: cfg %lld latency %d < 1", (long long)x, lat[x]);
    if (cost[x] < 0 || cost[x] > LLAMA_MAX_COST) return fail(c, LLAMA_E_RANGE, "set_profiles: cfg %lld cost out of [0, 2^40]", (long long)x);
  }
  if (hw_res_total)
    for (int h = 0; h < n_hw; ++h)
      if (hw_res_total[h] < 1 || hw_res_total[h] > LLAMA_MAX_RES_TOTAL)
        return fail(c, LLAMA_E_RANGE, "set_profiles: hw_res_total[%d] not in [1, 2^40]", h);

  std::vector<int32_t> ref_k(n_ops);
  for (int v = 0; v < n_ops; ++v) {
    const int a = cfg_off[v], b = cfg_off[v + 1];
    if (ref_cfg) {
      if (ref_cfg[v] < 0 || ref_cfg[v] >= b - a)
        return fail(c, LLAMA_E_RANGE, "set_profiles: ref_cfg[%d] = %d out of range", v, ref_cfg[v]);
      ref_k[v] = ref_cfg[v];
      continue;
    }
    int best = -1;  // hw 0, batch 1, smallest resource, lowest index
    for (int x = a; x < b; ++x)
      if (hw[x] == 0 && batch[x] == 1 && (best < 0 || res[x] < res[best])) best = x;
    if (best < 0) return fail(c, LLAMA_E_STATE, "set_profiles: op %d has no hw-0 batch-1 configuration for the reference", v);
    ref_k[v] = best - a;
  }
  // Path latencies must stay below 2^46 so that q * W and ref * R fit int64.
  for (int p = 0; p < c->n_pipelines; ++p) {
    int64_t mx = 0;
    for (int v = c->pipe_off[p]; v < c->pipe_off[p + 1]; ++v)
      mx = std::max<int64_t>(mx, lat[cfg_off[v] + ref_k[v]]);
    const int64_t nv = c->pipe_off[p + 1] - c->pipe_off[p];
    if (mx > 0 && nv > ((int64_t)1 << 46) / mx)
      return fail(c, LLAMA_E_RANGE, "set_profiles: pipeline %d: ops * max reference latency >= 2^46", p);
  }

  c->has_prof = false;
  c->has_alpha = false;
  c->fb_ready = false;    // the feedback arrays follow the table's shape
  c->host_stale = false;
  c->perm_cap = 0;  // full-scan scratch is sized by the op count: regrow on demand
  if (hw_res_total) c->res_total.assign(hw_res_total, hw_res_total + n_hw);
  else c->res_total.clear();
  // Eq. 2 partial sums (allocated here, never during a decision call, so the
  // queueing-time launch can be captured in a graph)
  if (!c->d_qacc.p &&
      (rc = upload(c, c->d_qacc, nullptr, (size_t)16 * llama::MAX_HW * llama::QUEUE_PARTS, "queue partial sums")))
    return rc;
  c->n_hw = n_hw;
  c->n_cfg = n_cfg;
  c->cfg_off.assign(cfg_off, cfg_off + n_ops + 1);
  c->hw.assign(hw, hw + n_cfg);
  c->batch.assign(batch, batch + n_cfg);
  c->res.assign(res, res + n_cfg);
  c->lat.assign(lat, lat + n_cfg);
  c->cost.assign(cost, cost + n_cfg);
  c->ref_k.swap(ref_k);

  // Dense rank of C/B within each op -> packed keys (caller order).
  c->key.assign(n_cfg, 0);
#pragma omp parallel for schedule(dynamic, 64)
  for (int v = 0; v < n_ops; ++v) {
    const int a = c->cfg_off[v], b = c->cfg_off[v + 1];
    std::vector<int32_t> idx(b - a);
    std::iota(idx.begin(), idx.end(), a);
    std::stable_sort(idx.begin(), idx.end(), [c](int32_t x, int32_t y) { return per_item_less(c, x, y); });
    uint32_t rank = 0;
    for (size_t j = 0; j < idx.size(); ++j) {
      if (j > 0 && per_item_less(c, idx[j - 1], idx[j])) ++rank;
      c->key[idx[j]] = (rank << 16) | (uint32_t)(idx[j] - a);
    }
  }
  if ((rc = build_tables(c))) return rc;
  c->has_prof = true;
  return LLAMA_OK;
}

int llama_update_latencies(llama_ctx* c, const int32_t* lat) {
  int rc = enter(c);
  if (rc) return rc;
  if (!c->has_prof) return fail(c, LLAMA_E_STATE, "update_latencies: no profiles");
  if (!lat) return fail(c, LLAMA_E_ARG, "update_latencies: null pointer");
  for (int64_t x = 0; x < c->n_cfg; ++x)
    if (lat[x] < 1) return fail(c, LLAMA_E_RANGE, "update_latencies: cfg %lld latency %d < 1", (long long)x, lat[x]);
  for (int p = 0; p < c->n_pipelines; ++p) {
    int64_t mx = 0;
    for (int v = c->pipe_off[p]; v < c->pipe_off[p + 1]; ++v)
      mx = std::max<int64_t>(mx, lat[c->cfg_off[v] + c->ref_k[v]]);
    const int64_t nv = c->pipe_off[p + 1] - c->pipe_off[p];
    if (mx > 0 && nv > ((int64_t)1 << 46) / mx)
      return fail(c, LLAMA_E_RANGE, "update_latencies: pipeline %d: ops * max reference latency >= 2^46", p);
  }
  c->has_prof = false;
  c->host_stale = false;
  c->lat.assign(lat, lat + c->n_cfg);
  if ((rc = build_tables(c))) return rc;
  c->has_prof = true;
  if (c->has_alpha) {
    c->has_alpha = false;
    if ((rc = llama::build_alpha_tables(c))) return rc;
    c->has_alpha = true;
  }
  return LLAMA_OK;
}

int llama_relax(llama_ctx* c, void* stream) { return llama_relax_modes(c, 3, stream); }

int llama_relax_modes(llama_ctx* c, int32_t modes, void* stream) {
  int rc = enter(c);
  if (rc) return rc;
  if (!c->has_prof) return fail(c, LLAMA_E_STATE, "relax: no profiles");
  if (modes < 1 || modes > 3) return fail(c, LLAMA_E_ARG, "relax_modes: mode mask %d is not 1, 2 or 3", modes);
  hipError_t e = llama::relax_next(c, (hipStream_t)stream, modes);
  if (e != hipSuccess) return hip_fail(c, e, "relax launch");
  return LLAMA_OK;
}

}  // extern "C"

namespace {

// Everything derived from the latencies: reference latency, fastest config,
// frontiers, full table; then W and thresholds on the GPU.
int build_tables(llama_ctx* c) {
  const int n_ops = c->n_ops, n_hw = c->n_hw;
  const int hs = llama::header_stride(n_hw);
  c->ref.assign(n_ops, 0);
  c->fastest.assign(n_ops, 0);
  std::vector<int32_t> seg_off((size_t)n_ops * n_hw + 1, 0);
  std::vector<int64_t> front_cnt((size_t)n_ops * n_hw, 0);
  std::vector<uint2> tab(c->n_cfg);

  // Pass 1: per op, reference, fastest, backend segments of the full table,
  // and frontier sizes.
  std::vector<std::vector<uint2>> fronts(n_ops);
#pragma omp parallel for schedule(dynamic, 64)
  for (int v = 0; v < n_ops; ++v) {
    const int a = c->cfg_off[v], b = c->cfg_off[v + 1];
    c->ref[v] = c->lat[a + c->ref_k[v]];
    int f = a;
    for (int x = a + 1; x < b; ++x)
      if (c->lat[x] < c->lat[f]) f = x;
    c->fastest[v] = f - a;
    std::vector<int32_t> cnt(n_hw + 1, 0);
    for (int x = a; x < b; ++x) cnt[c->hw[x] + 1]++;
    for (int h = 0; h < n_hw; ++h) cnt[h + 1] += cnt[h];
    std::vector<int32_t> order(b - a);
    {
      std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
      for (int x = a; x < b; ++x) order[fill[c->hw[x]]++] = x;  // stable by caller index
    }
    for (int j = 0; j < b - a; ++j) tab[a + j] = make_uint2((uint32_t)c->lat[order[j]], c->key[order[j]]);
    for (int h = 0; h < n_hw; ++h) seg_off[(size_t)v * n_hw + h] = a + cnt[h];
    // frontier of each backend: latency ascending (key ascending among equal
    // latencies); keep entries whose key beats every faster entry's.
    std::vector<uint2>& fr = fronts[v];
    for (int h = 0; h < n_hw; ++h) {
      std::vector<int32_t> s(order.begin() + cnt[h], order.begin() + cnt[h + 1]);
      std::sort(s.begin(), s.end(), [c](int32_t x, int32_t y) {
        return c->lat[x] != c->lat[y] ? c->lat[x] < c->lat[y] : c->key[x] < c->key[y];
      });
      uint32_t best = llama::KEY_NONE;
      int64_t kept = 0;
      for (int32_t x : s)
        if (c->key[x] < best) {
          best = c->key[x];
          fr.push_back(make_uint2((uint32_t)c->lat[x], c->key[x]));
          ++kept;
        }
      front_cnt[(size_t)v * n_hw + h] = kept;
    }
  }
  seg_off[(size_t)n_ops * n_hw] = (int32_t)c->n_cfg;

  // Queue-free merged frontier of each op over all backends: latency
  // ascending (key ascending among equal latencies), keeping each entry whose
  // key beats every faster one's.  Its thresholds are refreshed on the GPU
  // after every relaxation; the record's other words are fixed here.
  std::vector<std::vector<uint2>> merged(n_ops);
#pragma omp parallel for schedule(dynamic, 64)
  for (int v = 0; v < n_ops; ++v) {
    std::vector<uint2> all(fronts[v]);
    std::sort(all.begin(), all.end(), [](const uint2& p, const uint2& q) {
      return p.x != q.x ? p.x < q.x : p.y < q.y;
    });
    uint32_t best = llama::KEY_NONE;
    for (const uint2& e : all)
      if (e.y < best) {
        best = e.y;
        merged[v].push_back(e);
      }
  }
  // Capacity layout: every per-op structure (merged frontier, per-backend
  // frontiers, overflow) lives inside the op's own configuration range
  // [cfg_off[v], cfg_off[v+1]), which bounds its size, so a rebuild on the
  // device (after feedback) never moves another op's data.
  std::vector<int32_t> mst_n(n_ops, 0);
  for (int v = 0; v < n_ops; ++v) mst_n[v] = (int32_t)merged[v].size();
  std::vector<uint2> mst(c->n_cfg);
  std::vector<uint4> rec_hot((size_t)2 * n_ops), rec_tail((size_t)2 * n_ops * llama::REC_TAIL_VECS),
      rec_tail2((size_t)2 * n_ops * llama::REC_TAIL2_VECS);
  for (int v = 0; v < n_ops; ++v) {
    const int n = (int)merged[v].size();
    for (int j = 0; j < n; ++j) {
      mst[c->cfg_off[v] + j] = merged[v][j];
    }
    uint32_t w[llama::REC_WORDS] = {0};
    // thresholds (and the code of the smallest) are written by the GPU after relaxation
    w[0] = (uint32_t)c->fastest[v] | (0xFFFFu << 16);
    w[llama::REC_N_WORD] = (uint32_t)n;
    for (int slot = 0; slot < llama::REC_SLOTS; ++slot) {
      const int j = n - 1 - slot;
      w[llama::rec_u_word(slot)] = 0x7FFFFFFFu;
      const uint32_t k = j >= 0 ? (merged[v][j].y & 0xFFFFu) : 0u;
      w[llama::rec_k_word(slot)] |= k << llama::rec_k_shift(slot);
    }
    for (int mode = 0; mode < 2; ++mode)
      for (int k = 0; k < llama::REC_WORDS; ++k)
        *llama::rec_word(rec_hot.data(), rec_tail.data(), rec_tail2.data(), (int64_t)mode * n_ops + v, k) = w[k];
  }
  merged.clear();

  // Pass 2: frontier offsets and headers.
  std::vector<int32_t> hdr((size_t)n_ops * hs, 0);
  int64_t n_entries = 0;
  for (int v = 0; v < n_ops; ++v) {
    int64_t pos = c->cfg_off[v];
    for (int h = 0; h < n_hw; ++h) {
      hdr[(size_t)v * hs + h] = (int32_t)pos;
      pos += front_cnt[(size_t)v * n_hw + h];
    }
    hdr[(size_t)v * hs + n_hw] = (int32_t)pos;
    hdr[(size_t)v * hs + n_hw + 1] = c->fastest[v];
    n_entries += pos - c->cfg_off[v];
  }
  c->n_front = n_entries;
  const int64_t pos = c->n_cfg;  // capacity of the frontier and overflow arrays
  std::vector<uint2> front_L(pos);
#pragma omp parallel for schedule(dynamic, 64)
  for (int v = 0; v < n_ops; ++v)
    std::copy(fronts[v].begin(), fronts[v].end(), front_L.begin() + hdr[(size_t)v * hs]);
  fronts.clear();

  int rc;
  if ((rc = upload_vec(c, c->d_ref, c->ref, "ref")) ||
      (rc = upload(c, c->d_W, nullptr, sizeof(int64_t) * 2 * (size_t)n_ops, "W")) ||
      (rc = upload_vec(c, c->d_hdr, hdr, "hdr")) ||
      (rc = upload_vec(c, c->d_front_L, front_L, "front_L")) ||
      (rc = upload_vec(c, c->d_rec[0], rec_hot, "records")) ||
      (rc = upload_vec(c, c->d_rec_tail[0], rec_tail, "record tails")) ||
      (rc = upload_vec(c, c->d_rec_tail2[0], rec_tail2, "record second tails")) ||
      (rc = upload_vec(c, c->d_rec[1], rec_hot, "records")) ||
      (rc = upload_vec(c, c->d_rec_tail[1], rec_tail, "record tails")) ||
      (rc = upload_vec(c, c->d_rec_tail2[1], rec_tail2, "record second tails")) ||
      (rc = upload_vec(c, c->d_mst, mst, "merged frontier")) ||
      (rc = upload_vec(c, c->d_mst_n, mst_n, "merged frontier sizes")) ||
      (rc = upload(c, c->d_ovf[0], nullptr, sizeof(uint2) * 2 * (size_t)pos, "record overflow")) ||
      (rc = upload(c, c->d_ovf[1], nullptr, sizeof(uint2) * 2 * (size_t)pos, "record overflow")) ||
      (rc = upload(c, c->d_rec_q, nullptr, sizeof(uint4) * (size_t)n_ops, "records (queue)")) ||
      (rc = upload(c, c->d_rec_tail_q, nullptr, sizeof(uint4) * llama::REC_TAIL_VECS * (size_t)n_ops, "record tails (queue)")) ||
      (rc = upload(c, c->d_rec_tail2_q, nullptr, sizeof(uint4) * llama::REC_TAIL2_VECS * (size_t)n_ops, "record second tails (queue)")) ||
      (rc = upload(c, c->d_ovf_q, nullptr, sizeof(uint2) * (size_t)pos, "record overflow (queue)")) ||
      (rc = upload_vec(c, c->d_seg_off, seg_off, "seg_off")) ||
      (rc = upload_vec(c, c->d_cfg_off, c->cfg_off, "cfg_off")) ||
      (rc = upload_vec(c, c->d_cfg_hw, c->hw, "cfg_hw")) ||
      (rc = upload_vec(c, c->d_cfg_lat, c->lat, "cfg_lat")) ||
      (rc = upload_vec(c, c->d_cfg_batch, c->batch, "cfg_batch")) ||
      (rc = upload_vec(c, c->d_cfg_key, c->key, "cfg_key")) ||
      (rc = upload(c, c->d_cnt, nullptr, sizeof(int32_t) * ((size_t)n_ops + 1), "bucket counts")) ||
      (rc = upload(c, c->d_start, nullptr, sizeof(int32_t) * ((size_t)n_ops + 1), "bucket starts")) ||
      (rc = upload(c, c->d_cursor, nullptr, sizeof(int32_t) * (size_t)n_ops, "bucket cursors")) ||
      (rc = upload_vec(c, c->d_tab, tab, "tab")))
    return rc;
  // Eq. 2 reads, per queued invocation, one 16-byte record {L, R, hw, 0} of
  // its configuration (only with resource limits); the host copy lives until
  // the synchronisation below, like every staged table here
  std::vector<uint4> cq;
  if (!c->res_total.empty()) {
    cq.resize(c->n_cfg);
    for (int64_t x = 0; x < c->n_cfg; ++x)
      cq[x] = make_uint4((uint32_t)c->lat[x], (uint32_t)c->res[x], (uint32_t)c->hw[x], 0u);
    if ((rc = upload_vec(c, c->d_cfg_q, cq, "queue records"))) return rc;
  } else {
    c->d_cfg_q.release();
  }
  hipError_t e = llama::relax_next(c, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "relax launch");
  return sync_ctx(c, "set_profiles");
}


int check_batch(llama_ctx* c, int64_t n, const void* op, const char* fn) {
  if (!c->has_prof) return fail(c, LLAMA_E_STATE, "%s: call llama_set_dag and llama_set_profiles first", fn);
  if (n < 0) return fail(c, LLAMA_E_ARG, "%s: n_inv < 0", fn);
  if (n > 0 && !op) return fail(c, LLAMA_E_ARG, "%s: null invocation pointer", fn);
  return LLAMA_OK;
}

}  // namespace

int reserve_perm(llama_ctx* c, int64_t n, hipStream_t stream) {
  if (n <= c->perm_cap) return LLAMA_OK;
  if (n > INT32_MAX) return fail(c, LLAMA_E_RANGE, "full scan: more than 2^31-1 invocations in one call");
  if (stream) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &st) == hipSuccess && st != hipStreamCaptureStatusNone)
      return fail(c, LLAMA_E_STATE, "full scan: scratch for %lld invocations must be reserved before graph capture (llama_reserve)", (long long)n);
  }
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(c, e, "reserve sync");
  int rc = upload(c, c->d_perm, nullptr, sizeof(int32_t) * (size_t)n, "full-scan permutation");
  if (!rc)
    rc = upload(c, c->d_hist, nullptr, sizeof(int32_t) * (size_t)llama::full_scan_hist_words(n, c->n_ops),
                "full-scan histograms");
  if (rc) {
    c->perm_cap = 0;
    return rc;
  }
  c->perm_cap = n;
  return LLAMA_OK;
}

extern "C" {

int llama_targets(llama_ctx* c, int64_t n, const int32_t* op, const int32_t* elapsed,
                  const int32_t* slo, const int64_t* queue, int32_t mode, int32_t* target,
                  void* stream) {
  int rc = enter(c);
  if (rc) return rc;
  if ((rc = check_batch(c, n, op, "targets"))) return rc;
  if (n > 0 && (!elapsed || !slo || !target)) return fail(c, LLAMA_E_ARG, "targets: null pointer");
  if (mode != LLAMA_SLACK_PAPER && mode != LLAMA_SLACK_PROB) return fail(c, LLAMA_E_ARG, "targets: bad slack_mode %d", mode);
  llama::Batch b{};
  b.n = n; b.op = op; b.elapsed = elapsed; b.slo = slo; b.queue = queue; b.target_out = target; b.mode = mode;
  hipError_t e = llama::launch_targets(c->tables(), b, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "targets launch");
  return LLAMA_OK;
}

int llama_select(llama_ctx* c, int64_t n, const int32_t* op, const int32_t* target, int32_t* cfg,
                 uint8_t* flag, void* stream) {
  int rc = enter(c);
  if (rc) return rc;
  if ((rc = check_batch(c, n, op, "select"))) return rc;
  if (n > 0 && (!target || !cfg)) return fail(c, LLAMA_E_ARG, "select: null pointer");
  llama::Batch b{};
  b.n = n; b.op = op; b.target = target; b.cfg = cfg; b.flag = flag;
  hipError_t e = llama::launch_select_indexed(c->tables(), b, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "select launch");
  return LLAMA_OK;
}

int llama_decide(llama_ctx* c, int64_t n, const int32_t* op, const int32_t* elapsed,
                 const int32_t* slo, const int64_t* queue, int32_t mode, int32_t scan,
                 int32_t* cfg, uint8_t* flag, void* stream) {
  int rc = enter(c);
  if (rc) return rc;
  if ((rc = check_batch(c, n, op, "decide"))) return rc;
  if (n > 0 && (!elapsed || !slo || !cfg)) return fail(c, LLAMA_E_ARG, "decide: null pointer");
  if (mode != LLAMA_SLACK_PAPER && mode != LLAMA_SLACK_PROB) return fail(c, LLAMA_E_ARG, "decide: bad slack_mode %d", mode);
  if (scan < LLAMA_SCAN_AUTO || scan > LLAMA_SCAN_WAVE) return fail(c, LLAMA_E_ARG, "decide: bad scan_mode %d", scan);
  llama::Batch b{};
  b.n = n; b.op = op; b.elapsed = elapsed; b.slo = slo; b.queue = queue; b.cfg = cfg; b.flag = flag; b.mode = mode;
  hipError_t e;
  if (scan == LLAMA_SCAN_FULL) {
    if ((rc = reserve_perm(c, n, (hipStream_t)stream))) return rc;
    llama::FullScratch w{c->d_cnt.as<int32_t>(), c->d_start.as<int32_t>(), c->d_cursor.as<int32_t>(),
                         c->d_perm.as<int32_t>(), c->d_hist.as<int32_t>()};
    e = llama::launch_decide_full(c->tables(), b, w, (hipStream_t)stream);
  } else if (scan == LLAMA_SCAN_WAVE) {
    e = llama::launch_decide_wave(c->tables(), b, (hipStream_t)stream);
  } else {
    if (!queue && !llama::records_current(c, mode))
      return fail(c, LLAMA_E_STATE, "decide: the last relaxation left out the records of slack mode %d (llama_relax_modes)", mode);
    e = llama::launch_decide_indexed(c->tables(), b, (hipStream_t)stream);
  }
  if (e != hipSuccess) return hip_fail(c, e, "decide launch");
  return LLAMA_OK;
}

int llama_select_rows(llama_ctx* c, int64_t n, const int32_t* op, const int32_t* target, const int32_t* lat,
                      int64_t lat_stride, int32_t* cfg, uint8_t* flag, void* stream) {
  int rc = enter(c);
  if (rc) return rc;
  if ((rc = check_batch(c, n, op, "select_rows"))) return rc;
  if (n > 0 && (!target || !lat || !cfg)) return fail(c, LLAMA_E_ARG, "select_rows: null pointer");
  if (lat_stride < 1) return fail(c, LLAMA_E_ARG, "select_rows: lat_stride < 1");
  llama::Batch b{};
  b.n = n; b.op = op; b.target = target; b.cfg = cfg; b.flag = flag;
  hipError_t e = llama::launch_select_rows(c->tables(), b, lat, lat_stride, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "select_rows launch");
  return LLAMA_OK;
}

int llama_autotune(llama_ctx* c, int64_t n, const int32_t* op, const int32_t* elapsed, const int32_t* slo,
                   int32_t* cfg_scratch, int32_t* chosen_ipt, float* best_us, void* stream) {
  int rc = enter(c);
  if (rc) return rc;
  if ((rc = check_batch(c, n, op, "autotune"))) return rc;
  if (n < 1 || !elapsed || !slo || !cfg_scratch) return fail(c, LLAMA_E_ARG, "autotune: need a non-empty batch and scratch");
  hipStream_t s = (hipStream_t)stream;
  std::vector<int> cands = {llama::SCHED_DIRECT1, llama::SCHED_DIRECT2, llama::SCHED_DIRECT4,
                            llama::SCHED_DIRECT1_NT, llama::SCHED_DIRECT2_NT, llama::SCHED_DIRECT4_NT};
  if (c->n_ops <= llama::LDS_REC_MAX_OPS) cands.push_back(llama::SCHED_LDS);
  float best = 0.0f;
  int best_ipt = llama::SCHED_DIRECT1;
  std::vector<int32_t> ref_out, out;
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return fail(c, LLAMA_E_DEVICE, "autotune events");
  const int saved = c->decide_sched;
  for (size_t ci = 0; ci < cands.size(); ++ci) {
    c->decide_sched = cands[ci];
    llama::Batch bt{};
    bt.n = n; bt.op = op; bt.elapsed = elapsed; bt.slo = slo; bt.cfg = cfg_scratch;
    bt.mode = llama::records_current(c, LLAMA_SLACK_PAPER) ? LLAMA_SLACK_PAPER : LLAMA_SLACK_PROB;
    hipError_t e = llama::launch_decide_indexed(c->tables(), bt, s);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(a, s);
    for (int r = 0; r < 10 && e == hipSuccess; ++r) e = llama::launch_decide_indexed(c->tables(), bt, s);
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    // every schedule must give the same decisions
    out.resize(n);
    if (e == hipSuccess) e = hipMemcpy(out.data(), cfg_scratch, sizeof(int32_t) * n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      c->decide_sched = saved;
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
      return hip_fail(c, e, "autotune");
    }
    if (ci == 0) ref_out = out;
    else if (out != ref_out) {
      c->decide_sched = saved;
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
      return fail(c, LLAMA_E_DEVICE, "autotune: schedule %d changed the decisions", cands[ci]);
    }
    const float us = ms * 100.0f;  // ms / 10 launches, in us
    if (ci == 0 || us < best) {
      best = us;
      best_ipt = cands[ci];
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  c->decide_sched = best_ipt;
  if (chosen_ipt) *chosen_ipt = best_ipt;
  if (best_us) *best_us = best;
  return LLAMA_OK;
}

int llama_set_schedule(llama_ctx* c, int32_t schedule) {
  int rc = enter(c);
  if (rc) return rc;
  if (schedule < llama::SCHED_DIRECT1 || schedule > llama::SCHED_DIRECT4_NT)
    return fail(c, LLAMA_E_ARG, "set_schedule: schedule %d outside 0..6", schedule);
  if (schedule == llama::SCHED_LDS && c->n_ops > llama::LDS_REC_MAX_OPS)
    return fail(c, LLAMA_E_ARG, "set_schedule: the LDS schedule needs at most %d ops", llama::LDS_REC_MAX_OPS);
  c->decide_sched = schedule;
  return LLAMA_OK;
}

int llama_autotune_full(llama_ctx* c, int64_t n, const int32_t* op, const int32_t* elapsed, const int32_t* slo,
                        int32_t slack_mode, int32_t* cfg_scratch, int32_t* cross_num, int32_t* cross_den,
                        float* best_us, void* stream) {
  int rc = enter(c);
  if (rc) return rc;
  if ((rc = check_batch(c, n, op, "autotune_full"))) return rc;
  if (n < 1 || !elapsed || !slo || !cfg_scratch)
    return fail(c, LLAMA_E_ARG, "autotune_full: need a non-empty batch and scratch");
  if (slack_mode != LLAMA_SLACK_PAPER && slack_mode != LLAMA_SLACK_PROB)
    return fail(c, LLAMA_E_ARG, "autotune_full: bad slack_mode %d", slack_mode);
  hipStream_t s = (hipStream_t)stream;
  if ((rc = reserve_perm(c, n, s))) return rc;
  // crossovers, from "lanes = configurations unless far cheaper" to "lanes =
  // invocations unless far cheaper", and the two pure layouts
  const int32_t cands[][2] = {{1, 4}, {1, 2}, {1, 1}, {2, 1}, {4, 1}, {0, 1}, {1 << 20, 1}};
  const int n_c = (int)(sizeof(cands) / sizeof(cands[0]));
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return fail(c, LLAMA_E_DEVICE, "autotune_full events");
  const int32_t saved_num = c->full_cross_num, saved_den = c->full_cross_den;
  std::vector<int32_t> ref_out, out;
  float best = 0.0f;
  int best_i = 2;
  hipError_t e = hipSuccess;
  for (int ci = 0; ci < n_c && e == hipSuccess; ++ci) {
    c->full_cross_num = cands[ci][0];
    c->full_cross_den = cands[ci][1];
    llama::Batch bt{};
    bt.n = n; bt.op = op; bt.elapsed = elapsed; bt.slo = slo; bt.cfg = cfg_scratch; bt.mode = slack_mode;
    llama::FullScratch w{c->d_cnt.as<int32_t>(), c->d_start.as<int32_t>(), c->d_cursor.as<int32_t>(),
                         c->d_perm.as<int32_t>(), c->d_hist.as<int32_t>()};
    e = llama::launch_decide_full(c->tables(), bt, w, s);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(a, s);
    for (int r = 0; r < 5 && e == hipSuccess; ++r) e = llama::launch_decide_full(c->tables(), bt, w, s);
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    out.resize(n);
    if (e == hipSuccess) e = hipMemcpy(out.data(), cfg_scratch, sizeof(int32_t) * n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) break;
    if (ci == 0) {
      ref_out = out;
    } else if (out != ref_out) {
      c->full_cross_num = saved_num;
      c->full_cross_den = saved_den;
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
      return fail(c, LLAMA_E_DEVICE, "autotune_full: crossover %d/%d changed the decisions", cands[ci][0], cands[ci][1]);
    }
    const float us = ms * 200.0f;  // ms / 5 launches, in us
    if (ci == 0 || us < best) {
      best = us;
      best_i = ci;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) {
    c->full_cross_num = saved_num;
    c->full_cross_den = saved_den;
    return hip_fail(c, e, "autotune_full");
  }
  c->full_cross_num = cands[best_i][0];
  c->full_cross_den = cands[best_i][1];
  if (cross_num) *cross_num = c->full_cross_num;
  if (cross_den) *cross_den = c->full_cross_den;
  if (best_us) *best_us = best;
  return LLAMA_OK;
}

int llama_set_full_schedule(llama_ctx* c, int32_t cross_num, int32_t cross_den) {
  int rc = enter(c);
  if (rc) return rc;
  if (cross_num < 0 || cross_den < 1 || cross_num > (1 << 20))
    return fail(c, LLAMA_E_ARG, "set_full_schedule: need 0 <= num <= 2^20 and den >= 1");
  c->full_cross_num = cross_num;
  c->full_cross_den = cross_den;
  return LLAMA_OK;
}

int llama_reserve(llama_ctx* c, int64_t max_inv) {
  int rc = enter(c);
  if (rc) return rc;
  if (max_inv < 0) return fail(c, LLAMA_E_ARG, "reserve: negative size");
  return reserve_perm(c, max_inv, nullptr);
}

int llama_get_stats(llama_ctx* c, llama_stats* out, int32_t reset_error) {
  int rc = enter(c);
  if (rc) return rc;
  if (!out) return fail(c, LLAMA_E_ARG, "get_stats: null pointer");
  std::memset(out, 0, sizeof *out);
  out->n_ops = c->n_ops;
  out->n_hw = c->n_hw;
  out->n_pipelines = c->n_pipelines;
  out->max_depth = c->max_depth;
  out->n_cfg = c->n_cfg;
  out->n_edges = c->n_edges;
  out->frontier_entries = c->n_front;
  out->device_bytes = c->device_bytes();
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(c, e, "get_stats sync");
  uint32_t w = 0;
  e = hipMemcpy(&w, c->d_err.p, sizeof w, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, "get_stats read");
  out->device_error = w;
  if (reset_error) {
    e = hipMemset(c->d_err.p, 0, sizeof(uint32_t));
    if (e != hipSuccess) return hip_fail(c, e, "get_stats reset");
  }
  return LLAMA_OK;
}

int llama_debug_export(llama_ctx* c, int32_t what, void* out, int64_t bytes) {
  int rc = enter(c);
  if (rc) return rc;
  if (!out) return fail(c, LLAMA_E_ARG, "debug_export: null pointer");
  if (!c->has_prof) return fail(c, LLAMA_E_STATE, "debug_export: no profiles");
  if ((rc = llama::pull_profiles(c))) return rc;
  const void* src = nullptr;
  int64_t need = 0;
  bool device = false;
  switch (what) {
    case 0: src = c->d_W.p; need = 8ll * c->n_ops; device = true; break;
    case 1: src = c->d_W.as<int64_t>() + c->n_ops; need = 8ll * c->n_ops; device = true; break;
    case 2: src = c->key.data(); need = 4ll * c->n_cfg; break;
    case 3: src = c->ref.data(); need = 4ll * c->n_ops; break;
    case 4: src = c->fastest.data(); need = 4ll * c->n_ops; break;
    case 5: src = c->lat.data(); need = 4ll * c->n_cfg; break;
    default: return fail(c, LLAMA_E_ARG, "debug_export: unknown table %d", what);
  }
  if (bytes < need) return fail(c, LLAMA_E_ARG, "debug_export: need %lld bytes", (long long)need);
  if (!device) {
    std::memcpy(out, src, need);
    return LLAMA_OK;
  }
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(out, src, need, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, "debug_export copy");
  return LLAMA_OK;
}

}  // extern "C"
