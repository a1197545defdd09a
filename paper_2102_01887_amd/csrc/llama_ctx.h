// Internal: the context object shared by the host sources of libllama.
#pragma once

#include <hip/hip_runtime_api.h>

#include <string>
#include <vector>

#include "llama.h"
#include "llama_internal.h"

namespace llama {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

// Learned-surrogate state (surrogate_host.cpp).
struct Surrogate {
  bool ready = false;
  int64_t n_rows = 0, n_params = 0, step = 0;
  DevBuf master, adam_m, adam_v, grad;              // fp32 [n_params], layout E, W1, b1, W2, b2, W3, b3
  DevBuf E16, W1_16, W2_16, W2p16, W3_16;           // bf16 shadows
  DevBuf W1T16, W2T16;                              // transposed bf16 shadows (backward products)
  DevBuf dE;                                        // int64 [nE] embedding-gradient accumulator (2^-40 units), zero between steps
  int64_t ws_batch = 0;                             // forward workspace capacity (rows)
  DevBuf X16, z1, h1, z2, h2, out;
  int64_t part_chunks = 0;                          // training partial-gradient capacity (chunks)
  DevBuf part;                                      // fp32 [part_chunks][n_params - nE]
};

}  // namespace llama

using llama::DevBuf;
using llama::DevTables;


struct llama_ctx {
  int device = 0;
  std::string err;
  hipStream_t stream = nullptr;  // the context's own stream for ingest work

  // DAG
  bool has_dag = false;
  int32_t n_pipelines = 0, n_ops = 0, max_depth = 0;
  int32_t max_pipe_ops = 0, max_pipe_edges = 0;  // largest pipeline (ops, edges)
  int64_t n_edges = 0;
  std::vector<int32_t> pipe_off, succ_off, succ_ids, pipe_of;
  std::vector<uint32_t> succ_q;
  DevBuf d_pipe_off, d_pipe_desc, d_lvl_bnd, d_lvl_ops, d_succ_off, d_succ_ids, d_succ_q;
  DevBuf d_lvl_edge, d_lvl_edge_q, d_lvl_ebnd;

  // profiles
  bool has_prof = false;
  int32_t n_hw = 0;
  int64_t n_cfg = 0, n_front = 0;
  std::vector<int32_t> cfg_off, hw, batch, res, lat, ref_k, ref, fastest;
  std::vector<int64_t> cost;
  std::vector<uint32_t> key;  // caller order
  DevBuf d_ref, d_W, d_hdr, d_front_L, d_rec_q, d_rec_tail_q, d_rec_tail2_q, d_ovf_q, d_seg_off, d_tab;
  // Decision records, double-buffered: each relaxation writes the set the
  // previous one did not, and decisions read the set of the latest one, so a
  // relaxation can overlap the decisions of the batch before it.
  DevBuf d_rec[2], d_rec_tail[2], d_rec_tail2[2], d_ovf[2];
  int rec_cur = 0;  // set written by the latest relaxation
  int rec_modes[2] = {3, 3};  // slack modes (bit m = mode m) whose records each set holds
  DevBuf d_mst, d_mst_n;
  DevBuf d_cfg_off, d_cfg_hw, d_cfg_lat, d_cfg_key, d_cfg_q, d_cfg_batch;
  std::vector<int64_t> res_total;  // [n_hw] or empty
  // finite-alpha objective (llama_set_alpha)
  bool has_alpha = false;
  uint32_t alpha_num = 0, alpha_den = 1;
  int32_t alpha_steps = 0, alpha_msteps = 0;
  DevBuf d_a_lat, d_a_ps, d_m_lat, d_m_pf, d_m_si, d_a_val;
  DevBuf d_a_smp, d_a_soff;
  DevBuf d_a_fk, d_a_ik, d_aq_T, d_aq_pf, d_aq_si, d_aq_cnt, d_m_cnt;  // finite alpha: per-configuration keys; per-call merged order
  int32_t alpha_max_op = 0;
  DevBuf d_aff_scratch;  // Eq. 3 sort keys, indices and sort temporary storage
  DevBuf d_batch_scratch;  // safe delayed batching: count, then the queue of invocations left to scan
  DevBuf d_qacc;  // Eq. 2 partial sums, QUEUE_PARTS x MAX_HW x 2 x 64 bits
  DevBuf d_sim_a, d_sim_b, d_sim_row_op;  // simulator: content coefficients per (op, backend) and op, op of each row
  double sim_sigma = 0.0;
  bool has_sim = false;
  // feedback (llama_feedback): static arrays of the device rebuild, zeroed
  // accumulators, and whether the host copy of the latencies is behind
  bool fb_ready = false, host_stale = false;
  DevBuf d_fb_ksrc, d_fb_tab_src, d_fb_ref_k, d_fb_count, d_fb_sum, d_fb_dirty;
  DevBuf d_err;
  llama::Surrogate surr;
  DevBuf d_cnt, d_start, d_cursor, d_perm, d_hist;  // bucketed full scan
  int64_t perm_cap = 0;
  int32_t decide_sched = 0;  // schedule chosen by llama_autotune (llama::DecideSchedule)
  int32_t full_cross_num = 1, full_cross_den = 1;  // full-scan schedule crossover (llama_autotune_full)
  int32_t n_cu = 256;        // compute units of the device

  DevTables tables() const {
    DevTables t{};
    t.n_ops = n_ops;
    t.n_hw = n_hw;
    t.n_pipelines = n_pipelines;
    t.hs = llama::header_stride(n_hw);
    t.n_front = n_cfg;  // stride of the capacity layout
    t.decide_sched = decide_sched;
    t.full_cross_num = full_cross_num;
    t.full_cross_den = full_cross_den;
    t.n_cu = n_cu;
    // relaxation stage: the largest pipeline, within 1024 ops / 3072 edges
    t.relax_ops = max_pipe_ops < 1024 ? max_pipe_ops : 1024;
    t.relax_edges = max_pipe_edges < 3072 ? max_pipe_edges : 3072;
    t.relax_lvls = max_depth < 1024 ? max_depth : 1024;
    t.max_pipe_ops = max_pipe_ops;
    t.pipe_off = d_pipe_off.as<int32_t>();
    t.pipe_desc = d_pipe_desc.as<int4>();
    t.lvl_bnd = d_lvl_bnd.as<int32_t>();
    t.lvl_ops = d_lvl_ops.as<int32_t>();
    t.lvl_edge = d_lvl_edge.as<uint32_t>();
    t.lvl_edge_q = d_lvl_edge_q.as<uint32_t>();
    t.lvl_ebnd = d_lvl_ebnd.as<int32_t>();
    t.succ_off = d_succ_off.as<int32_t>();
    t.succ_ids = d_succ_ids.as<int32_t>();
    t.succ_q = d_succ_q.as<uint32_t>();
    t.ref = d_ref.as<int32_t>();
    t.W = d_W.as<int64_t>();
    t.hdr = d_hdr.as<int32_t>();
    t.front_L = d_front_L.as<uint2>();
    t.mst = d_mst.as<uint2>();
    t.mst_n = d_mst_n.as<int32_t>();
    t.rec = d_rec[rec_cur].as<uint4>();
    t.rec_tail = d_rec_tail[rec_cur].as<uint4>();
    t.rec_tail2 = d_rec_tail2[rec_cur].as<uint4>();
    t.rec_tail_q = d_rec_tail_q.as<uint4>();
    t.rec_tail2_q = d_rec_tail2_q.as<uint4>();
    t.ovf = d_ovf[rec_cur].as<uint2>();
    t.rec_q = d_rec_q.as<uint4>();
    t.ovf_q = d_ovf_q.as<uint2>();
    t.cfg_off = d_cfg_off.as<int32_t>();
    t.cfg_hw = d_cfg_hw.as<int32_t>();
    t.cfg_lat = d_cfg_lat.as<int32_t>();
    t.cfg_key = d_cfg_key.as<uint32_t>();
    t.cfg_q = d_cfg_q.as<uint4>();
    t.cfg_batch = d_cfg_batch.as<int32_t>();
    t.a_lat = d_a_lat.as<int32_t>();
    t.a_ps = d_a_ps.as<uint2>();
    t.a_steps = alpha_steps;
    t.m_lat = d_m_lat.as<int32_t>();
    t.m_pf = d_m_pf.as<uint32_t>();
    t.m_si = d_m_si.as<uint32_t>();
    t.m_steps = alpha_msteps;
    t.a_smp = d_a_smp.as<int32_t>();
    t.a_soff = d_a_soff.as<int32_t>();
    t.a_val = d_a_val.as<double>();
    t.a_fk = d_a_fk.as<uint32_t>();
    t.a_ik = d_a_ik.as<uint32_t>();
    t.aq_T = d_aq_T.as<uint32_t>();
    t.aq_pf = d_aq_pf.as<uint32_t>();
    t.aq_si = d_aq_si.as<uint32_t>();
    t.aq_cnt = d_aq_cnt.as<uint16_t>();
    t.m_cnt = d_m_cnt.as<uint16_t>();
    t.alpha_max_op = alpha_max_op;
    t.seg_off = d_seg_off.as<int32_t>();
    t.tab = d_tab.as<uint2>();
    t.err = d_err.as<uint32_t>();
    return t;
  }

  // Tables with the record set `set` (the relaxation's output).
  DevTables tables_for(int set) const {
    DevTables t = tables();
    t.rec = d_rec[set].as<uint4>();
    t.rec_tail = d_rec_tail[set].as<uint4>();
    t.rec_tail2 = d_rec_tail2[set].as<uint4>();
    t.ovf = d_ovf[set].as<uint2>();
    return t;
  }

  int64_t device_bytes() const {
    const DevBuf* all[] = {&d_pipe_off, &d_pipe_desc, &d_lvl_edge, &d_lvl_edge_q, &d_lvl_ebnd, &d_lvl_bnd, &d_lvl_ops, &d_succ_off,
                           &d_succ_ids, &d_succ_q, &d_ref, &d_W, &d_hdr, &d_front_L,
                           &d_rec[0], &d_rec_tail[0], &d_rec_tail2[0], &d_ovf[0], &d_rec[1], &d_rec_tail[1], &d_rec_tail2[1], &d_ovf[1], &d_rec_q, &d_rec_tail_q, &d_rec_tail2_q, &d_ovf_q, &d_seg_off, &d_tab, &d_err,
                           &d_cnt, &d_start, &d_cursor, &d_perm, &d_hist, &d_mst,
                           &d_mst_n, &d_cfg_off, &d_cfg_hw, &d_cfg_lat, &d_cfg_key, &d_cfg_q, &d_cfg_batch, &d_a_lat, &d_a_ps, &d_m_lat, &d_m_pf, &d_m_si, &d_a_val, &d_a_smp, &d_a_soff, &d_a_fk, &d_a_ik, &d_aq_T, &d_aq_pf, &d_aq_si, &d_aq_cnt, &d_m_cnt, &d_aff_scratch, &d_batch_scratch, &d_qacc, &d_fb_ksrc, &d_fb_tab_src, &d_fb_ref_k, &d_fb_count, &d_fb_sum, &d_fb_dirty, &d_sim_a, &d_sim_b, &d_sim_row_op};
    int64_t s = 0;
    for (auto* b : all) s += (int64_t)b->bytes;
    return s;
  }
};


namespace llama {
// helpers implemented in llama_host.cpp
int fail(llama_ctx* c, int code, const char* fmt, ...);
int hip_fail(llama_ctx* c, hipError_t e, const char* what);
int upload(llama_ctx* c, DevBuf& buf, const void* src, size_t bytes, const char* what);
int enter(llama_ctx* c);
int sync_ctx(llama_ctx* c, const char* what);
// finite-alpha tables (next_host.cpp); called by llama_set_alpha and after latency updates
int build_alpha_tables(llama_ctx* c);
}  // namespace llama
// Grows the context's full-scan scratch (permutation and histograms) to n
// invocations; refused while `stream` is being captured.
int reserve_perm(llama_ctx* c, int64_t n, hipStream_t stream);
namespace llama {
// feedback (feedback_host.cpp): refresh the host copies of the latencies
// after device-side feedback
int pull_profiles(llama_ctx* c);
// Relaxation into the record set not written last (then decisions use it).
hipError_t relax_next(llama_ctx* c, hipStream_t s, int modes = 3);
// noalloc.hip: resolve the static scratch array's address on `device` (current)
hipError_t noalloc_attach(int device);
// Whether the current record set holds the records of slack mode `mode`.
inline bool records_current(const llama_ctx* c, int mode) { return (c->rec_modes[c->rec_cur] >> mode) & 1; }
// noalloc.hip: resolve the static scratch array's address on `device` (current)
hipError_t noalloc_attach(int device);
}  // namespace llama
