// Internal interface between the host side of libllama (llama_host.cpp) and
// its HIP kernels (llama_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace llama {

constexpr uint32_t KEY_NONE = 0xFFFFFFFFu;   // "no feasible configuration"
constexpr uint32_t THR_NEVER = 0xFFFFFFFFu;  // remaining-time threshold never met
constexpr int MAX_HW = 8;
constexpr uint32_t DEVERR_QUEUE_ENTRY = 2u;  // device error bit: queued entry out of range

// Per-op decision record (112 bytes in three arrays).  The op's frontier
// over all backends in remaining-time space: entries {T, k} such that
// configuration k (local index) is feasible for an invocation iff
// slo - elapsed >= T, with T strictly increasing and the configuration's cost
// key strictly decreasing along the frontier.  The record keeps the REC_SLOTS
// entries with the largest T (the cheapest configurations, which most
// invocations can afford), in descending T order, thresholds stored as
// U = T - 1 (feasible iff U < slo - elapsed; U = 2^31 - 1 for an unused slot
// never is):
//   hot, 16 bytes (one uint4 per op):
//     word 0        fastest configuration (low 16 bits) | rec_floor_code of
//                   the smallest U of the whole frontier (high 16 bits)
//     words 1, 2    U of slots 0 and 1 (slot 0 = largest T)
//     word 3        k of slots 0 and 1 (16-bit halves)
//   tail, 32 bytes (two uint4 per op, one 32-byte sector):
//     word 4        entry count n (low 16 bits) | k of slot 2
//     words 5, 6    k of slots (3, 4) and (5, 6)
//     words 7..11   U of slots 2..6
//   second tail, 64 bytes (four uint4 per op), written and read only for ops
//   with more than REC_SLOTS_TAIL entries:
//     words 12..21  U of slots 7..16
//     words 22..26  k of slots (7, 8) ... (15, 16); word 27 unused
// The hot words alone decide every invocation that can afford one of the two
// cheapest entries, and every invocation that can afford none (slo - elapsed
// at or below the rounded-down smallest U: the fastest configuration, flag
// 0).  The entries past the record (the n - REC_SLOTS smallest T), ascending
// in T, are in the overflow array at [hdr offset of the op, + n - REC_SLOTS);
// the decision reads them only when no slot is feasible.
constexpr int ALPHA_BLOCK = 16;  // latencies per sampled block of the finite-alpha runs
constexpr int REC_WORDS = 28;
constexpr int REC_SLOTS = 17;
constexpr int REC_SLOTS_TAIL = 7;   // slots in the hot words and the first tail
constexpr int REC_TAIL_VECS = 2;    // uint4 per record in the tail array
constexpr int REC_TAIL2_VECS = 4;   // uint4 per record in the second-tail array
constexpr int REC_N_WORD = 4;       // word holding the entry count (low half)
__host__ __device__ inline constexpr int rec_u_word(int slot) { return slot < 2 ? 1 + slot : slot + 5; }
__host__ __device__ inline constexpr int rec_k_word(int slot) {
  return slot < 2 ? 3 : slot < REC_SLOTS_TAIL ? 4 + (slot - 1) / 2 : 22 + (slot - REC_SLOTS_TAIL) / 2;
}
__host__ __device__ inline constexpr int rec_k_shift(int slot) {
  return slot < 2 ? 16 * (slot & 1) : 16 * ((slot + 1) & 1);
}
// Address of word w of record r (r = mode * n_ops + op) in the three arrays.
__host__ __device__ inline uint32_t* rec_word(uint4* hot, uint4* tail, uint4* tail2, int64_t r, int w) {
  return w < 4 ? reinterpret_cast<uint32_t*>(hot + r) + w
         : w < 12 ? reinterpret_cast<uint32_t*>(tail + r * REC_TAIL_VECS) + (w - 4)
                  : reinterpret_cast<uint32_t*>(tail2 + r * REC_TAIL2_VECS) + (w - 12);
}
// 16-bit code of a stored threshold, rounded down: for u >= 0, an 11-bit
// mantissa m and a shift e with m << e <= u < (m + 1) << e; 0xFFFF (value
// INT32_MIN) for u < 0.  rec_code_value(rec_floor_code(u)) <= u for every u,
// so "slo - elapsed <= value" proves that no entry is feasible.
__host__ __device__ inline uint32_t rec_floor_code(int32_t u) {
  if (u < 0) return 0xFFFFu;
  const uint32_t x = (uint32_t)u;
  const int bits = 32 - __builtin_clz(x | 1u);
  const int e = bits > 11 ? bits - 11 : 0;
  return ((uint32_t)e << 11) | (x >> e);
}
__host__ __device__ inline int32_t rec_code_value(uint32_t c) {
  return c == 0xFFFFu ? INT32_MIN : (int32_t)((c & 0x7FFu) << (c >> 11));
}

// Schedules of the indexed decision (chosen by llama_autotune): 1, 2 or 4
// invocations per thread, LDS-staged hot records, and the direct schedules
// with non-temporal loads of the invocation stream.
enum DecideSchedule {
  SCHED_DIRECT1 = 0, SCHED_DIRECT2 = 1, SCHED_DIRECT4 = 2, SCHED_LDS = 3,
  SCHED_DIRECT1_NT = 4, SCHED_DIRECT2_NT = 5, SCHED_DIRECT4_NT = 6
};
constexpr int LDS_REC_MAX_OPS = 9216;  // 16 bytes per op staged in LDS (144 KB)

// Stride (int32 words) of the per-op header: frontier offsets for each
// backend (n_hw + 1 entries), then the fastest configuration, padded to a
// multiple of 4 words so the header can be read with 16-byte loads.
inline constexpr int header_stride(int n_hw) { return (n_hw + 2 + 3) & ~3; }

// Device-resident tables of one context.  All pointers are device memory
// owned by the context.
struct DevTables {
  int32_t n_ops;
  int32_t n_hw;
  int32_t n_pipelines;
  int32_t hs;              // header_stride(n_hw)
  int64_t n_front;         // capacity of the frontier and overflow arrays (n_cfg)
  int32_t decide_sched;    // DecideSchedule of the indexed decision
  int32_t full_cross_num;  // full scan: lanes = invocations when its cost x den <= the other's x num
  int32_t full_cross_den;
  int32_t n_cu;            // compute units of the device
  // LDS capacities of the relaxation (ops, edges, levels of one pipeline);
  // larger pipelines are relaxed in global memory
  int32_t relax_ops, relax_edges, relax_lvls;
  int32_t max_pipe_ops;      // ops of the largest pipeline

  // DAG
  const int32_t* pipe_off;   // [P+1] op range of each pipeline
  const int4* pipe_desc;     // [2*P] {first op, ops, first edge, edges}, {first level in lvl_bnd, levels, 0, 0}
  const int32_t* lvl_bnd;    // [n_levels+1] start of each level in lvl_ops
  const int32_t* lvl_ops;    // [n_ops] ops ordered by pipeline, then height (outputs first)
  const int32_t* succ_off;   // [n_ops+1]
  const int32_t* succ_ids;   // [n_edges]
  const uint32_t* succ_q;    // [n_edges] Q16 branch probability
  const uint32_t* lvl_edge;  // [n_edges] per pipeline, by source height: src | dst << 16 (pipeline-local)
  const uint32_t* lvl_edge_q;  // [n_edges] Q16 branch probability of lvl_edge
  const int32_t* lvl_ebnd;   // [n_levels+1] first lvl_edge of each level

  // profiles
  const int32_t* ref;        // [n_ops] reference-configuration latency
  int64_t* W;                // [2*n_ops] remaining worst-path latency: PAPER rows, then PROB rows
  const int32_t* hdr;        // [n_ops*hs] frontier offsets per backend + fastest (local index)
  const uint2* front_L;      // [n_front] {latency, key}: per (op, backend), latency ascending, key strictly descending
  const uint2* mst;          // [n_cfg] {L, key}, per op ascending in L from cfg_off[v]
  const int32_t* mst_n;      // [n_ops] entries of each op's merged frontier
  uint4* rec;                // [2*n_ops] record words 0..3, PAPER then PROB, queue = 0
  uint4* rec_tail;           // [2*n_ops*REC_TAIL_VECS] record tails
  uint4* rec_tail2;          // [2*n_ops*REC_TAIL2_VECS] record second tails
  uint2* ovf;                // [2*n_front] full frontiers {T, key} ascending, PAPER then PROB
  uint4* rec_q;              // [n_ops] records for a per-call queueing-time vector
  uint4* rec_tail_q;         // [n_ops*REC_TAIL_VECS]
  uint4* rec_tail2_q;        // [n_ops*REC_TAIL2_VECS]
  uint2* ovf_q;              // [n_front]
  const int32_t* cfg_off;    // [n_ops+1] caller-order configuration rows of each op
  const int32_t* cfg_hw;     // [n_cfg] backend, caller order
  const int32_t* cfg_lat;    // [n_cfg] profiled latency, caller order
  const uint32_t* cfg_key;   // [n_cfg] rank << 16 | k, caller order
  const uint4* cfg_q;        // [n_cfg] {L, R, hw, 0} caller order (with resource limits only)
  const int32_t* cfg_batch;  // [n_cfg] batch size, caller order
  // finite-alpha objective, per (op, backend) segment of seg_off, sorted by latency
  const int32_t* a_lat;      // [n_cfg] latency
  // [n_cfg + n_ops*n_hw] per segment of len entries, len + 1 pairs {min
  // feasible key over its first j entries, min infeasible key over entries j..}
  // (KEY_NONE for none), the pair of global entry index x at x + segment index
  const uint2* a_ps;
  int32_t a_steps;           // binary-search steps covering the longest segment
  // the same per op over all backends (cfg_off segments), for Q = 0
  const int32_t* m_lat;
  const uint32_t* m_pf;
  const uint32_t* m_si;
  int32_t m_steps;
  // samples of the (op, backend) runs of a_lat for two-level counts: the last
  // latency of every block of ALPHA_BLOCK entries, padded with INT32_MAX to a
  // multiple of four samples; an op's runs start at a_soff[v], one after the other
  const int32_t* a_smp;
  const int32_t* a_soff;     // [n_ops + 1]
  const double* a_val;       // [2 n_cfg] objective value of each rank, per op from 2 cfg_off[v]
  const int32_t* seg_off;    // [n_ops*n_hw+1] backend segments of the full table
  // finite alpha, per configuration in the a_lat order: its feasible and
  // infeasible keys (rank << 16 | local index)
  const uint32_t* a_fk;
  const uint32_t* a_ik;
  // finite alpha with queueing times, rebuilt per call: each op's
  // configurations merged over its backends by T + Q[backend] (T the
  // remaining-time threshold, 2^31 = never), with prefix minima of feasible
  // keys and suffix minima of infeasible keys in that order
  uint32_t* aq_T;
  uint32_t* aq_pf;
  uint32_t* aq_si;
  uint16_t* aq_cnt;           // [n_cfg * n_hw] per merged position p and backend h: entries of h before p
  const uint16_t* m_cnt;      // [n_cfg * n_hw] the same for the merged latency order (m_lat)
  int32_t alpha_max_op;      // most configurations of one op (finite-alpha tables)
  const uint2* tab;          // [n_cfg] {latency, key}, grouped by (op, backend), caller order inside
  uint32_t* err;             // device error word
};

// Per-call invocation batch (device pointers owned by the caller).
struct Batch {
  int64_t n;
  const int32_t* op;
  const int32_t* elapsed;
  const int32_t* slo;
  const int64_t* queue;      // [n_hw] or nullptr
  const int32_t* target;     // [n*n_hw] (select only)
  int32_t* target_out;       // [n*n_hw] (targets only)
  int32_t* cfg;
  uint8_t* flag;             // may be nullptr
  int32_t mode;              // 0 = PAPER, 1 = PROB
};

// modes: bit m set = rebuild the decision records of slack mode m (W is
// always relaxed for both modes).
hipError_t launch_relax(const DevTables& t, int modes, hipStream_t s);
// Build records for modes [mode0, mode0 + n_modes) into rec/rec_tail/
// rec_tail2/ovf (consecutive per-mode blocks of n_ops, 3*n_ops, 4*n_ops uint4
// and n_front uint2).
hipError_t launch_records(const DevTables& t, int mode0, int n_modes, const int64_t* queue, uint4* rec,
                          uint4* rec_tail, uint4* rec_tail2, uint2* ovf, hipStream_t s);
hipError_t launch_targets(const DevTables& t, const Batch& b, hipStream_t s);
hipError_t launch_select_indexed(const DevTables& t, const Batch& b, hipStream_t s);
hipError_t launch_decide_indexed(const DevTables& t, const Batch& b, hipStream_t s);
// Scratch of the bucketed full scan (device memory owned by the context).
struct FullScratch {
  int32_t* cnt;     // [n_ops + 1]
  int32_t* start;   // [n_ops + 1]
  int32_t* cursor;  // [n_ops]
  int32_t* perm;    // [n_inv]
  int32_t* hist;    // [full_scan_hist_words(n_inv, n_ops)]
};
// Words of per-chunk histogram scratch the full scan needs for n_inv invocations.
int64_t full_scan_hist_words(int64_t n_inv, int32_t n_ops);
hipError_t launch_decide_full(const DevTables& t, const Batch& b, const FullScratch& w, hipStream_t s);
hipError_t launch_decide_wave(const DevTables& t, const Batch& b, hipStream_t s);
// Eq. 2: per-workgroup 128-bit partial sums of L*R per backend (at most
// QUEUE_PARTS workgroups, scratch of QUEUE_PARTS x MAX_HW x 16 bytes), then
// their total divided by R_total.
constexpr int QUEUE_PARTS = 1024;
struct ResTotals {
  int64_t r[MAX_HW];
};
hipError_t launch_queue_time(const DevTables& t, int64_t n, const int32_t* q_op, const int32_t* q_cfg,
                             unsigned long long* part, const ResTotals& rt, int64_t* out, hipStream_t s);
// With queueing times and scratch w (FullScratch of b.n invocations) the
// invocations are first grouped by op when a counting sort applies
// (decide_alpha_ops_kernel); otherwise, or with w null, one thread per
// invocation.
hipError_t launch_decide_alpha(const DevTables& t, const Batch& b, const FullScratch* w, hipStream_t s);
// Eq. 3: affinities [n x n_hw] and, if order != nullptr, per backend the
// invocations by decreasing affinity (stable), using scratch of
// n * (8 n_hw + 8 + 4) bytes plus the sort's temporary storage.  With w
// (FullScratch of b.n invocations) the invocations are first grouped by op
// when a counting sort applies (affinity_ops_kernel); otherwise one thread
// per invocation with a search per backend.
hipError_t launch_affinity(const DevTables& t, const Batch& b, double* aff, int32_t* order, void* scratch,
                           size_t scratch_bytes, const FullScratch* w, hipStream_t s);
// Safe delayed batching: per op, invocations available now, expected from
// upstream, and the estimated wait for them; cfg CFG_WAIT means wait.
constexpr int CFG_WAIT = -2;
struct BatchingArgs {
  const int32_t* available;
  const int32_t* upstream;
  const int32_t* wait_us;
  uint2* queue;      // scratch: BATCH_QUEUES sub-queues of {invocation, x* | meets << 16} left
                     // for the batch-limited scan, each of batch_queue_capacity(n) entries
  uint32_t* count;   // scratch: entries of sub-queue j at count[32 * j] (one 128-byte line each)
  // scratch of the grouping by op (batch_group_words): per-op counts, starts
  // and cursors, the slots by op, and the counting sort's histograms
  int32_t* op_cnt;
  int32_t* op_start;
  int32_t* op_cursor;
  int32_t* perm;
  int32_t* hist;
};
// The commit kernel's workgroup g appends to sub-queue g mod BATCH_QUEUES, so
// that no single counter takes every workgroup's atomic.
constexpr int BATCH_QUEUES = 64;
constexpr int BATCH_BLOCK = 256;
inline int64_t batch_queue_capacity(int64_t n) {
  const int64_t groups = (n + BATCH_BLOCK - 1) / BATCH_BLOCK;
  return ((groups + BATCH_QUEUES - 1) / BATCH_QUEUES) * BATCH_BLOCK;
}
int64_t full_scan_hist_words(int64_t n_inv, int32_t n_ops);
// Words of the grouping scratch, each part on a 64-word boundary.
inline int64_t batch_words64(int64_t w) { return (w + 63) & ~(int64_t)63; }
inline int64_t batch_group_words(int64_t n, int32_t n_ops) {
  const int64_t slots = (int64_t)BATCH_QUEUES * batch_queue_capacity(n);
  return 3 * batch_words64((int64_t)n_ops + 1) + batch_words64(slots) + batch_words64(full_scan_hist_words(slots, n_ops));
}
inline size_t batch_scratch_bytes(int64_t n, int32_t n_ops) {
  return sizeof(uint32_t) * 32 * BATCH_QUEUES + sizeof(uint2) * (size_t)BATCH_QUEUES * (size_t)batch_queue_capacity(n) +
         sizeof(int32_t) * (size_t)batch_group_words(n, n_ops);
}
hipError_t launch_decide_batching(const DevTables& t, const Batch& b, const BatchingArgs& a, hipStream_t s);
// Finite-alpha Eq. 1 with queueing times through the per-call merged order
// (alpha_kernels.hip); for tables with at most ALPHA_MERGE_MAX configurations
// per op.
constexpr int ALPHA_MERGE_MAX = 4096;
hipError_t launch_decide_alpha_queue(const DevTables& t, const Batch& b, hipStream_t s);
// Eq. 3 affinity through a merged order (one search, then each backend's
// position from the per-backend counts): with queueing times the per-call
// order, without them the static latency order.
hipError_t launch_affinity_queue(const DevTables& t, const Batch& b, double* aff, int32_t* order, void* scratch,
                                 size_t scratch_bytes, hipStream_t s);
// Stable LSD radix sort of (uint64 key, int32 value) pairs (sort_kernels.hip).
hipError_t sort_pairs_bytes(int n, size_t* bytes);
hipError_t sort_pairs(void* tmp, size_t tmp_bytes, const uint64_t* kin, uint64_t* kout, const int32_t* vin,
                      int32_t* vout, int n, hipStream_t s);

// Feedback: smoothing of the profiled latencies from observations, then the
// device rebuild of every latency-derived table (reference latencies,
// fastest configurations, per-backend and merged frontiers, the full table).
constexpr uint32_t DEVERR_OBSERVATION = 4u;  // device error bit: observation out of range
struct FeedbackArgs {
  int32_t* lat;              // [n_cfg] profiled latency, caller order (updated)
  uint32_t* count;           // [n_cfg] observations per configuration (zero between calls)
  unsigned long long* sum;   // [n_cfg] their sum (zero between calls)
  uint32_t* dirty;           // [n_ops] an observation touched the op (zero between calls)
  const int32_t* ksrc;       // [n_cfg] the op's configurations in ascending key order (caller rows)
  const int32_t* ref_k;      // [n_ops] reference configuration (local index)
  const int32_t* tab_src;    // [n_cfg] caller row of each position of tab
  int32_t* ref;              // [n_ops]
  int32_t* hdr;              // [n_ops * hs]
  uint2* front;              // [n_cfg] per-backend frontiers (capacity layout)
  uint2* mst;                // [n_cfg] merged frontiers (capacity layout)
  int32_t* mst_n;            // [n_ops]
  uint2* tab;                // [n_cfg]
  uint4* cfg_q;              // [n_cfg] or nullptr
};
hipError_t launch_feedback(const DevTables& t, const FeedbackArgs& f, int64_t n, const int32_t* obs_op,
                           const int32_t* obs_cfg, const int32_t* obs_lat, uint32_t beta_q16, hipStream_t s);
hipError_t launch_select_rows(const DevTables& t, const Batch& b, const int32_t* lat, int64_t stride,
                              hipStream_t s);

// ---------------------------------------------------------------------------
// Learned surrogate
// ---------------------------------------------------------------------------
constexpr int SURR_EMB = 16, SURR_FEAT = 16, SURR_IN = 32, SURR_HID = 256, SURR_OUT = 2;

// Device buffers of the surrogate (BF16 arrays as void*).  Parameters are one
// FP32 vector laid out E [n_rows][16], W1 [256][32], b1 [256], W2 [256][256],
// b2 [256], W3 [2][256], b3 [2]; o* are the offsets of each part.
struct SurrogateBufs {
  int64_t n_params, nE, oW1, ob1, oW2, ob2, oW3, ob3;
  float *master, *adam_m, *adam_v, *grad;
  const float *b1, *b2, *b3;
  void *E16, *W1_16, *W2_16, *W2p16, *W3_16;
  void *W1T16, *W2T16;       // transposed shadows: W1T[k][o], W2T[k][o]
  unsigned long long* dE;    // [nE] embedding-gradient accumulator (fixed point, 2^-40), zero between steps
  float* part;               // [TRAIN_MAX_CHUNKS][n_params - nE] per-chunk partial gradients
  // forward workspace, B rows
  void *X16, *h1, *h2;
  float *z1, *z2, *out;
};

struct LearnedArgs {
  const void* feat;          // [n_inv][16] BF16 content features
  const void *E16, *W1_16, *W2p16, *W3_16;
  const float *b1, *b2, *b3;
  float spread_max;          // fall back to the profile when q - mu is outside [0, spread_max]
  int32_t* lat_out;          // optional [n_inv][lat_stride] predicted p95 latency per row
  int64_t lat_stride;
};

hipError_t launch_gemm_bf16(int M, int N, int K, const void* a, int64_t sam, int64_t sak, const void* b,
                            int64_t sbk, int64_t sbn, float* c, int64_t ldc, const float* bias, bool accumulate,
                            hipStream_t s);
hipError_t launch_surrogate_forward(const SurrogateBufs& w, int64_t B, const int32_t* rows, const void* feat,
                                    hipStream_t s);

// Fused training step.  launch_train_chunks: one workgroup per TRAIN_ROWS
// rows runs the forward and backward passes of its rows with every
// activation in LDS and registers, writes its partial gradients of W1, b1,
// W2, b2, W3, b3 to part[chunk] (all of them) and adds its embedding
// gradients to dE atomically; at most TRAIN_MAX_CHUNKS chunks a launch.
// launch_train_reduce: a thread per parameter sums the chunks' partials in
// chunk order (dE for the embedding, which it then clears), adds them to grad
// (or overwrites it when `first`), and with `update` applies AdamW and writes
// the BF16 shadows of the new value.
constexpr int TRAIN_ROWS = 64;
constexpr int TRAIN_MAX_CHUNKS = 256;
struct TrainArgs {
  int64_t n;                 // rows of this launch
  const int32_t* rows;       // [n] profile rows
  const void* feat;          // [n][16] BF16 features
  const float* y;            // [n] observed ln latency
  float inv_B;               // 1 / rows of the whole step
  float* loss_sum;           // optional: += the rows' loss
};
hipError_t launch_train_chunks(const SurrogateBufs& w, const TrainArgs& a, hipStream_t s);
hipError_t launch_train_reduce(const SurrogateBufs& w, int n_chunks, bool first, bool update, float lr, float wd,
                               int64_t step, hipStream_t s);
hipError_t launch_shadows(const SurrogateBufs& w, hipStream_t s);
hipError_t launch_decide_learned(const DevTables& t, const Batch& b, const LearnedArgs& a, hipStream_t s);

// Pipeline simulator (sim_kernels.hip): samples first .. first + n - 1.
struct SimArgs {
  int64_t n, first;
  uint64_t seed;
  int64_t n_rows;
  int32_t n_hw;
  const int32_t* row_op;   // [n_rows] op of each profile row
  const int32_t* cfg_hw;   // [n_rows]
  const int32_t* cfg_lat;  // [n_rows] profiled latency (us)
  const double* a_coef;    // [n_ops * n_hw] ln latency per ln(1 + objects)
  const double* b_coef;    // [n_ops] ln latency per ln(pixels / 720p pixels)
  double sigma;            // noise of ln latency
  int32_t* rows;           // [n] out
  void* feat;              // [n][16] BF16 out
  float* y;                // [n] out: observed ln latency
};
hipError_t launch_simulate(const SimArgs& a, hipStream_t s);

// Serving ring shared by the host and the persistent decision kernels: the
// request, feature, result and timestamp arrays and the control words are in
// pinned host memory mapped into the device's address space; the claim
// counters are in device memory.  Request seq sits in slot seq % cap.
struct ServeRing {
  const int4* req;              // [cap] {op, elapsed_us, slo_us, 0}
  const void* feat;             // [cap][16] BF16 content features (learned form) or nullptr
  unsigned long long* res;      // [cap] (seq + 1 mod 2^32) << 32 | (cfg + 1) | flag << 31
  unsigned long long* ts;       // [cap] device clock when the decision was written
  const long long* head;        // requests published by the host: seq < *head
  const int* stop;              // nonzero: the kernels finish their claims and exit
  const int* probe;             // clock probe number written by the host
  int* ack;                     // last probe answered, after *stamp
  unsigned long long* stamp;    // device clock when that probe was seen
  int* exited;                  // set by the last wavefront to exit
  unsigned long long* ctr;      // device memory: [0] next seq to claim, [1] claims, [2] largest claim,
                                // [3] wavefronts alive, [4] device clock of the latest claim
  int64_t cap;
  int32_t mode;                 // slack mode
  int32_t chunk;                // requests a wavefront claims at once (plain form, 1..64)
  uint64_t idle_ticks;          // device-clock ticks without work before a wavefront exits
  uint64_t life_ticks;          // device-clock ticks before a wavefront exits in any case
};
// Persistent plain decisions (records of r.mode, no queueing times) by
// `workgroups` workgroups of four wavefronts.
hipError_t launch_serve_plain(const DevTables& t, const ServeRing& r, int workgroups, hipStream_t s);
// Persistent learned decisions: one wavefront per invocation.
// prepare_serve_learned raises the kernel's LDS limit (once, before capture).
hipError_t prepare_serve_learned(const DevTables& t);
hipError_t launch_serve_learned(const DevTables& t, const ServeRing& r, const LearnedArgs& a, int workgroups,
                                hipStream_t s);
// Clock handshake for host/device time calibration: for round k < rounds the
// kernel waits (at most timeout_ticks) until *flag == k + 1, then writes its
// clock to stamp[k] and sets *ack = k + 1.
hipError_t launch_clock_probe(const int* flag, int* ack, unsigned long long* stamp, int rounds,
                              uint64_t timeout_ticks, hipStream_t s);

}  // namespace llama
