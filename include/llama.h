/*
 * llama.h -- C ABI of the MI355X (gfx950) decision engine for Llama
 * (Romero, Zhao, Yadwadkar, Kozyrakis, arXiv 2102.01887).
 *
 * For every pending operation invocation the library computes, on the GPU,
 *   (1) the invocation's latency target ("slack") for every backend, by
 *       splitting the remaining end-to-end time along the remaining DAG path
 *       weighted by reference-configuration latencies (Alg. 1, Sec. 4.1), and
 *   (2) the cheapest configuration of the operation whose latency is strictly
 *       below the slack of its own backend, by cost per item C/B, or the
 *       fastest configuration when none qualifies (Eq. 1, Sec. 4.2).  The
 *       fallback is a rule of this library, not a limit of Eq. 1: Eq. 1
 *       ranks a configuration that misses its slack by C/B plus a weighted
 *       penalty that never names a value for the weight alpha, and as alpha
 *       grows that ranking orders such configurations by L*R/(B*R_total), not
 *       by L.  When none meets its slack this library takes the smallest L,
 *       lowest index on ties; the finite-alpha objective is llama_decide_alpha.
 *
 * Units: latencies and times are int32 microseconds, costs int64 nano-dollars
 * per configuration run.  All arithmetic is integer, so results are exact.
 *
 * Conventions for every function:
 *   - return LLAMA_OK (0) or a negative status; no exception crosses the ABI;
 *     on failure llama_last_error() describes the first problem found and
 *     outputs are unspecified;
 *   - "host" pointers are read during the call only; the library copies what
 *     it keeps, so the caller may free them on return;
 *   - "device" pointers are caller-owned GPU memory (for example torch
 *     tensors) and are never retained after the work enqueued by the call;
 *   - `stream` is a hipStream_t (NULL = the default stream); decision calls
 *     only enqueue work and return; outputs are valid once the stream has
 *     synchronised; they may be captured into a hipGraph and allocate
 *     nothing, except the scratch growth (outside capture) described at
 *     llama_decide, llama_decide_alpha, llama_affinity and
 *     llama_decide_batching;
 *   - a context is not thread-safe: use one per thread or lock around it.
 */
#ifndef LLAMA_H
#define LLAMA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct llama_ctx llama_ctx;

enum llama_status {
    LLAMA_OK = 0,
    LLAMA_E_ARG = -1,    /* null pointer, negative count, bad enum, size mismatch */
    LLAMA_E_RANGE = -2,  /* a value outside the documented bounds below */
    LLAMA_E_CYCLE = -3,  /* the successor lists contain a cycle */
    LLAMA_E_STATE = -4,  /* call order, missing reference configuration */
    LLAMA_E_DEVICE = -5, /* HIP runtime error (text in llama_last_error) */
    LLAMA_E_NOMEM = -6   /* device or host allocation failed */
};

/* Path latency used by the slack (Alg. 1 RemainingPathLatency). */
enum llama_slack_mode {
    /* Sum of reference latencies from op (inclusive) to the output; slack is
     * the minimum over all paths through op (Alg. 1 as printed). */
    LLAMA_SLACK_PAPER = 0,
    /* Each downstream edge is discounted by its branch probability q/65536,
     * applied tail-first with a floor at every step; equals PAPER when every
     * q = 65536. */
    LLAMA_SLACK_PROB = 1
};

/* How llama_decide evaluates Eq. 1 (the result is identical in every mode). */
enum llama_scan_mode {
    LLAMA_SCAN_AUTO = 0,    /* library's choice (currently INDEXED) */
    /* Each op's cost/latency frontier over all backends, turned into
     * remaining-time thresholds (one 64-byte record per op). */
    LLAMA_SCAN_INDEXED = 1,
    /* Every configuration of the op: invocations are bucketed by op on the
     * GPU and one wavefront per op scans its table for its invocations, in
     the layout the schedule table picks (llama_autotune_full).  Uses
     * context scratch of 4 bytes per invocation, 8 with more than 12,288 ops
     * (see llama_reserve). */
    LLAMA_SCAN_FULL = 2,
    /* Every configuration, one wavefront per invocation, lanes over the
     * configurations, wavefront min reduction; no scratch. */
    LLAMA_SCAN_WAVE = 3
};

#define LLAMA_MAX_HW 8                 /* backends (hardware types) */
#define LLAMA_MAX_CFG_PER_OP 65535     /* configurations of one operation */
#define LLAMA_MAX_COST ((int64_t)1 << 40)
#define LLAMA_MAX_BATCH 65536
#define LLAMA_Q_ONE 65536              /* branch probability 1.0 in Q16 */
#define LLAMA_MAX_RES_TOTAL ((int64_t)1 << 40)  /* resource limit of a backend */
#define LLAMA_ALPHA_MAX_CFG_PER_OP 32767        /* finite-alpha objective */

/* Device error word bits (llama_stats.device_error). */
#define LLAMA_DEVERR_INVALID_INVOCATION 1u
#define LLAMA_DEVERR_INVALID_QUEUE_ENTRY 2u
#define LLAMA_DEVERR_INVALID_OBSERVATION 4u

/* Create a context bound to HIP device `device` (its ordinal). */
int llama_create(llama_ctx **out, int32_t device);

/* Release a context and every device buffer it owns; NULL is ignored.
 * Waits for the context's own work; the caller must have synchronised any
 * stream that still runs decision work against it. */
void llama_destroy(llama_ctx *ctx);

/* Text of the last failure on this context ("" after success).  The string
 * belongs to the context and is valid until its next call. */
const char *llama_last_error(const llama_ctx *ctx);

/*
 * Pipeline DAGs (Sec. 3.2 Application Interface and Pipeline-Decomposer;
 * Sec. 2 sequential, parallel and branching patterns).  All host pointers.
 *
 *   n_pipelines      >= 1
 *   pipe_op_offsets  [n_pipelines+1], pipeline p owns the global op ids
 *                    [off[p], off[p+1]); off[0] = 0, non-decreasing;
 *                    n_ops = off[n_pipelines] >= 1
 *   succ_offsets     [n_ops+1] CSR row offsets of successor lists
 *   succ_ids         [n_edges] successor op ids; every edge stays inside its
 *                    pipeline; no self-loops
 *   succ_prob_q16    [n_edges] branch probability * 65536 in [1, 65536];
 *                    NULL means 65536 (unconditional) for every edge
 *
 * Every op with no successor is an output operation, every op with no
 * predecessor an input operation; any number of either is accepted.
 * Errors: LLAMA_E_ARG, LLAMA_E_RANGE (ids, probabilities, pipeline bounds),
 * LLAMA_E_CYCLE.  Replaces any previous DAG and drops the profile tables
 * (llama_set_profiles must be called again).
 */
int llama_set_dag(llama_ctx *ctx, int32_t n_pipelines,
                  const int32_t *pipe_op_offsets, const int32_t *succ_offsets,
                  const int32_t *succ_ids, const uint32_t *succ_prob_q16);

/*
 * Configuration specifications of every operation (Sec. 3.2
 * Operation-Profiler: knob values, latency and resource use per
 * configuration; reference configuration).  All host pointers; row x of op v
 * lies in [cfg_offsets[v], cfg_offsets[v+1]) and its local (caller) index
 * k = x - cfg_offsets[v] is what llama_select / llama_decide return.
 *
 *   n_ops          must equal the DAG's op count (llama_set_dag first)
 *   n_hw           number of backends, 1..LLAMA_MAX_HW
 *   cfg_offsets    [n_ops+1]; 1..LLAMA_MAX_CFG_PER_OP configurations per op
 *   cfg_hw         [n_cfg] backend of the configuration, 0..n_hw-1
 *                  (0 is the CPU backend used by the reference rule)
 *   cfg_batch      [n_cfg] batch size B, 1..LLAMA_MAX_BATCH
 *   cfg_res        [n_cfg] resource size R (cores, MB, ...), >= 1
 *   cfg_lat_us     [n_cfg] profiled latency L, >= 1
 *   cfg_cost_nusd  [n_cfg] cost C of one run, 0..LLAMA_MAX_COST
 *   ref_cfg        [n_ops] local index of each op's reference configuration,
 *                  or NULL for the paper's rule: the hw-0 (CPU), batch-1
 *                  configuration with the smallest resource size, lowest
 *                  index on ties (LLAMA_E_STATE if an op has none)
 *   hw_res_total   [n_hw] resource limit per backend (R_total of Eq. 1 and
 *                  Eq. 2), 1..LLAMA_MAX_RES_TOTAL; may be NULL when neither
 *                  llama_queue_time nor the finite-alpha objective is used
 *
 * Also bounded: (ops in a pipeline) * (largest reference latency in it)
 * < 2^46, so every path latency and every intermediate product fits int64.
 * Builds the device tables and computes the remaining-path latencies for
 * both slack modes before returning (synchronously).
 */
int llama_set_profiles(llama_ctx *ctx, int32_t n_ops, int32_t n_hw,
                       const int32_t *cfg_offsets, const int32_t *cfg_hw,
                       const int32_t *cfg_batch, const int32_t *cfg_res,
                       const int32_t *cfg_lat_us, const int64_t *cfg_cost_nusd,
                       const int32_t *ref_cfg, const int64_t *hw_res_total);

/*
 * Recompute, on `stream`, the largest remaining reference-path latency W[v]
 * of every op for both slack modes (Alg. 1 RemainingPathLatency with the
 * minimum over paths, as a level-synchronous longest-path relaxation from the
 * outputs upward) and the per-configuration remaining-time thresholds that
 * llama_decide uses.  llama_set_profiles already does this; call it again
 * after changing reference latencies (llama_update_latencies).
 * The thresholds are double-buffered: each call writes the set the previous
 * call did not, and decision calls issued after it read the new set.  So a
 * relaxation may run on one stream while the decisions that follow the
 * previous relaxation run on another; the caller orders each decision after
 * its relaxation, and each relaxation after the decisions of the
 * relaxation before the previous one (which used the same set).
 */
int llama_relax(llama_ctx *ctx, void *stream);

/*
 * llama_relax for the slack modes in `modes` only (bit m = LLAMA_SLACK_*
 * value m: 1 = PAPER, 2 = PROB, 3 = both, the same as llama_relax).  W is
 * relaxed for both modes; the thresholds are rebuilt only for the modes
 * asked for, so a caller that decides in one mode halves the relaxation's
 * record writes.  Until the next relaxation, the record-reading calls
 * (llama_decide in the INDEXED/AUTO mode without a queue vector,
 * llama_decide_batching without one, llama_serve_open in the plain form)
 * return LLAMA_E_STATE for a mode left out; the other calls read W directly
 * and are unaffected.  LLAMA_E_ARG for a mask outside 1..3.
 */
int llama_relax_modes(llama_ctx *ctx, int32_t modes, void *stream);

/*
 * Replace the profiled latency of every configuration (for example after
 * feedback, Sec. 3.3 Manager) without changing the table's shape; host
 * pointer [n_cfg], same bounds as in llama_set_profiles.  Rebuilds the
 * frontier tables and runs llama_relax synchronously.
 */
int llama_update_latencies(llama_ctx *ctx, const int32_t *cfg_lat_us);

/*
 * Feedback (Sec. 3.3, Manager): update the profiled latencies from observed
 * ones by exponential smoothing, then rebuild every table derived from them
 * on the device and rerun the relaxation, all on `stream`.  Device pointers:
 *   d_obs_op    [n_obs] global op id of each completed invocation
 *   d_obs_cfg   [n_obs] the configuration it ran with (local index)
 *   d_obs_lat   [n_obs] its observed latency (us, >= 1)
 * beta_q16 in [0, 65536] is the smoothing factor times 65536.  The m
 * observations of one configuration in a call, with sum S, make one step
 * toward their mean: L' = L + floor(beta * (S - m L) / (65536 m)), clamped to
 * [1, 2^31 - 1].  Observations out of range are left out and set
 * LLAMA_DEVERR_INVALID_OBSERVATION.  Only the ops with an observation are
 * rebuilt.  Needs fewer than 2^15 ops per pipeline (LLAMA_E_RANGE
 * otherwise), so that any latencies keep path sums below 2^46.  The first call allocates 12 bytes
 * per configuration of scratch and copies static arrays (make it before
 * capturing a graph); calls on one context must not overlap.  Drops the
 * finite-alpha tables (call llama_set_alpha again).
 */
int llama_feedback(llama_ctx *ctx, int64_t n_obs, const int32_t *d_obs_op,
                   const int32_t *d_obs_cfg, const int32_t *d_obs_lat, uint32_t beta_q16,
                   void *stream);

/*
 * Alg. 1 for n_inv invocations (device pointers):
 *   d_inv_op      [n_inv] global op id of the invocation
 *   d_elapsed_us  [n_inv] time already spent by the invocation's pipeline run
 *   d_slo_us      [n_inv] the pipeline's end-to-end latency target
 *   d_queue_us    [n_hw] estimated queueing time per backend (Eq. 2), or NULL
 *                 for zero
 *   slack_mode    LLAMA_SLACK_PAPER or LLAMA_SLACK_PROB
 *   d_target_us   [n_inv * n_hw] output, row-major (invocation, backend):
 *                 R = clamp(slo - elapsed - queue[h], 0, 2^31-1) and
 *                 target = R == 0 ? 0 : floor(ref[v] * R / W[v])
 * An invocation with op outside [0, n_ops) or a negative elapsed or slo is
 * invalid: its targets are -1 and the device error word records it.
 */
int llama_targets(llama_ctx *ctx, int64_t n_inv, const int32_t *d_inv_op,
                  const int32_t *d_elapsed_us, const int32_t *d_slo_us,
                  const int64_t *d_queue_us, int32_t slack_mode,
                  int32_t *d_target_us, void *stream);

/*
 * Eq. 1 given targets (device pointers):
 *   d_target_us   [n_inv * n_hw] as written by llama_targets (any values)
 *   d_cfg         [n_inv] output: local index of the configuration with the
 *                 smallest C/B among those with L < target[hw], lowest index
 *                 on ties; if none, the smallest L, lowest index on ties;
 *                 -1 for an op outside [0, n_ops)
 *   d_flag        [n_inv] output: 1 = a configuration met its slack,
 *                 0 = fallback or invalid; may be NULL
 */
int llama_select(llama_ctx *ctx, int64_t n_inv, const int32_t *d_inv_op,
                 const int32_t *d_target_us, int32_t *d_cfg, uint8_t *d_flag,
                 void *stream);

/*
 * llama_targets followed by llama_select, fused, without materialising the
 * targets.  Same arguments and results; scan_mode picks the evaluation
 * strategy (every mode gives identical outputs).
 *
 * Context-owned device buffers used per call: with d_queue_us != NULL the
 * INDEXED mode rebuilds the op records for that queue vector, and the FULL
 * mode buckets invocations; two such calls on one context must therefore not
 * run concurrently on different streams.  The FULL mode needs scratch for
 * n_inv invocations: the library grows it on demand, except while `stream`
 * is being captured into a graph (then LLAMA_E_STATE; call llama_reserve
 * first).
 */
int llama_decide(llama_ctx *ctx, int64_t n_inv, const int32_t *d_inv_op,
                 const int32_t *d_elapsed_us, const int32_t *d_slo_us,
                 const int64_t *d_queue_us, int32_t slack_mode,
                 int32_t scan_mode, int32_t *d_cfg, uint8_t *d_flag,
                 void *stream);

/*
 * Eq. 1 given targets and a latency per (invocation, configuration) instead
 * of the profile's (for example measured or predicted latencies):
 *   d_target_us [n_inv * n_hw] as in llama_select;
 *   d_lat_us    [n_inv * lat_stride], configuration k of invocation i's op at
 *               [i * lat_stride + k] (caller order); an op with more than
 *               lat_stride configurations makes the invocation invalid (-1);
 * feasible iff lat < target[hw]; cheapest C/B (profile costs) among the
 * feasible, else the smallest latency; lowest index on ties.
 */
int llama_select_rows(llama_ctx *ctx, int64_t n_inv, const int32_t *d_inv_op,
                      const int32_t *d_target_us, const int32_t *d_lat_us,
                      int64_t lat_stride, int32_t *d_cfg, uint8_t *d_flag, void *stream);

/*
 * Eq. 2 (Sec. 4.3): estimated queueing time of every backend from the
 * invocations queued there (the speculative and commit queues together),
 *     Q[h] = floor( sum over queued i with hw(x_i) = h of L(x_i) * R(x_i)
 *                   / R_total(h) ),
 * x_i being the configuration already chosen for queued invocation i; the
 * products are summed exactly (128-bit) and divided once; a quotient above
 * 2^62 is reported as 2^62.  Device pointers:
 *   d_q_op        [n_queued] global op id of each queued invocation
 *   d_q_cfg       [n_queued] its configuration, local index within the op
 *   d_queue_out   [n_hw] int64 output, usable directly as the d_queue_us of
 *                 llama_targets / llama_decide / llama_decide_alpha
 * Entries with an op or configuration out of range are left out and set
 * LLAMA_DEVERR_INVALID_QUEUE_ENTRY in the device error word.  Needs
 * hw_res_total (LLAMA_E_STATE otherwise).  Uses 128 KB of context-owned
 * scratch for per-workgroup partial sums: calls on one context must not
 * overlap.
 */
int llama_queue_time(llama_ctx *ctx, int64_t n_queued, const int32_t *d_q_op,
                     const int32_t *d_q_cfg, int64_t *d_queue_out, void *stream);

/*
 * Eq. 1 with a finite weight alpha = alpha_num / alpha_den (Sec. 4.2): every
 * configuration x of the invocation's op is scored
 *     obj(x) = C/B                                    if L < slack_{hw(x)}
 *            = C/B + alpha * L * R / (B * R_total(hw(x)))   otherwise
 * and the smallest obj wins, lowest caller index on ties; flag 1 when the
 * chosen configuration meets its slack.  llama_set_alpha builds the tables:
 * for each op the exact dense ranks of its 2n possible objective values
 * (compared by 256-bit cross-multiplication) and, per (op, backend), the
 * configurations in latency order with prefix minima of the feasible keys
 * and suffix minima of the infeasible keys.  Needs hw_res_total; alpha_num
 * < 2^32, 1 <= alpha_den < 2^32; every op at most
 * LLAMA_ALPHA_MAX_CFG_PER_OP configurations (LLAMA_E_RANGE otherwise).
 * Synchronous.  llama_update_latencies rebuilds the tables; llama_set_profiles
 * drops them.
 */
int llama_set_alpha(llama_ctx *ctx, uint32_t alpha_num, uint32_t alpha_den);

/*
 * Alg. 1 targets (as llama_targets, with d_queue_us or zeros) and the
 * finite-alpha Eq. 1 choice, fused; device pointers as in llama_decide.
 * Invalid invocations get -1 / flag 0 and set the device error word.  With
 * d_queue_us, when no op has more than 4,096 configurations and the batch
 * has at least one invocation per eight configurations (8 n_inv >= n_cfg),
 * each call first merges every op's configurations by remaining-time
 * threshold plus its backend's queueing time into context-owned tables (12
 * bytes per configuration), so calls with queueing times that overlap on one
 * context must be ordered; otherwise the invocations are grouped by op (a
 * counting sort in the scratch that LLAMA_SCAN_FULL uses, grown on demand as
 * by llama_reserve, so such calls that overlap on one context must be
 * ordered too) and each op's backend lists are counted once per invocation;
 * while `stream` is being captured and that scratch is too small, each
 * invocation searches each backend's list instead.  Without d_queue_us, one
 * search per invocation in the op's list merged over its backends.  Every
 * path gives the same decisions.
 */
int llama_decide_alpha(llama_ctx *ctx, int64_t n_inv, const int32_t *d_inv_op,
                       const int32_t *d_elapsed_us, const int32_t *d_slo_us,
                       const int64_t *d_queue_us, int32_t slack_mode, int32_t *d_cfg,
                       uint8_t *d_flag, void *stream);

/*
 * Safe delayed batching (Sec. 4.4).  Per op (device pointers [n_ops]):
 *   d_available   invocations of the op ready now
 *   d_upstream    invocations of the op expected from upstream work already
 *                 running
 *   d_wait_us     the estimated time until they arrive
 * For each invocation (other arguments as in llama_decide):
 *   1. x* = the Eq. 1 choice over every configuration (fastest fallback);
 *   2. B(x*) <= available: commit x*;
 *   3. else, if x* meets its slack, available + upstream >= B(x*) and
 *      wait_us + L(x*) < the slack of x*'s backend: wait
 *      (d_cfg = LLAMA_CFG_WAIT, d_flag = 1);
 *   4. else commit the Eq. 1 choice among the configurations with
 *      B <= max(available, 1), or x* if none has.
 * d_flag is 1 when the committed configuration meets its slack.  Invalid
 * invocations get -1 / 0 and set the device error word.  The context keeps a
 * scratch queue of about 8 bytes per invocation (those that need the
 * batch-limited choice, grouped by op for that choice: about 8 bytes more per
 * invocation and 12 per op); it grows on demand but not while `stream` is
 * being captured (LLAMA_E_STATE: call once before capturing).  Calls that
 * overlap on one context share it and must be ordered.  n_inv above
 * 2^31 - 1 is LLAMA_E_RANGE.
 */
#define LLAMA_CFG_WAIT (-2)
int llama_decide_batching(llama_ctx *ctx, int64_t n_inv, const int32_t *d_inv_op,
                          const int32_t *d_elapsed_us, const int32_t *d_slo_us,
                          const int64_t *d_queue_us, int32_t slack_mode,
                          const int32_t *d_available, const int32_t *d_upstream,
                          const int32_t *d_wait_us, int32_t *d_cfg, uint8_t *d_flag, void *stream);

/*
 * Eq. 3 (Sec. 4.4, priority-based commit): the affinity of each invocation's
 * op to each backend h,
 *     affinity = min obj over the op's configurations not on h
 *                / min obj over its configurations on h,
 * obj being the finite-alpha Eq. 1 objective (llama_set_alpha first) with
 * every configuration judged against its own backend's Alg. 1 slack
 * (d_queue_us as in llama_decide).  Readings: no configuration on h -> 0;
 * none elsewhere -> +infinity; a zero minimum on h -> +infinity, or 1 when
 * the other minimum is zero as well.  Device pointers:
 *   d_affinity  [n_inv * n_hw] double output, row-major (invocation, backend);
 *               the objective values are rounded to double once per value,
 *               so the ratio is within 1e-15 relative of the exact one
 *   d_order     [n_hw * n_inv] int32 output or NULL: for each backend, the
 *               invocation indices by decreasing affinity, ties by index
 *               (the commit order)
 * With d_order the context keeps scratch of n_inv * (8 n_hw + 12) bytes plus
 * the sort's temporary storage; it grows on demand but not while `stream` is
 * being captured (LLAMA_E_STATE: call once before capturing).  Invalid
 * invocations get affinity 0 and set the device error word.  Unless the
 * per-call merge of llama_decide_alpha applies, the invocations are grouped
 * by op in the scratch that LLAMA_SCAN_FULL uses (grown on demand as by
 * llama_reserve; calls that overlap on one context must be ordered); while
 * `stream` is being captured and that scratch is too small, one search per
 * invocation instead.  Every path gives the same affinities.
 */
int llama_affinity(llama_ctx *ctx, int64_t n_inv, const int32_t *d_inv_op,
                   const int32_t *d_elapsed_us, const int32_t *d_slo_us,
                   const int64_t *d_queue_us, int32_t slack_mode, double *d_affinity,
                   int32_t *d_order, void *stream);

/*
 * Autotuner: time every schedule of the indexed decision kernel (0, 1, 2:
 * 1, 2 or 4 invocations per thread; 3: persistent workgroups with every op's
 * first 16 record bytes staged in LDS, offered when there are at most 9,216
 * ops; 4, 5, 6: as 0, 1, 2 with non-temporal loads of the invocations) on the
 * caller's batch (device pointers; d_cfg_scratch
 * [n_inv] receives decisions), check that all of them give identical
 * decisions (LLAMA_E_DEVICE otherwise), and keep the fastest for this
 * context.  *chosen receives its number (0..6) and *best_us its time per launch
 * (either may be NULL).  Synchronous.
 */
int llama_autotune(llama_ctx *ctx, int64_t n_inv, const int32_t *d_inv_op,
                   const int32_t *d_elapsed_us, const int32_t *d_slo_us, int32_t *d_cfg_scratch,
                   int32_t *chosen, float *best_us, void *stream);

/*
 * Pin the schedule of the indexed decision kernel (0..6, numbered as for
 * llama_autotune) instead of timing them, e.g. when the decision runs beside
 * other kernels and the schedule that is fastest alone is not.  Schedule 3
 * needs at most 9,216 ops (LLAMA_E_ARG otherwise, as for a number outside
 * 0..6).  Every schedule gives the same decisions.
 */
int llama_set_schedule(llama_ctx *ctx, int32_t schedule);

/*
 * Schedule table of the full scan (LLAMA_SCAN_FULL), per the per-operation
 * configuration space of Sec. 4.2: each op's bucket of k invocations is
 * evaluated against its c configurations either with lanes = invocations
 * (the table as wave-uniform operands) or with lanes = configurations
 * (groups of 16, 32 or 64 lanes and a group minimum), whichever has the
 * smaller instruction count under the crossover: lanes = invocations when
 * its count x cross_den <= the other's x cross_num (num 0: always
 * configurations; num 2^20: almost always invocations).
 * llama_autotune_full times seven crossovers on the caller's batch (device
 * pointers, d_cfg_scratch [n_inv]; scratch reserved as by llama_reserve),
 * checks that they decide alike and keeps the fastest, returning it (either
 * output may be NULL) and its time per call; synchronous.  The chosen pair
 * is the table a caller may store and restore with llama_set_full_schedule
 * (LLAMA_E_ARG outside 0 <= num <= 2^20, den >= 1).  Default 1/1.
 */
int llama_autotune_full(llama_ctx *ctx, int64_t n_inv, const int32_t *d_inv_op,
                        const int32_t *d_elapsed_us, const int32_t *d_slo_us, int32_t slack_mode,
                        int32_t *d_cfg_scratch, int32_t *cross_num, int32_t *cross_den,
                        float *best_us, void *stream);
int llama_set_full_schedule(llama_ctx *ctx, int32_t cross_num, int32_t cross_den);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * decisions as llama_decide with LLAMA_SCAN_FULL, bit for bit, with the
 * bucketing scratch (per-op counts, starts and cursors, the permutation of
 * invocations, per-chunk histograms) taken from one static device array of
 * LLAMA_NOALLOC_SCRATCH_BYTES per GPU instead of context buffers.  The call
 * allocates nothing; the array is set up when a context is first created on
 * a device and is held until the process ends.  Arguments, outputs and
 * device errors as in llama_decide.  A batch whose scratch
 * (llama_decide_full_noalloc_words(n_inv, n_ops) 4-byte words) exceeds the
 * limit is rejected with LLAMA_E_RANGE before anything is launched.  Every
 * call on one GPU shares the array (each call rewrites what it reads, and
 * clears its counts with a kernel), so calls that may overlap on one GPU,
 * from any context or stream, race and must be ordered by the caller.
 */
#define LLAMA_NOALLOC_SCRATCH_BYTES ((int64_t)32 << 20)
int llama_decide_full_noalloc(llama_ctx *ctx, int64_t n_inv, const int32_t *d_inv_op,
                              const int32_t *d_elapsed_us, const int32_t *d_slo_us,
                              const int64_t *d_queue_us, int32_t slack_mode,
                              int32_t *d_cfg, uint8_t *d_flag, void *stream);
/* Scratch words one llama_decide_full_noalloc call needs (-1 for negative sizes). */
int64_t llama_decide_full_noalloc_words(int64_t n_inv, int32_t n_ops);

/* Pre-size the scratch that LLAMA_SCAN_FULL (and the grouping by op of
 * llama_decide_alpha, llama_affinity) needs for batches of up to max_inv
 * invocations (device memory, 4 bytes per invocation, 8 with more than
 * 12,288 ops).  Synchronous. */
int llama_reserve(llama_ctx *ctx, int64_t max_inv);

/* Context-level counters (Tab. 3 analogue).  Synchronises the context. */
typedef struct llama_stats {
    int32_t n_ops, n_hw, n_pipelines, max_depth;
    int64_t n_cfg, n_edges;
    int64_t frontier_entries;   /* entries in the per-(op, backend) frontiers */
    uint32_t device_error;      /* LLAMA_DEVERR_* bits seen since the last reset */
    int64_t device_bytes;       /* device memory owned by the context */
} llama_stats;

/* Fill *out; when reset_error is non-zero, clear the device error word. */
int llama_get_stats(llama_ctx *ctx, llama_stats *out, int32_t reset_error);

/*
 * Copy internal tables to host memory, for tests of the ingest step:
 *   what = 0: W for PAPER mode   (int64 [n_ops])
 *   what = 1: W for PROB mode    (int64 [n_ops])
 *   what = 2: packed keys, caller order (uint32 [n_cfg]): rank << 16 | k,
 *             where rank is the dense rank of C/B within the op
 *   what = 3: reference latency  (int32 [n_ops])
 *   what = 4: fastest config     (int32 [n_ops], local index)
 *   what = 5: profiled latencies (int32 [n_cfg], caller order; after
 *             llama_feedback, the smoothed values)
 * `bytes` is the capacity of `host_out`; LLAMA_E_ARG if it is too small.
 */
int llama_debug_export(llama_ctx *ctx, int32_t what, void *host_out, int64_t bytes);

/* ------------------------------------------------------------------------
 * Learned latency surrogate.
 *
 * The paper corrects profiled latencies through a feedback loop and notes
 * that estimators other than exponential smoothing can be used (Sec. 3.3,
 * Manager); it also shows that input content changes an operation's latency
 * several-fold (Sec. 2, Fig. 3).  The surrogate predicts, for each
 * (invocation, configuration) row, the mean and the 95th percentile of
 * ln(latency in microseconds) from a per-row embedding (one per profile row)
 * and 16 content features:
 *     x = [E[row] (16), f (16)], h1 = GELU(W1 x + b1), h2 = GELU(W2 h1 + b2)
 *     (mu, q) = W3 h2 + b3,      hidden width 256, GELU = tanh form
 * BF16 weights, embedding, features and activations; FP32 accumulation, FP32
 * master weights and AdamW state.  Training loss per row:
 *     (mu - y)^2 + rho_0.95(y - q),  rho_t(u) = u (t - [u < 0]),
 * y = observed ln latency.  Parameters are one float vector laid out
 *     E [n_cfg][16], W1 [256][32], b1 [256], W2 [256][256], b2 [256],
 *     W3 [2][256], b3 [2]
 * with n_cfg = the profile's configuration rows.  Features are BF16 bit
 * patterns (uint16), 16 per invocation or training row.
 * ---------------------------------------------------------------------- */
#define LLAMA_SURR_EMB 16
#define LLAMA_SURR_FEAT 16
#define LLAMA_SURR_HIDDEN 256

/* Number of floats in the parameter vector for n_rows profile rows. */
int64_t llama_surrogate_param_count(int64_t n_rows);

/* Deterministic initial parameters from `seed` (normal weights scaled by
 * fan-in, zero biases, b3 = (mean_log_latency, mean_log_latency + 0.5));
 * resets AdamW state.  Needs llama_set_profiles.  Synchronous. */
int llama_surrogate_init(llama_ctx *ctx, uint64_t seed, float mean_log_latency);

/* Replace / read the FP32 parameter vector (host pointer, n floats exactly
 * llama_surrogate_param_count(n_cfg)).  _set resets AdamW state.  Synchronous. */
int llama_surrogate_set(llama_ctx *ctx, const float *params, int64_t n);
int llama_surrogate_get(llama_ctx *ctx, float *params, int64_t n);

/* Gradient of the mean batch loss from the last llama_surrogate_train_step
 * (host pointer, same layout).  Synchronous. */
int llama_surrogate_grads(llama_ctx *ctx, float *grads, int64_t n);

/* Pre-size the training workspace for batches of up to max_batch rows
 * (needed before capturing training or forward calls into a graph). */
int llama_surrogate_reserve(llama_ctx *ctx, int64_t max_batch);

/*
 * The pipeline simulator that generates the surrogate's training executions
 * on the GPU (content-dependent latency, Sec. 2 and Fig. 3).  An execution
 * gets a profile row x uniform over the n_cfg rows, content, and the
 * observed ln latency
 *     ln L[x] + a[op(x) * n_hw + hw(x)] ln(1 + n_obj) + b[op(x)] ln(px / (1280 * 720))
 *     + sigma N(0, 1)
 * with L the row's current profiled latency.  Content: people and cars
 * Poisson with rate exp(ln 2 + N(0, 1)) (people at most 60, cars at most
 * 60 - people), faces Binomial(people, 0.6), resolution 854x480, 1280x720
 * or 1920x1080 uniformly, motion, blur, brightness U(0, 1), branch hit rate
 * Beta(3, 7), frame phase U(0, 2 pi); the 16 BF16 features are people / 60,
 * cars / 60, faces / 60, ln(1 + n_obj) / ln 61, width / 1920, height / 1080,
 * pixels / (1920 * 1080), motion, blur, brightness, hit rate, sin and cos of
 * the phase, and three zeros.  Random numbers: Philox4x32-10 under key
 * (seed mod 2^32, seed / 2^32) at counters (sample, k, 0, 0), k = 0..5, the
 * 24 words used as: 0 row (floor(w n_cfg / 2^32)); 1-4 two Box-Muller pairs
 * (people and cars rates; noise); 5, 6 Poisson inversions; 7 binomial
 * inversion; 8 resolution (floor(3 w / 2^32)); 9-11 motion, blur,
 * brightness; 12-21 the Beta as G3 / (G3 + G7) from sums of unit
 * exponentials; 22 phase; with u = (w + 1/2) / 2^32; arithmetic in FP64.
 * Sample i depends only on (seed, i), so batches may be drawn in any split.
 * llama_set_simulator copies a [n_ops * n_hw], b [n_ops] (host, finite) and
 * sigma >= 0; llama_simulate writes samples first .. first + n - 1
 * (first + n <= 2^32) to device pointers d_rows [n], d_feat [n][16] BF16,
 * d_y [n] FP32 on `stream`.
 */
int llama_set_simulator(llama_ctx *ctx, const double *a_coef, const double *b_coef, double sigma);
int llama_simulate(llama_ctx *ctx, int64_t n, uint64_t seed, int64_t first, int32_t *d_rows,
                   uint16_t *d_feat, float *d_y, void *stream);

/* Training-path forward for n rows (device pointers): d_rows [n] profile row
 * ids, d_feat [n][16] BF16, d_out [n][2] FP32 (mu, q). */
int llama_surrogate_forward(llama_ctx *ctx, int64_t n, const int32_t *d_rows,
                            const uint16_t *d_feat, float *d_out, void *stream);

/* One training step on a batch (device pointers d_rows, d_feat, d_y [batch]
 * observed ln latency): forward, backward into the gradient buffer and, when
 * `update` is non-zero, one AdamW step (betas 0.9, 0.999, eps 1e-8; decoupled
 * weight decay on E, W1, W2, W3) with learning rate lr.  d_loss_sum, when not
 * NULL, has the batch's summed loss added to it.  Two launches per 16,384
 * rows: a fused forward + backward kernel (one workgroup per 64 rows, partial
 * gradients per chunk) and a kernel that sums the chunks in order, applies
 * AdamW and writes the BF16 shadows.  The partial-gradient workspace
 * (299 KB per 64 rows, at most 76.5 MB) is allocated on the first batch of a
 * new size, so reserve it (one uncaptured step of the largest batch) before
 * capturing steps into a graph.  Row ids outside [0, n_cfg) train as zero
 * embedding rows. */
int llama_surrogate_train_step(llama_ctx *ctx, int64_t batch, const int32_t *d_rows,
                               const uint16_t *d_feat, const float *d_y, float lr,
                               float weight_decay, int32_t update, float *d_loss_sum,
                               void *stream);

/* The training recipe, enqueued natively on `stream`: `epochs` passes over n
 * samples (device pointers as in llama_surrogate_train_step) in consecutive
 * batches of `batch` rows (n / batch steps per epoch), one AdamW step each,
 * learning rate lr_max * (1 + cos(pi * step / total)) / 2.  d_loss_sum, when
 * not NULL, accumulates the summed loss of the last tenth of the final epoch. */
int llama_surrogate_fit(llama_ctx *ctx, int64_t n, const int32_t *d_rows,
                        const uint16_t *d_feat, const float *d_y, int32_t epochs,
                        int64_t batch, float lr_max, float weight_decay,
                        float *d_loss_sum, void *stream);

/* Checkpoint: parameters, AdamW moments and step count in one versioned
 * binary file; _load requires the same number of profile rows. */
int llama_surrogate_save(llama_ctx *ctx, const char *path);
int llama_surrogate_load(llama_ctx *ctx, const char *path);

/*
 * llama_decide with the surrogate's latency in place of the profile: for
 * every configuration x of the invocation's op, L(x) = ceil(exp(q)) when the
 * predicted spread q - mu is finite and in [0, spread_max], otherwise the
 * profiled latency; Eq. 1 then runs on those latencies (fallback: the
 * smallest predicted latency).  d_feat [n_inv][16] BF16 content features.
 * d_lat_out, when not NULL, receives each row's latency at
 * [i * lat_stride + k] (lat_stride >= the largest configuration count).
 * The fused kernel keeps every hidden activation on chip.
 */
int llama_decide_learned(llama_ctx *ctx, int64_t n_inv, const int32_t *d_inv_op,
                         const int32_t *d_elapsed_us, const int32_t *d_slo_us,
                         const int64_t *d_queue_us, int32_t slack_mode,
                         const uint16_t *d_feat, float spread_max, int32_t *d_cfg,
                         uint8_t *d_flag, int32_t *d_lat_out, int64_t lat_stride,
                         void *stream);

/* ------------------------------------------------------------------------
 * Serving loop: continuous batching of arriving invocations (the Manager
 * spawning invocations and the Configurator deciding them, Sec. 3.3 and
 * Sec. 4; admission bounded like the paper's commit queues, Sec. 4.3).
 *
 * Requests sit in a ring in pinned host memory mapped into the device: a
 * slot holds a request (16 bytes), its result (8) and the device time it
 * was decided (8), plus 32 bytes of BF16 features in the learned form
 * (llama_serve_bytes_per_request).  The ring is allocated with
 * min(n_slots, mem_budget_bytes / bytes per request) slots, and a request
 * holds its slot from admission until its decision is collected, so the
 * smaller of the two limits how many requests are admitted at once;
 * llama_serve_submit admits the longest prefix that fits and publishes it to
 * the device at once.  A persistent decision kernel of max_inflight
 * workgroups (captured as a HIP graph and relaunched by submit and poll
 * whenever it has exited with requests outstanding) claims published
 * requests as they appear, up to max_batch (at most 64) per wavefront in the
 * plain form and one per workgroup in the learned form (its four wavefronts
 * split the op's configuration rows), and writes each decision with the
 * device time it was made; the kernel exits once no wavefront has claimed
 * work for 20 ms, and after 250 ms in any case.  Decisions are collected in
 * admission order (llama_serve_poll), which frees slots.  While a server is
 * open, the context's tables and surrogate must not be changed.  A server is
 * driven by one caller thread.
 * ---------------------------------------------------------------------- */
typedef struct llama_server llama_server;

typedef struct llama_serve_config {
    int32_t n_slots;           /* ring capacity, >= 1 */
    int64_t mem_budget_bytes;  /* admission budget, >= one request */
    int32_t max_batch;         /* requests one wavefront claims at once (plain form; capped at 64), >= 1 */
    int32_t max_inflight;      /* workgroups of the persistent decision kernel, 1..256 */
    int32_t learned;           /* 0: profile latencies, 1: surrogate (features required) */
    int32_t slack_mode;        /* LLAMA_SLACK_PAPER or LLAMA_SLACK_PROB */
    float spread_max;          /* learned mode: see llama_decide_learned */
} llama_serve_config;

typedef struct llama_serve_stats {
    int64_t submitted, admitted, rejected, decided, collected;
    int64_t batches;            /* claims made by the kernel's wavefronts */
    int64_t bytes_in_use, peak_bytes_in_use;
    int64_t max_batch_seen;     /* largest claim */
    int64_t in_flight_batches;  /* 1 while the persistent kernel runs */
    int64_t capacity;           /* ring slots: min(n_slots, budget / bytes per request) */
    int64_t kernel_launches;    /* graph launches of the persistent kernel */
    int64_t clock_rtt_ns;       /* host round trip of the clock handshake at open (anchor error <= half) */
    int64_t clock_anchors;      /* re-anchorings by handshakes with the running kernel */
    int64_t clock_rate_ppb;     /* fitted device clock period vs its nominal one, parts per 10^9 */
    int64_t clock_probes;       /* handshakes tried with the running kernel */
    int64_t clock_probe_timeouts;     /* of which unanswered within 50 us */
    int64_t clock_probe_rtt_min_ns;   /* shortest answered round trip */
    int64_t clock_probe_rtt_last_ns;  /* latest answered round trip */
} llama_serve_stats;

/* Ring bytes a request holds while admitted (32, or 64 with features). */
int64_t llama_serve_bytes_per_request(int32_t learned);

int llama_serve_open(llama_ctx *ctx, const llama_serve_config *cfg, llama_server **out);

/* Offer n requests (host pointers; feat [n][16] BF16 in learned mode, else
 * may be NULL; arrival_ns: CLOCK_MONOTONIC arrival times, NULL = now).
 * *n_admitted receives how many, from the front, were admitted; tickets
 * [n] (may be NULL) receive their sequence numbers. */
int llama_serve_submit(llama_server *srv, int32_t n, const int32_t *op, const int32_t *elapsed_us,
                       const int32_t *slo_us, const uint16_t *feat, const int64_t *arrival_ns,
                       int64_t *tickets, int32_t *n_admitted);

/* Collect up to max decided requests in admission order (waiting up to
 * wait_ms for the first): tickets, choices, flags and the latency from
 * arrival to the device time of the decision in ns (device clock mapped to
 * CLOCK_MONOTONIC by a handshake at open, re-anchored by handshakes with the
 * running kernel every 10 ms of polling, each waiting at most 50 us, with
 * the rate refitted over the baseline since open; any output may be NULL).
 * *n_out receives the count. */
int llama_serve_poll(llama_server *srv, int32_t max, int64_t *tickets, int32_t *cfg, uint8_t *flag,
                     int64_t *latency_ns, int32_t *n_out, int32_t wait_ms);

int llama_serve_stats_get(llama_server *srv, llama_serve_stats *out);

/* Decide every admitted request (waiting at most 10 s), stop the kernel and
 * free the server. */
int llama_serve_close(llama_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* LLAMA_H */
