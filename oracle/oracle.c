/*
 * CPU oracle for the per-invocation decision path of Llama (Romero, Zhao,
 * Yadwadkar, Kozyrakis, "Llama: A Heterogeneous & Serverless Framework for
 * Auto-Tuning Video Analytics Pipelines", arXiv 2102.01887).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  The product path (the HIP
 * library under paper_2102_01887_amd/) never calls, links or includes it, and
 * this file includes nothing from there.
 *
 * It is written to be read against the paper, not to be fast: every loop is
 * the plain definition, integer arithmetic is exact (128-bit products where
 * a product could need it), and there is no blocking, sorting, ranking or
 * precomputed index of any kind.
 *
 * What it computes
 *   - reference latency of each operation (Sec. 3.2, Operation-Profiler: the
 *     smallest CPU configuration, 1 core and batch 1);
 *   - W[v], the largest remaining reference-path latency from v to any output
 *     operation (Alg. 1, RemainingPathLatency, taken over every sequential
 *     path that contains v; Sec. 4.1 says the path latency starts at op);
 *   - the per-invocation, per-backend slack of Alg. 1:
 *         min over paths P containing v of  ref[v] / pLat(v,P) * remaining
 *     which, because floor(a/x) does not increase with x, equals
 *         floor(ref[v] * remaining / W[v]);
 *   - the Eq. 1 choice: among configurations whose latency is strictly below
 *     the slack of their own backend, the one with the smallest cost per
 *     item C/B, lowest caller index on ties; if none qualifies, the fastest
 *     configuration (smallest L, lowest index on ties).
 *
 * Readings of points the paper leaves open (all integer):
 *   - latencies and times are microseconds, costs nano-dollars;
 *   - remaining = slo - elapsed - Q[h] in 64-bit, clamped to [0, 2^31-1];
 *     a remaining time of 0 gives slack 0 (Alg. 1 is silent past the deadline);
 *   - the slack is the floor of the exact quotient;
 *   - PROB mode discounts each downstream edge by its branch probability,
 *     q/65536 with q in [1, 65536], applied tail-first along the path with a
 *     floor at every step; with every q = 65536 it is Alg. 1 exactly;
 *   - an invocation is invalid when its op is out of range or its elapsed or
 *     slo field is negative: its slack is -1 for every backend and its choice
 *     is -1 with flag 0.
 *
 * Parity pins: the test suite checks this file against literal path
 * enumeration with exact rationals on every 5-op DAG, against closed forms
 * (single op, equal-reference chains, symmetric forks), against a worked
 * example derived by hand from Alg. 1 and Eq. 1, and against invariants.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_E_ARG (-1)
#define ORACLE_E_RANGE (-2)
#define ORACLE_E_CYCLE (-3)
#define ORACLE_E_STATE (-4)

#define ORACLE_PAPER 0
#define ORACLE_PROB 1

#define Q_ONE 65536

/*
 * Reference configuration of each operation (Sec. 3.2): among the op's
 * configurations on hardware type 0 (CPU) with batch 1, the one with the
 * smallest resource size; the lowest caller index wins a tie.  An op with no
 * such configuration is an error (ORACLE_E_STATE).  ref_k receives the local
 * (per-op) index.
 */
int oracle_reference_cfg(int32_t n_ops, const int32_t *cfg_off,
                         const int32_t *hw, const int32_t *batch,
                         const int32_t *res, int32_t *ref_k)
{
    if (n_ops < 0 || !cfg_off || !hw || !batch || !res || !ref_k)
        return ORACLE_E_ARG;
    for (int32_t v = 0; v < n_ops; ++v) {
        int32_t best = -1;
        for (int32_t x = cfg_off[v]; x < cfg_off[v + 1]; ++x) {
            if (hw[x] != 0 || batch[x] != 1)
                continue;
            if (best < 0 || res[x] < res[best])
                best = x;
        }
        if (best < 0)
            return ORACLE_E_STATE;
        ref_k[v] = best - cfg_off[v];
    }
    return ORACLE_OK;
}

/* Value that the edge v->w contributes to W[v] (both modes). */
static int64_t edge_value(int32_t mode, uint32_t q, int64_t w_succ)
{
    if (mode == ORACLE_PAPER)
        return w_succ;
    /* floor(q * W[w] / 65536), exact in 128 bits */
    __int128 p = (__int128)q * (__int128)w_succ;
    return (int64_t)(p / Q_ONE);
}

/*
 * W[v] = ref[v] + max over successors w of edge_value(W[w]); W[v] = ref[v]
 * at an output operation.  This is the largest remaining reference-path
 * latency over every path from v to an output (in PROB mode the Horner form
 * of the path latency, evaluated from the tail).
 *
 * Computed as a plain fixpoint: start from W = ref and sweep every op until
 * nothing changes.  On a DAG this settles after at most (longest path + 1)
 * sweeps; if it is still changing after n_ops + 1 sweeps the graph has a
 * cycle.  succ_q16 may be NULL (every q = 65536).
 */
int oracle_worst_path(int32_t n_ops, const int32_t *succ_off,
                      const int32_t *succ_ids, const uint32_t *succ_q16,
                      const int64_t *ref_lat, int32_t mode, int64_t *W)
{
    if (n_ops < 0 || !succ_off || !ref_lat || !W)
        return ORACLE_E_ARG;
    if (mode != ORACLE_PAPER && mode != ORACLE_PROB)
        return ORACLE_E_ARG;
    for (int32_t v = 0; v < n_ops; ++v)
        W[v] = ref_lat[v];
    for (int64_t sweep = 0; sweep <= (int64_t)n_ops + 1; ++sweep) {
        int changed = 0;
        for (int32_t v = n_ops - 1; v >= 0; --v) {
            int64_t m = 0;
            for (int32_t e = succ_off[v]; e < succ_off[v + 1]; ++e) {
                int32_t w = succ_ids[e];
                if (w < 0 || w >= n_ops)
                    return ORACLE_E_RANGE;
                uint32_t q = succ_q16 ? succ_q16[e] : Q_ONE;
                int64_t c = edge_value(mode, q, W[w]);
                if (c > m)
                    m = c;
            }
            int64_t nv = ref_lat[v] + m;
            if (nv != W[v]) {
                W[v] = nv;
                changed = 1;
            }
        }
        if (!changed)
            return ORACLE_OK;
    }
    return ORACLE_E_CYCLE;
}

/* Remaining time for backend h (reading: clamped to [0, 2^31-1]). */
static int64_t remaining_time(int32_t elapsed, int32_t slo, int64_t q)
{
    __int128 r = (__int128)slo - (__int128)elapsed - (__int128)q;
    if (r < 0)
        r = 0;
    if (r > INT32_MAX)
        r = INT32_MAX;
    return (int64_t)r;
}

/*
 * Alg. 1 for every invocation and every backend h:
 *   target[i*n_hw + h] = floor(ref[v] * R_h / W[v]),  R_h = slo - elapsed - Q[h]
 * Q may be NULL (all zero).  Invalid invocations get -1 for every backend.
 */
int oracle_targets(int64_t n_inv, const int32_t *inv_op,
                   const int32_t *elapsed, const int32_t *slo, int32_t n_hw,
                   const int64_t *Q, int32_t n_ops, const int64_t *ref_lat,
                   const int64_t *W, int32_t *target)
{
    if (n_inv < 0 || n_hw < 1 || n_ops < 0)
        return ORACLE_E_ARG;
    if (n_inv > 0 && (!inv_op || !elapsed || !slo || !target))
        return ORACLE_E_ARG;
    if (!ref_lat || !W)
        return ORACLE_E_ARG;
    for (int64_t i = 0; i < n_inv; ++i) {
        int32_t v = inv_op[i];
        int valid = v >= 0 && v < n_ops && elapsed[i] >= 0 && slo[i] >= 0;
        for (int32_t h = 0; h < n_hw; ++h) {
            int32_t t = -1;
            if (valid) {
                int64_t R = remaining_time(elapsed[i], slo[i], Q ? Q[h] : 0);
                __int128 num = (__int128)ref_lat[v] * (__int128)R;
                t = (int32_t)(num / (__int128)W[v]);
            }
            target[i * n_hw + h] = t;
        }
    }
    return ORACLE_OK;
}

/* Cost per item of x is strictly below that of y: C_x/B_x < C_y/B_y, by exact
 * cross-multiplication. */
static int per_item_less(const int64_t *cost, const int32_t *batch, int32_t x, int32_t y)
{
    __int128 lhs = (__int128)cost[x] * (__int128)batch[y];
    __int128 rhs = (__int128)cost[y] * (__int128)batch[x];
    return lhs < rhs;
}

/*
 * Eq. 1 with the fallback "fastest": for invocation i of op v, scan every
 * configuration x of v.  x is feasible when lat[x] < target[i][hw[x]]
 * (strict, as in Eq. 1).  Among feasible x pick the smallest cost[x]/batch[x]
 * (compared exactly by cross-multiplication), lowest index on ties; flag 1.
 * If none is feasible pick the smallest lat[x], lowest index on ties; flag 0.
 * cfg receives the local index (x - cfg_off[v]); an invocation whose op is
 * out of range gets cfg -1, flag 0.  flag may be NULL.
 */
int oracle_select(int64_t n_inv, const int32_t *inv_op, const int32_t *target,
                  int32_t n_hw, int32_t n_ops, const int32_t *cfg_off,
                  const int32_t *hw, const int32_t *batch,
                  const int32_t *lat, const int64_t *cost, int32_t *cfg,
                  uint8_t *flag)
{
    if (n_inv < 0 || n_hw < 1 || n_ops < 0)
        return ORACLE_E_ARG;
    if (n_inv > 0 && (!inv_op || !target || !cfg))
        return ORACLE_E_ARG;
    if (!cfg_off || !hw || !batch || !lat || !cost)
        return ORACLE_E_ARG;
    for (int64_t i = 0; i < n_inv; ++i) {
        int32_t v = inv_op[i];
        if (v < 0 || v >= n_ops) {
            cfg[i] = -1;
            if (flag)
                flag[i] = 0;
            continue;
        }
        int32_t best = -1;
        for (int32_t x = cfg_off[v]; x < cfg_off[v + 1]; ++x) {
            int32_t h = hw[x];
            if (h < 0 || h >= n_hw)
                return ORACLE_E_RANGE;
            if (!(lat[x] < target[i * n_hw + h]))
                continue;
            if (best < 0) {
                best = x;
                continue;
            }
            if (per_item_less(cost, batch, x, best))
                best = x;
        }
        if (best >= 0) {
            cfg[i] = best - cfg_off[v];
            if (flag)
                flag[i] = 1;
            continue;
        }
        int32_t fast = cfg_off[v];
        for (int32_t x = cfg_off[v] + 1; x < cfg_off[v + 1]; ++x)
            if (lat[x] < lat[fast])
                fast = x;
        cfg[i] = cfg_off[v + 1] > cfg_off[v] ? fast - cfg_off[v] : -1;
        if (flag)
            flag[i] = 0;
    }
    return ORACLE_OK;
}

/*
 * The whole decision for each invocation: Alg. 1 slack for every backend,
 * then the Eq. 1 choice.  Invalid invocations (op out of range, negative
 * elapsed or slo) get cfg -1, flag 0.  target_scratch holds n_hw int32 and is
 * the caller's (so this file allocates nothing per invocation).
 */
int oracle_decide(int64_t n_inv, const int32_t *inv_op, const int32_t *elapsed,
                  const int32_t *slo, int32_t n_hw, const int64_t *Q,
                  int32_t n_ops, const int64_t *ref_lat, const int64_t *W,
                  const int32_t *cfg_off, const int32_t *hw,
                  const int32_t *batch, const int32_t *lat,
                  const int64_t *cost, int32_t *cfg, uint8_t *flag,
                  int32_t *target_scratch)
{
    if (n_inv < 0 || n_hw < 1 || !target_scratch)
        return ORACLE_E_ARG;
    for (int64_t i = 0; i < n_inv; ++i) {
        int rc = oracle_targets(1, inv_op + i, elapsed + i, slo + i, n_hw, Q,
                                n_ops, ref_lat, W, target_scratch);
        if (rc)
            return rc;
        if (target_scratch[0] < 0) {
            cfg[i] = -1;
            if (flag)
                flag[i] = 0;
            continue;
        }
        rc = oracle_select(1, inv_op + i, target_scratch, n_hw, n_ops, cfg_off,
                           hw, batch, lat, cost, cfg + i, flag ? flag + i : 0);
        if (rc)
            return rc;
    }
    return ORACLE_OK;
}

/*
 * Eq. 1 with per-invocation latencies (the learned form): identical to
 * oracle_select except that configuration x of invocation i is feasible when
 * lat_inv[i * lat_stride + (x - cfg_off[v])] < target[i][hw[x]], and the
 * fallback is the configuration with the smallest such latency (lowest index
 * on ties).  Costs and batches are the profile's.
 */
int oracle_select_lat(int64_t n_inv, const int32_t *inv_op, const int32_t *target,
                      int32_t n_hw, int32_t n_ops, const int32_t *cfg_off,
                      const int32_t *hw, const int32_t *batch,
                      const int32_t *lat_inv, int64_t lat_stride,
                      const int64_t *cost, int32_t *cfg, uint8_t *flag)
{
    if (n_inv < 0 || n_hw < 1 || n_ops < 0 || lat_stride < 0)
        return ORACLE_E_ARG;
    if (n_inv > 0 && (!inv_op || !target || !cfg || !lat_inv))
        return ORACLE_E_ARG;
    if (!cfg_off || !hw || !batch || !cost)
        return ORACLE_E_ARG;
    for (int64_t i = 0; i < n_inv; ++i) {
        int32_t v = inv_op[i];
        if (v < 0 || v >= n_ops || cfg_off[v + 1] - cfg_off[v] > lat_stride) {
            cfg[i] = -1;
            if (flag)
                flag[i] = 0;
            continue;
        }
        const int32_t *L = lat_inv + i * lat_stride - cfg_off[v];
        int32_t best = -1;
        for (int32_t x = cfg_off[v]; x < cfg_off[v + 1]; ++x) {
            int32_t h = hw[x];
            if (h < 0 || h >= n_hw)
                return ORACLE_E_RANGE;
            if (!(L[x] < target[i * n_hw + h]))
                continue;
            if (best < 0) {
                best = x;
                continue;
            }
            if (per_item_less(cost, batch, x, best))
                best = x;
        }
        if (best >= 0) {
            cfg[i] = best - cfg_off[v];
            if (flag)
                flag[i] = 1;
            continue;
        }
        int32_t fast = cfg_off[v];
        for (int32_t x = cfg_off[v] + 1; x < cfg_off[v + 1]; ++x)
            if (L[x] < L[fast])
                fast = x;
        cfg[i] = fast - cfg_off[v];
        if (flag)
            flag[i] = 0;
    }
    return ORACLE_OK;
}

/*
 * Eq. 2 (Sec. 4.3): the estimated queueing time of backend h over the
 * invocations queued there (the speculative and the commit queue together),
 *     Q[h] = sum over queued i with hw(x_i) = h of L(x_i) * R(x_i) / R_total(h),
 * where x_i is the configuration chosen for queued invocation i.  Reading:
 * the products L * R are summed exactly (128-bit), the sum is divided once by
 * R_total(h) and floored; a quotient above 2^62 is reported as 2^62 (such a
 * queueing time already leaves no remaining time).  Queued entries whose op
 * or configuration index is out of range are left out; *n_skipped (if not
 * NULL) receives their number.  n_hw is at most 64.
 */
int oracle_queue_time(int64_t n_q, const int32_t *q_op, const int32_t *q_cfg,
                      int32_t n_hw, int32_t n_ops, const int32_t *cfg_off,
                      const int32_t *hw, const int32_t *res, const int32_t *lat,
                      const int64_t *r_total, int64_t *Q, int64_t *n_skipped)
{
    unsigned __int128 sum[64];
    int64_t skipped = 0;
    if (n_q < 0 || n_hw < 1 || n_hw > 64 || n_ops < 0 || !Q || !r_total)
        return ORACLE_E_ARG;
    if (n_q > 0 && (!q_op || !q_cfg))
        return ORACLE_E_ARG;
    for (int32_t h = 0; h < n_hw; ++h) {
        if (r_total[h] < 1)
            return ORACLE_E_RANGE;
        sum[h] = 0;
    }
    for (int64_t i = 0; i < n_q; ++i) {
        int32_t v = q_op[i];
        if (v < 0 || v >= n_ops || q_cfg[i] < 0 || q_cfg[i] >= cfg_off[v + 1] - cfg_off[v]) {
            ++skipped;
            continue;
        }
        int32_t x = cfg_off[v] + q_cfg[i];
        if (hw[x] < 0 || hw[x] >= n_hw)
            return ORACLE_E_RANGE;
        sum[hw[x]] += (unsigned __int128)(uint32_t)lat[x] * (unsigned __int128)(uint32_t)res[x];
    }
    for (int32_t h = 0; h < n_hw; ++h) {
        unsigned __int128 q = sum[h] / (unsigned __int128)r_total[h];
        Q[h] = q > ((unsigned __int128)1 << 62) ? ((int64_t)1 << 62) : (int64_t)q;
    }
    if (n_skipped)
        *n_skipped = skipped;
    return ORACLE_OK;
}

/* a * b as a 256-bit number, four 64-bit limbs, least significant first. */
static void wide_product(unsigned __int128 a, unsigned __int128 b, uint64_t out[4])
{
    uint64_t al = (uint64_t)a, ah = (uint64_t)(a >> 64);
    uint64_t bl = (uint64_t)b, bh = (uint64_t)(b >> 64);
    unsigned __int128 ll = (unsigned __int128)al * bl;
    unsigned __int128 lh = (unsigned __int128)al * bh;
    unsigned __int128 hl = (unsigned __int128)ah * bl;
    unsigned __int128 hh = (unsigned __int128)ah * bh;
    unsigned __int128 mid = (ll >> 64) + (uint64_t)lh + (uint64_t)hl;
    out[0] = (uint64_t)ll;
    out[1] = (uint64_t)mid;
    unsigned __int128 top = (mid >> 64) + (lh >> 64) + (hl >> 64) + (uint64_t)hh;
    out[2] = (uint64_t)top;
    out[3] = (uint64_t)(top >> 64) + (uint64_t)(hh >> 64);
}

/* n1/d1 < n2/d2 for non-negative numerators and positive denominators,
 * decided on the exact 256-bit products n1*d2 and n2*d1. */
static int fraction_below(unsigned __int128 n1, unsigned __int128 d1,
                          unsigned __int128 n2, unsigned __int128 d2)
{
    uint64_t p[4], r[4];
    wide_product(n1, d2, p);
    wide_product(n2, d1, r);
    for (int k = 3; k >= 0; --k)
        if (p[k] != r[k])
            return p[k] < r[k];
    return 0;
}

/*
 * Eq. 1 with a finite weight alpha = alpha_num / alpha_den (Sec. 4.2): for
 * invocation i of op v every configuration x of v is scored
 *     obj(x) = C/B                                    when L < slack_{hw(x)}
 *     obj(x) = C/B + alpha * L * R / (B * R_total(hw(x)))   otherwise,
 * written as the single fraction
 *     (C * R_total * alpha_den + [L >= slack] * alpha_num * L * R)
 *       / (B * R_total * alpha_den),
 * and the configuration with the smallest obj is chosen, lowest caller index
 * on ties; flag 1 when the chosen configuration meets its slack.  Bounds that
 * keep every numerator and denominator below 2^128: cost <= 2^40, batch <=
 * 2^16, R_total <= 2^40, alpha_num < 2^32, 1 <= alpha_den < 2^32.
 */
int oracle_select_alpha(int64_t n_inv, const int32_t *inv_op, const int32_t *target,
                        int32_t n_hw, int32_t n_ops, const int32_t *cfg_off,
                        const int32_t *hw, const int32_t *batch, const int32_t *res,
                        const int32_t *lat, const int64_t *cost, const int64_t *r_total,
                        uint32_t alpha_num, uint32_t alpha_den, int32_t *cfg, uint8_t *flag)
{
    if (n_inv < 0 || n_hw < 1 || n_ops < 0 || alpha_den < 1)
        return ORACLE_E_ARG;
    if (n_inv > 0 && (!inv_op || !target || !cfg))
        return ORACLE_E_ARG;
    if (!cfg_off || !hw || !batch || !res || !lat || !cost || !r_total)
        return ORACLE_E_ARG;
    for (int64_t i = 0; i < n_inv; ++i) {
        int32_t v = inv_op[i];
        if (v < 0 || v >= n_ops || cfg_off[v + 1] <= cfg_off[v]) {
            cfg[i] = -1;
            if (flag)
                flag[i] = 0;
            continue;
        }
        int32_t best = -1;
        int best_meets = 0;
        unsigned __int128 best_n = 0, best_d = 1;
        for (int32_t x = cfg_off[v]; x < cfg_off[v + 1]; ++x) {
            int32_t h = hw[x];
            if (h < 0 || h >= n_hw || r_total[h] < 1)
                return ORACLE_E_RANGE;
            int meets = lat[x] < target[i * n_hw + h];
            unsigned __int128 num = (unsigned __int128)(uint64_t)cost[x] * (uint64_t)r_total[h] * alpha_den;
            if (!meets)
                num += (unsigned __int128)alpha_num * (uint32_t)lat[x] * (uint32_t)res[x];
            unsigned __int128 den = (unsigned __int128)(uint32_t)batch[x] * (uint64_t)r_total[h] * alpha_den;
            if (best < 0 || fraction_below(num, den, best_n, best_d)) {
                best = x;
                best_meets = meets;
                best_n = num;
                best_d = den;
            }
        }
        cfg[i] = best - cfg_off[v];
        if (flag)
            flag[i] = (uint8_t)best_meets;
    }
    return ORACLE_OK;
}

/* Alg. 1 slack for every backend, then oracle_select_alpha, per invocation.
 * Invalid invocations (op out of range, negative elapsed or slo) get cfg -1,
 * flag 0.  target_scratch holds n_hw int32 (the caller's). */
int oracle_decide_alpha(int64_t n_inv, const int32_t *inv_op, const int32_t *elapsed,
                        const int32_t *slo, int32_t n_hw, const int64_t *Q,
                        int32_t n_ops, const int64_t *ref_lat, const int64_t *W,
                        const int32_t *cfg_off, const int32_t *hw, const int32_t *batch,
                        const int32_t *res, const int32_t *lat, const int64_t *cost,
                        const int64_t *r_total, uint32_t alpha_num, uint32_t alpha_den,
                        int32_t *cfg, uint8_t *flag, int32_t *target_scratch)
{
    if (n_inv < 0 || n_hw < 1 || !target_scratch)
        return ORACLE_E_ARG;
    for (int64_t i = 0; i < n_inv; ++i) {
        int rc = oracle_targets(1, inv_op + i, elapsed + i, slo + i, n_hw, Q,
                                n_ops, ref_lat, W, target_scratch);
        if (rc)
            return rc;
        if (target_scratch[0] < 0) {
            cfg[i] = -1;
            if (flag)
                flag[i] = 0;
            continue;
        }
        rc = oracle_select_alpha(1, inv_op + i, target_scratch, n_hw, n_ops, cfg_off, hw,
                                 batch, res, lat, cost, r_total, alpha_num, alpha_den,
                                 cfg + i, flag ? flag + i : 0);
        if (rc)
            return rc;
    }
    return ORACLE_OK;
}

/* n1/d1 < n2/d2 for 128-bit operands given as two 64-bit limbs each (least
 * significant first); exported so that the 256-bit comparison can be checked
 * on its own over the full operand range. */
int oracle_fraction_below(const uint64_t *n1, const uint64_t *d1, const uint64_t *n2,
                          const uint64_t *d2)
{
    unsigned __int128 a = ((unsigned __int128)n1[1] << 64) | n1[0];
    unsigned __int128 b = ((unsigned __int128)d1[1] << 64) | d1[0];
    unsigned __int128 c = ((unsigned __int128)n2[1] << 64) | n2[0];
    unsigned __int128 d = ((unsigned __int128)d2[1] << 64) | d2[0];
    return fraction_below(a, b, c, d);
}

/*
 * Feedback (Sec. 3.3, Manager): the profiled latency of each configuration is
 * updated from observed latencies by exponential smoothing.  Readings: the
 * smoothing factor is beta = beta_q16 / 65536 in [0, 1]; the m >= 1
 * observations of a configuration in one batch, with sum S, make one
 * smoothing step toward their mean,
 *     L_new = L + floor(beta_q16 * (S - m * L) / (65536 * m)),
 * the floor taken exactly (also for negative numerators) and the result
 * clamped to [1, 2^31 - 1]; with m = 1 this is floor((1 - beta) L + beta obs).
 * Observations whose op or configuration index is out of range, or whose
 * latency is below 1, are left out; *n_skipped (if not NULL) counts them.
 * lat is updated in place (caller order).
 */
int oracle_feedback(int64_t n_obs, const int32_t *obs_op, const int32_t *obs_cfg,
                    const int32_t *obs_lat, int32_t n_ops, const int32_t *cfg_off,
                    int32_t *lat, uint32_t beta_q16, int64_t *n_skipped)
{
    if (n_obs < 0 || n_ops < 0 || !cfg_off || !lat || beta_q16 > 65536u)
        return ORACLE_E_ARG;
    if (n_obs > 0 && (!obs_op || !obs_cfg || !obs_lat))
        return ORACLE_E_ARG;
    int64_t n_cfg = cfg_off[n_ops];
    int64_t skipped = 0;
    /* count and sum of each configuration's observations */
    int64_t *m = calloc((size_t)(n_cfg > 0 ? n_cfg : 1), sizeof(int64_t));
    __int128 *S = calloc((size_t)(n_cfg > 0 ? n_cfg : 1), sizeof(__int128));
    if (!m || !S) {
        free(m);
        free(S);
        return ORACLE_E_ARG;
    }
    for (int64_t i = 0; i < n_obs; ++i) {
        int32_t v = obs_op[i];
        if (v < 0 || v >= n_ops || obs_cfg[i] < 0 || obs_cfg[i] >= cfg_off[v + 1] - cfg_off[v] ||
            obs_lat[i] < 1) {
            ++skipped;
            continue;
        }
        int64_t x = cfg_off[v] + obs_cfg[i];
        m[x] += 1;
        S[x] += obs_lat[i];
    }
    /* one smoothing step per observed configuration */
    for (int64_t x = 0; x < n_cfg; ++x) {
        if (m[x] == 0)
            continue;
        __int128 num = (__int128)beta_q16 * (S[x] - (__int128)m[x] * lat[x]);
        __int128 den = (__int128)65536 * m[x];
        __int128 q = num / den;
        if (num % den != 0 && num < 0)
            q -= 1; /* floor, not truncation */
        __int128 nl = (__int128)lat[x] + q;
        if (nl < 1)
            nl = 1;
        if (nl > 2147483647)
            nl = 2147483647;
        lat[x] = (int32_t)nl;
    }
    free(m);
    free(S);
    if (n_skipped)
        *n_skipped = skipped;
    return ORACLE_OK;
}

/*
 * Eq. 3 (Sec. 4.4, priority-based commit): the affinity of an invocation of
 * op v to backend h is
 *     min over x of v not on h of obj(x)  /  min over x of v on h of obj(x),
 * obj being Eq. 1 with the finite weight alpha (oracle_select_alpha) and each
 * configuration's slack that of its own backend.  This function returns the
 * two minima as exact fractions, per (invocation, backend), for the caller to
 * divide: own_* is the minimum over the backend's configurations, oth_* over
 * the others; each value is num / den with 128-bit num and den given as two
 * 64-bit limbs (least significant first) at [(i * n_hw + h) * 2].  A side
 * without any configuration has den 0.  Invalid invocations (op out of range,
 * negative elapsed or slo) get den 0 on both sides.
 */
int oracle_affinity_terms(int64_t n_inv, const int32_t *inv_op, const int32_t *elapsed,
                          const int32_t *slo, int32_t n_hw, const int64_t *Q,
                          int32_t n_ops, const int64_t *ref_lat, const int64_t *W,
                          const int32_t *cfg_off, const int32_t *hw, const int32_t *batch,
                          const int32_t *res, const int32_t *lat, const int64_t *cost,
                          const int64_t *r_total, uint32_t alpha_num, uint32_t alpha_den,
                          uint64_t *own_num, uint64_t *own_den, uint64_t *oth_num,
                          uint64_t *oth_den, int32_t *target_scratch)
{
    if (n_inv < 0 || n_hw < 1 || !target_scratch || alpha_den < 1)
        return ORACLE_E_ARG;
    for (int64_t i = 0; i < n_inv; ++i) {
        for (int32_t h = 0; h < n_hw; ++h) {
            int64_t o = (i * n_hw + h) * 2;
            own_num[o] = own_num[o + 1] = own_den[o] = own_den[o + 1] = 0;
            oth_num[o] = oth_num[o + 1] = oth_den[o] = oth_den[o + 1] = 0;
        }
        int rc = oracle_targets(1, inv_op + i, elapsed + i, slo + i, n_hw, Q, n_ops, ref_lat, W,
                                target_scratch);
        if (rc)
            return rc;
        if (target_scratch[0] < 0)
            continue;
        int32_t v = inv_op[i];
        for (int32_t h = 0; h < n_hw; ++h) {
            int have_own = 0, have_oth = 0;
            unsigned __int128 on = 0, od = 1, tn = 0, td = 1;
            for (int32_t x = cfg_off[v]; x < cfg_off[v + 1]; ++x) {
                int32_t g = hw[x];
                if (g < 0 || g >= n_hw || r_total[g] < 1)
                    return ORACLE_E_RANGE;
                int meets = lat[x] < target_scratch[g];
                unsigned __int128 num = (unsigned __int128)(uint64_t)cost[x] * (uint64_t)r_total[g] * alpha_den;
                if (!meets)
                    num += (unsigned __int128)alpha_num * (uint32_t)lat[x] * (uint32_t)res[x];
                unsigned __int128 den = (unsigned __int128)(uint32_t)batch[x] * (uint64_t)r_total[g] * alpha_den;
                if (g == h) {
                    if (!have_own || fraction_below(num, den, on, od)) {
                        on = num;
                        od = den;
                        have_own = 1;
                    }
                } else if (!have_oth || fraction_below(num, den, tn, td)) {
                    tn = num;
                    td = den;
                    have_oth = 1;
                }
            }
            int64_t o = (i * n_hw + h) * 2;
            if (have_own) {
                own_num[o] = (uint64_t)on;
                own_num[o + 1] = (uint64_t)(on >> 64);
                own_den[o] = (uint64_t)od;
                own_den[o + 1] = (uint64_t)(od >> 64);
            }
            if (have_oth) {
                oth_num[o] = (uint64_t)tn;
                oth_num[o + 1] = (uint64_t)(tn >> 64);
                oth_den[o] = (uint64_t)td;
                oth_den[o + 1] = (uint64_t)(td >> 64);
            }
        }
    }
    return ORACLE_OK;
}

/* Eq. 1 (fastest fallback) for one invocation over the configurations of op
 * v whose batch is at most max_batch; -1 if there is none.  *meets receives
 * whether the choice meets its slack. */
static int32_t select_within(int32_t v, const int32_t *target, const int32_t *cfg_off,
                             const int32_t *hw, const int32_t *batch, const int32_t *lat,
                             const int64_t *cost, int64_t max_batch, int *meets)
{
    int32_t best = -1, fast = -1;
    for (int32_t x = cfg_off[v]; x < cfg_off[v + 1]; ++x) {
        if (batch[x] > max_batch)
            continue;
        if (fast < 0 || lat[x] < lat[fast])
            fast = x;
        if (lat[x] < target[hw[x]] && (best < 0 || per_item_less(cost, batch, x, best)))
            best = x;
    }
    *meets = best >= 0;
    return best >= 0 ? best : fast;
}

/*
 * Safe delayed batching (Sec. 4.4).  Per invocation of op v, with
 * available[v] invocations of v ready now, upstream[v] more expected from
 * upstream work already running, and wait_us[v] the estimated time until
 * they arrive (all caller inputs, per op):
 *   1. x* = the Eq. 1 choice over every configuration (fastest fallback);
 *   2. if B(x*) <= available[v]: commit x*;
 *   3. else, if x* meets its slack, available[v] + upstream[v] >= B(x*) and
 *      wait_us[v] + L(x*) < slack of x*'s backend: wait (cfg -2, flag 1);
 *   4. else commit the Eq. 1 choice over the configurations with
 *      B <= max(available[v], 1) (fastest fallback), or x* if there is none.
 * flag is 1 when the committed configuration meets its slack.  Invalid
 * invocations get cfg -1, flag 0.  target_scratch holds n_hw int32.
 */
int oracle_decide_batching(int64_t n_inv, const int32_t *inv_op, const int32_t *elapsed,
                           const int32_t *slo, int32_t n_hw, const int64_t *Q,
                           int32_t n_ops, const int64_t *ref_lat, const int64_t *W,
                           const int32_t *cfg_off, const int32_t *hw, const int32_t *batch,
                           const int32_t *lat, const int64_t *cost, const int32_t *available,
                           const int32_t *upstream, const int32_t *wait_us, int32_t *cfg,
                           uint8_t *flag, int32_t *target_scratch)
{
    if (n_inv < 0 || n_hw < 1 || !target_scratch || !available || !upstream || !wait_us)
        return ORACLE_E_ARG;
    for (int64_t i = 0; i < n_inv; ++i) {
        int rc = oracle_targets(1, inv_op + i, elapsed + i, slo + i, n_hw, Q, n_ops, ref_lat, W,
                                target_scratch);
        if (rc)
            return rc;
        if (target_scratch[0] < 0) {
            cfg[i] = -1;
            flag[i] = 0;
            continue;
        }
        int32_t v = inv_op[i];
        int meets = 0;
        int32_t xs = select_within(v, target_scratch, cfg_off, hw, batch, lat, cost, INT64_MAX, &meets);
        int64_t avail = available[v];
        if (batch[xs] <= avail) {
            cfg[i] = xs - cfg_off[v];
            flag[i] = (uint8_t)meets;
            continue;
        }
        if (meets && avail + (int64_t)upstream[v] >= batch[xs] &&
            (int64_t)wait_us[v] + lat[xs] < target_scratch[hw[xs]]) {
            cfg[i] = -2;
            flag[i] = 1;
            continue;
        }
        int meets_r = 0;
        int32_t xr = select_within(v, target_scratch, cfg_off, hw, batch, lat, cost, avail > 1 ? avail : 1,
                                   &meets_r);
        if (xr < 0) {
            cfg[i] = xs - cfg_off[v];
            flag[i] = (uint8_t)meets;
        } else {
            cfg[i] = xr - cfg_off[v];
            flag[i] = (uint8_t)meets_r;
        }
    }
    return ORACLE_OK;
}
