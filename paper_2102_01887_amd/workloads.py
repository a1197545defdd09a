"""Seeded synthetic workloads for the decision path.

This module only draws inputs: pipeline DAGs (CSR successor lists with branch
probabilities in Q16), per-operation configuration tables (hardware type,
batch, resource size, latency in integer microseconds, cost in integer
nano-dollars) and pending invocations (op, elapsed time, SLO).  It computes
none of the method's quantities (no reference latency, path latency, slack or
choice), so both the GPU path and the CPU oracle can be fed from it.

Shapes follow the paper's pipelines (Tab. 2: AMBER Alert is 5 ops with a
branch and ~129 configurations per op; Toonify is parallel; Synthetic is a
7-op chain), scaled up to data-parallel sizes.  All randomness is numpy's
PCG64 (``np.random.default_rng(seed)``).
"""
from dataclasses import dataclass, field
import hashlib
from typing import Optional

import numpy as np

Q_ONE = 65536
INT32_MAX = 2**31 - 1


@dataclass
class Workload:
    name: str
    n_hw: int
    pipe_off: np.ndarray          # int32 [P+1]; pipeline p owns ops [pipe_off[p], pipe_off[p+1])
    succ_off: np.ndarray          # int32 [n_ops+1] CSR over global op ids
    succ_ids: np.ndarray          # int32 [n_edges]
    succ_q16: np.ndarray          # uint32 [n_edges], branch probability * 65536, in [1, 65536]
    cfg_off: np.ndarray           # int32 [n_ops+1]
    hw: np.ndarray                # int32 [n_cfg]
    batch: np.ndarray             # int32 [n_cfg]
    res: np.ndarray               # int32 [n_cfg]
    lat: np.ndarray               # int32 [n_cfg], microseconds, >= 1
    cost: np.ndarray              # int64 [n_cfg], nano-dollars per configuration run
    inv_op: np.ndarray            # int32 [n_inv]
    elapsed: np.ndarray           # int32 [n_inv], microseconds
    slo: np.ndarray               # int32 [n_inv], microseconds
    Q: Optional[np.ndarray] = None        # int64 [n_hw] queueing time per backend
    ref_cfg: Optional[np.ndarray] = None  # int32 [n_ops] or None (automatic rule)
    hw_res_total: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def n_ops(self):
        return len(self.cfg_off) - 1

    @property
    def n_pipelines(self):
        return len(self.pipe_off) - 1

    @property
    def n_cfg(self):
        return int(self.cfg_off[-1])

    @property
    def n_inv(self):
        return len(self.inv_op)

    def sha256(self):
        h = hashlib.sha256()
        for k in ("pipe_off", "succ_off", "succ_ids", "succ_q16", "cfg_off", "hw",
                  "batch", "res", "lat", "cost", "inv_op", "elapsed", "slo"):
            h.update(np.ascontiguousarray(getattr(self, k)).tobytes())
        if self.Q is not None:
            h.update(np.ascontiguousarray(self.Q).tobytes())
        return h.hexdigest()

    def with_invocations(self, inv_op, elapsed, slo, Q=None, name=None):
        import copy
        w = copy.copy(self)
        w.inv_op = np.ascontiguousarray(inv_op, np.int32)
        w.elapsed = np.ascontiguousarray(elapsed, np.int32)
        w.slo = np.ascontiguousarray(slo, np.int32)
        w.Q = None if Q is None else np.ascontiguousarray(Q, np.int64)
        if name:
            w.name = name
        return w


def with_resource_totals(w, per_hw=None, slots=16):
    """Copy of w with a resource limit per backend (R_total of Eq. 1 and
    Eq. 2): per_hw if given, else room for `slots` runs of the backend's
    largest configuration."""
    import copy
    w2 = copy.copy(w)
    if per_hw is None:
        per_hw = [slots * int(w.res[w.hw == h].max()) if (w.hw == h).any() else 1
                  for h in range(w.n_hw)]
    w2.hw_res_total = np.ascontiguousarray(per_hw, np.int64)
    return w2


def totals_for_queue(w, q_op, q_cfg, target_us=500_000):
    """Per-backend resource limits that make a queue snapshot's estimated
    waiting time about target_us (one value, or one per backend) on each
    backend (an input recipe: pools sized to their backlogs)."""
    x = w.cfg_off[q_op].astype(np.int64) + q_cfg
    tgt = np.broadcast_to(np.asarray(target_us, np.int64), (w.n_hw,))
    tot = [1] * w.n_hw
    for h in range(w.n_hw):
        sel = w.hw[x] == h
        load = int((w.lat[x[sel]].astype(np.int64) * w.res[x[sel]].astype(np.int64)).sum())
        tot[h] = max(1, load // int(tgt[h]))
    return tot


def queue_snapshot(w, rng, n_q):
    """n_q queued invocations (op, chosen configuration), ops drawn like the
    workload's invocations and configurations uniformly within the op."""
    q_op = w.inv_op[rng.integers(0, w.n_inv, n_q)] if w.n_inv else np.zeros(0, np.int32)
    n_cfg_op = (w.cfg_off[q_op + 1] - w.cfg_off[q_op]).astype(np.int64)
    q_cfg = (rng.random(n_q) * n_cfg_op).astype(np.int64)
    return np.ascontiguousarray(q_op, np.int32), np.ascontiguousarray(q_cfg, np.int32)


def observations(w, rng, n_obs, spread=(0.5, 2.0)):
    """Completed invocations for the feedback step: op and configuration drawn
    like a queue snapshot, observed latency = profile latency times a factor
    log-uniform in `spread` (contention or content making runs slower or
    faster than profiled)."""
    op, cfg = queue_snapshot(w, rng, n_obs)
    x = w.cfg_off[op].astype(np.int64) + cfg
    fac = np.exp(rng.uniform(np.log(spread[0]), np.log(spread[1]), n_obs))
    lat = np.clip(np.rint(w.lat[x] * fac), 1, 2**31 - 1).astype(np.int32)
    return op, cfg, lat


def csr_from_edges(n_ops, src, dst, q=None):
    """CSR successor lists (sorted by destination within each source)."""
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    q = np.full(len(src), Q_ONE, np.int64) if q is None else np.asarray(q, np.int64)
    order = np.lexsort((dst, src))
    src, dst, q = src[order], dst[order], q[order]
    off = np.zeros(n_ops + 1, np.int64)
    np.add.at(off, src + 1, 1)
    off = np.cumsum(off)
    return off.astype(np.int32), dst.astype(np.int32), q.astype(np.uint32)


# ---------------------------------------------------------------------------
# DAG shapes
# ---------------------------------------------------------------------------

def layered_dag(rng, n, d):
    """A layered DAG of n ops over d non-empty levels (ops numbered level by
    level).  Each op of a non-final level gets U{1..3} distinct successors in
    the next level; an op of a later level left without a predecessor gets
    one from the previous level.  Branch probabilities q = round(U[0.05,1]*2^16).
    Returns local (src, dst, q) edge arrays."""
    cuts = np.sort(rng.choice(np.arange(1, n), d - 1, replace=False)) if d > 1 else np.array([], int)
    bounds = np.concatenate([[0], cuts, [n]]).astype(np.int64)
    src, dst = [], []
    for l in range(d - 1):
        a, b = bounds[l], bounds[l + 1]
        c, e = bounds[l + 1], bounds[l + 2]
        width = e - c
        has_pred = np.zeros(width, bool)
        for v in range(a, b):
            k = int(rng.integers(1, 4))
            k = min(k, width)
            succ = rng.choice(width, k, replace=False)
            has_pred[succ] = True
            src.extend([v] * k)
            dst.extend((c + succ).tolist())
        for j in np.nonzero(~has_pred)[0]:
            src.append(int(rng.integers(a, b)))
            dst.append(int(c + j))
    m = len(src)
    q = np.clip(np.rint(rng.uniform(0.05, 1.0, m) * Q_ONE), 1, Q_ONE).astype(np.int64)
    return np.asarray(src, np.int64), np.asarray(dst, np.int64), q


def _assemble_dags(rng, sizes, depth_fn):
    """Concatenate one layered DAG per pipeline into global CSR arrays."""
    pipe_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    S, D, Qs = [], [], []
    for p, n in enumerate(sizes):
        d = depth_fn(int(n))
        s, t, q = layered_dag(rng, int(n), d)
        S.append(s + pipe_off[p])
        D.append(t + pipe_off[p])
        Qs.append(q)
    n_ops = int(pipe_off[-1])
    succ_off, succ_ids, succ_q16 = csr_from_edges(
        n_ops, np.concatenate(S), np.concatenate(D), np.concatenate(Qs))
    return pipe_off.astype(np.int32), succ_off, succ_ids, succ_q16


# ---------------------------------------------------------------------------
# Configuration 1: plain, tiny
# ---------------------------------------------------------------------------

def make_c1(seed=0, queue=False, n_inv=1000):
    """One 6-op DAG: chain 0-1-2-3-4 plus a conditional branch 2->5 taken with
    p = 0.3 (AMBER Alert's detect-then-branch shape).  2 hardware types,
    batch {1,2,4,8} (8 configs/op, k = 4*hw + log2 B, resource 1),
    per-(op,hw) L1 ~ U_int[1e3,1e5], gamma ~ U[0.3,0.9],
    L(B) = clip(floor(L1 * B^gamma), 1e3, 1e5); cost ~ U_int[10, 1e4];
    1000 invocations, SLO 500 ms, elapsed ~ U_int[0, SLO]."""
    rng = np.random.default_rng(seed)
    n_ops, n_hw = 6, 2
    src = [0, 1, 2, 3, 2]
    dst = [1, 2, 3, 4, 5]
    q = [Q_ONE, Q_ONE, Q_ONE, Q_ONE, 19661]
    succ_off, succ_ids, succ_q16 = csr_from_edges(n_ops, src, dst, q)
    B = np.array([1, 2, 4, 8])
    hw, batch, lat = [], [], []
    for v in range(n_ops):
        for h in range(n_hw):
            L1 = int(rng.integers(1000, 100001))
            g = rng.uniform(0.3, 0.9)
            L = np.clip(np.floor(L1 * B.astype(float) ** g), 1000, 100000).astype(np.int64)
            hw.extend([h] * 4)
            batch.extend(B.tolist())
            lat.extend(L.tolist())
    n_cfg = n_ops * 8
    cost = rng.integers(10, 10001, n_cfg).astype(np.int64)
    inv_op = rng.integers(0, n_ops, n_inv).astype(np.int32)
    slo = np.full(n_inv, 500000, np.int32)
    elapsed = rng.integers(0, 500001, n_inv).astype(np.int32)
    return Workload(
        name="c1-plain-tiny" + ("-queue" if queue else ""), n_hw=n_hw,
        pipe_off=np.array([0, n_ops], np.int32), succ_off=succ_off, succ_ids=succ_ids,
        succ_q16=succ_q16, cfg_off=(np.arange(n_ops + 1) * 8).astype(np.int32),
        hw=np.asarray(hw, np.int32), batch=np.asarray(batch, np.int32),
        res=np.ones(n_cfg, np.int32), lat=np.asarray(lat, np.int32), cost=cost,
        inv_op=inv_op, elapsed=elapsed, slo=slo,
        Q=np.array([20000, 5000], np.int64) if queue else None,
        meta={"seed": seed})


# ---------------------------------------------------------------------------
# Configurations 2 and 3: plain scaled / batched uneven
# ---------------------------------------------------------------------------

def _latency_cost(rng, n_ops, n_hw, cfg_off, hw, batch, mem, cost_model="uniform"):
    """Per (op, hw): L1 ~ U_int[1e3,1e5], gamma ~ U[0.3,0.9], beta ~ U[0,0.5];
    per op s ~ lognormal(0, 0.5);  L = clip(floor(s*L1*B^gamma*m^-beta), 1, 2^31-1).
    Cost: max(1, floor(s * U_int[10, 1e4])) ("uniform"), or the paper-shaped
    price_hw * m * L per run ("priced", Sec. 6 resource-second pricing)."""
    n_cfg = len(hw)
    s_op = rng.lognormal(0.0, 0.5, n_ops)
    L1 = rng.integers(1000, 100001, (n_ops, n_hw)).astype(np.float64)
    g = rng.uniform(0.3, 0.9, (n_ops, n_hw))
    be = rng.uniform(0.0, 0.5, (n_ops, n_hw))
    op_of = np.repeat(np.arange(n_ops), np.diff(cfg_off))
    s = s_op[op_of]
    lat = np.floor(s * L1[op_of, hw] * batch.astype(np.float64) ** g[op_of, hw]
                   * mem.astype(np.float64) ** (-be[op_of, hw]))
    lat = np.clip(lat, 1, INT32_MAX).astype(np.int32)
    if cost_model == "uniform":
        cost = np.maximum(1, np.floor(s * rng.integers(10, 10001, n_cfg))).astype(np.int64)
    elif cost_model == "priced":
        price = np.array([1, 3, 7, 12, 20, 30, 45, 60][:n_hw], np.int64)  # nano-$ per (unit * us)
        cost = (price[hw] * mem.astype(np.int64) * lat.astype(np.int64)).astype(np.int64)
    else:
        raise ValueError(cost_model)
    return lat, cost


def _invocations(rng, pipe_off, n_inv, slo_lo=100_000, slo_hi=10_000_000):
    P = len(pipe_off) - 1
    sizes = np.diff(pipe_off).astype(np.int64)
    p = rng.integers(0, P, n_inv)
    local = np.minimum((rng.random(n_inv) * sizes[p]).astype(np.int64), sizes[p] - 1)
    inv_op = (pipe_off[:-1].astype(np.int64)[p] + local).astype(np.int32)
    slo = rng.integers(slo_lo, slo_hi + 1, n_inv).astype(np.int64)
    elapsed = rng.integers(0, slo + 1).astype(np.int32)
    return inv_op, elapsed, slo.astype(np.int32)


def make_c2(seed=1, n_pipelines=256, n_inv=1_000_000, queue=False, cost_model="uniform"):
    """256 layered DAGs of U{10..40} ops over U{3..min(10,n)} levels; 4 hardware
    types x n_b ~ U{4..32} batch values ({1} plus distinct values in 2..64) x
    memory {1,2,4,8} = 64..512 configs/op in caller order (hw, B, mem);
    1M invocations, SLO ~ U_int[0.1 s, 10 s], elapsed ~ U_int[0, SLO]."""
    rng = np.random.default_rng(seed)
    n_hw = 4
    sizes = rng.integers(10, 41, n_pipelines)
    pipe_off, succ_off, succ_ids, succ_q16 = _assemble_dags(
        rng, sizes, lambda n: int(rng.integers(3, min(10, n) + 1)))
    n_ops = int(pipe_off[-1])
    mem_vals = np.array([1, 2, 4, 8], np.int32)
    counts = np.empty(n_ops, np.int64)
    HW, BB, MM = [], [], []
    for v in range(n_ops):
        nb = int(rng.integers(4, 33))
        bs = np.concatenate([[1], np.sort(rng.choice(np.arange(2, 65), nb - 1, replace=False))])
        h, b, m = np.meshgrid(np.arange(n_hw), bs, mem_vals, indexing="ij")
        HW.append(h.ravel()); BB.append(b.ravel()); MM.append(m.ravel())
        counts[v] = h.size
    cfg_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    hw = np.concatenate(HW).astype(np.int32)
    batch = np.concatenate(BB).astype(np.int32)
    res = np.concatenate(MM).astype(np.int32)
    lat, cost = _latency_cost(rng, n_ops, n_hw, cfg_off, hw, batch, res, cost_model)
    inv_op, elapsed, slo = _invocations(rng, pipe_off, n_inv)
    Q = rng.integers(0, 50001, n_hw).astype(np.int64) if queue else None
    return Workload(
        name="c2-plain-scaled" + ("-queue" if queue else "") + ("" if cost_model == "uniform" else "-" + cost_model),
        n_hw=n_hw, pipe_off=pipe_off, succ_off=succ_off, succ_ids=succ_ids,
        succ_q16=succ_q16, cfg_off=cfg_off, hw=hw, batch=batch, res=res, lat=lat,
        cost=cost, inv_op=inv_op, elapsed=elapsed, slo=slo, Q=Q,
        meta={"seed": seed, "n_pipelines": n_pipelines})


def make_c3(seed=2, n_pipelines=4096, n_inv=4_000_000, max_ops=200, max_cfg=2048):
    """4096 pipelines with op counts round(exp(U[ln 3, ln 200])) (the C2 DAG
    generator); configs/op round(exp(U[ln 16, ln 2048])): the reference triple
    (hw 0, B 1, mem 1) plus distinct (hw, B, mem) triples drawn from the
    4 x 64 x 8 grid (B in 1..64, mem in 1..128 powers of two), caller order
    (hw, B, mem); 4M invocations as in C2."""
    rng = np.random.default_rng(seed)
    n_hw = 4
    sizes = np.rint(np.exp(rng.uniform(np.log(3), np.log(max_ops), n_pipelines))).astype(np.int64)
    pipe_off, succ_off, succ_ids, succ_q16 = _assemble_dags(
        rng, sizes, lambda n: int(rng.integers(3, min(10, n) + 1)))
    n_ops = int(pipe_off[-1])
    grid = 4 * 64 * 8
    c = np.rint(np.exp(rng.uniform(np.log(16), np.log(max_cfg), n_ops))).astype(np.int64)
    c = np.minimum(c, grid)
    cfg_off = np.concatenate([[0], np.cumsum(c)]).astype(np.int64)
    idx = np.empty(int(cfg_off[-1]), np.int64)
    for v in range(n_ops):
        a = int(cfg_off[v])
        idx[a] = 0
        idx[a + 1:a + c[v]] = np.sort(rng.choice(grid - 1, c[v] - 1, replace=False) + 1)
    hw = (idx // 512).astype(np.int32)
    batch = ((idx // 8) % 64 + 1).astype(np.int32)
    res = (1 << (idx % 8)).astype(np.int32)
    del idx
    lat, cost = _latency_cost(rng, n_ops, n_hw, cfg_off, hw, batch, res)
    inv_op, elapsed, slo = _invocations(rng, pipe_off, n_inv)
    return Workload(
        name="c3-batched-uneven", n_hw=n_hw, pipe_off=pipe_off, succ_off=succ_off,
        succ_ids=succ_ids, succ_q16=succ_q16, cfg_off=cfg_off.astype(np.int32), hw=hw,
        batch=batch, res=res, lat=lat, cost=cost, inv_op=inv_op, elapsed=elapsed,
        slo=slo, meta={"seed": seed, "n_pipelines": n_pipelines})


# ---------------------------------------------------------------------------
# Small random problems for exhaustive / fuzz checks
# ---------------------------------------------------------------------------

def random_table(rng, n_ops, n_hw, cfg_lo=1, cfg_hi=8, lat_hi=50, cost_hi=30, batch_hi=4,
                 with_reference=True):
    """Random per-op tables with small value ranges (many ties).  When
    with_reference, every op's first configuration is (hw 0, batch 1, res 1)."""
    counts = rng.integers(cfg_lo, cfg_hi + 1, n_ops)
    cfg_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    n = int(cfg_off[-1])
    hw = rng.integers(0, n_hw, n).astype(np.int32)
    batch = rng.integers(1, batch_hi + 1, n).astype(np.int32)
    res = rng.integers(1, 4, n).astype(np.int32)
    lat = rng.integers(1, lat_hi + 1, n).astype(np.int32)
    cost = rng.integers(0, cost_hi + 1, n).astype(np.int64)
    if with_reference:
        first = cfg_off[:-1]
        hw[first] = 0
        batch[first] = 1
        res[first] = 1
    return cfg_off, hw, batch, res, lat, cost


def dag_from_mask(n_ops, mask):
    """DAG on n_ops vertices whose edge set is the bitmask over the
    upper-triangular pairs (i<j) in row-major order."""
    src, dst = [], []
    bit = 0
    for i in range(n_ops):
        for j in range(i + 1, n_ops):
            if (mask >> bit) & 1:
                src.append(i)
                dst.append(j)
            bit += 1
    return src, dst


def random_small(rng, n_ops=None, n_hw=None, n_inv=64, edge_p=0.35, name="fuzz",
                 q_choices=None, max_ref=1000, slo_hi=20000):
    """A single-pipeline random DAG (edges only from lower to higher ids, then
    relabelled by a random permutation) with a random small table."""
    n_ops = int(rng.integers(1, 9)) if n_ops is None else n_ops
    n_hw = int(rng.integers(1, 4)) if n_hw is None else n_hw
    src, dst = [], []
    for i in range(n_ops):
        for j in range(i + 1, n_ops):
            if rng.random() < edge_p:
                src.append(i)
                dst.append(j)
    perm = rng.permutation(n_ops)
    src = [int(perm[s]) for s in src]
    dst = [int(perm[t]) for t in dst]
    if q_choices is None:
        q = rng.integers(1, Q_ONE + 1, len(src))
    else:
        q = rng.choice(np.asarray(q_choices), len(src))
    succ_off, succ_ids, succ_q16 = csr_from_edges(n_ops, src, dst, q)
    cfg_off, hw, batch, res, lat, cost = random_table(rng, n_ops, n_hw, lat_hi=max_ref)
    inv_op = rng.integers(0, n_ops, n_inv).astype(np.int32)
    slo = rng.integers(0, slo_hi + 1, n_inv).astype(np.int32)
    elapsed = rng.integers(0, slo_hi + 1, n_inv).astype(np.int32)
    return Workload(name=name, n_hw=n_hw, pipe_off=np.array([0, n_ops], np.int32),
                    succ_off=succ_off, succ_ids=succ_ids, succ_q16=succ_q16,
                    cfg_off=cfg_off, hw=hw, batch=batch, res=res, lat=lat, cost=cost,
                    inv_op=inv_op, elapsed=elapsed, slo=slo)


# ---------------------------------------------------------------------------
# Configuration 4: learned surrogate (content features, simulator samples)
# ---------------------------------------------------------------------------

N_FEAT = 16
RESOLUTIONS = ((854, 480), (1280, 720), (1920, 1080))
PX_720P = 1280 * 720


@dataclass
class Content:
    """Per-invocation content: integer object counts and resolution (the
    truth model's inputs) and the 16 features the surrogate sees (BF16-exact
    float32 values)."""
    n_obj: np.ndarray      # int32 [n]
    px: np.ndarray         # int64 [n] pixels per frame
    feat: np.ndarray       # float32 [n, 16], already rounded to bfloat16


@dataclass
class SurrogateWorld:
    """C1's DAG with 64 configurations per op and the simulator's hidden truth
    coefficients: mean ln latency of row x for content f is
    ln L[x] + a[op, hw(x)] ln(1 + n_obj(f)) + b[op] ln(px(f) / px_720p),
    observed with lognormal(0, sigma) noise."""
    w: Workload
    a: np.ndarray          # float64 [n_ops, n_hw]
    b: np.ndarray          # float64 [n_ops]
    sigma: float


def _to_bf16_exact(x):
    x32 = np.ascontiguousarray(np.asarray(x, np.float32))
    u = x32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32)


def draw_content(rng, n):
    """Object counts: people and cars Poisson with rate lognormal(ln 2, 1),
    at most 60 objects in all; faces Binomial(people, 0.6); resolution 480p,
    720p or 1080p (the paper's videos are 720p and 1080p, Tab. 2); motion,
    blur, brightness U[0,1]; conditional-branch hit rate Beta(3, 7); frame
    phase U[0, 2 pi)."""
    people = rng.poisson(rng.lognormal(np.log(2.0), 1.0, n))
    cars = rng.poisson(rng.lognormal(np.log(2.0), 1.0, n))
    people = np.minimum(people, 60)
    cars = np.minimum(cars, 60 - people)
    faces = rng.binomial(people, 0.6)
    n_obj = people + cars
    res = rng.integers(0, 3, n)
    wh = np.asarray(RESOLUTIONS, np.int64)[res]
    px = wh[:, 0] * wh[:, 1]
    phase = rng.uniform(0, 2 * np.pi, n)
    f = np.zeros((n, N_FEAT), np.float64)
    f[:, 0] = people / 60.0
    f[:, 1] = cars / 60.0
    f[:, 2] = faces / 60.0
    f[:, 3] = np.log1p(n_obj) / np.log(61.0)
    f[:, 4] = wh[:, 0] / 1920.0
    f[:, 5] = wh[:, 1] / 1080.0
    f[:, 6] = px / (1920.0 * 1080.0)
    f[:, 7] = rng.uniform(0, 1, n)
    f[:, 8] = rng.uniform(0, 1, n)
    f[:, 9] = rng.uniform(0, 1, n)
    f[:, 10] = rng.beta(3, 7, n)
    f[:, 11] = np.sin(phase)
    f[:, 12] = np.cos(phase)
    return Content(n_obj.astype(np.int32), px.astype(np.int64), _to_bf16_exact(f))


def make_c4_world(seed=3, sigma=0.3):
    """C1's 6-op DAG; 64 configurations per op: 2 hardware types x batch
    {1,2,4,8} x 8 resource sizes {1,...,128}, k = 32 hw + 8 log2 B + log2 m;
    L = clip(floor(L1 B^gamma m^-beta), 1e3, 1e5) per (op, hw) draws as in C2;
    cost = price_hw * m * L (resource-seconds priced per backend, Sec. 6);
    truth coefficients a_CPU ~ U[0.3, 0.7], a_GPU ~ U[0.05, 0.35] (spanning
    Fig. 3's 17.2x and 4x at 60 objects), b ~ U[0.5, 1]."""
    base = make_c1(seed=seed, n_inv=1)
    rng = np.random.default_rng(seed + 1000)
    n_ops, n_hw = base.n_ops, 2
    B = np.array([1, 2, 4, 8])
    M = 2 ** np.arange(8)
    hw, batch, res, lat = [], [], [], []
    for v in range(n_ops):
        for h in range(n_hw):
            L1 = int(rng.integers(1000, 100001))
            g = rng.uniform(0.3, 0.9)
            be = rng.uniform(0.0, 0.5)
            for b in B:
                for m in M:
                    hw.append(h); batch.append(b); res.append(m)
                    lat.append(np.clip(np.floor(L1 * float(b) ** g * float(m) ** (-be)), 1000, 100000))
    hw = np.asarray(hw, np.int32)
    res = np.asarray(res, np.int32)
    lat = np.asarray(lat, np.int32)
    price = np.array([1, 3], np.int64)
    cost = price[hw] * res.astype(np.int64) * lat.astype(np.int64)
    n_cfg = len(hw)
    w = Workload(name="c4-surrogate", n_hw=n_hw, pipe_off=base.pipe_off, succ_off=base.succ_off,
                 succ_ids=base.succ_ids, succ_q16=base.succ_q16,
                 cfg_off=(np.arange(n_ops + 1) * 64).astype(np.int32), hw=hw,
                 batch=np.asarray(batch, np.int32), res=res, lat=lat, cost=cost,
                 inv_op=np.zeros(0, np.int32), elapsed=np.zeros(0, np.int32),
                 slo=np.zeros(0, np.int32), meta={"seed": seed})
    a = np.stack([rng.uniform(0.3, 0.7, n_ops), rng.uniform(0.05, 0.35, n_ops)], axis=1)
    b = rng.uniform(0.5, 1.0, n_ops)
    assert n_cfg == n_ops * 64
    return SurrogateWorld(w, a, b, sigma)


def simulate_c4(world, rng, n):
    """n simulator executions: a uniformly drawn profile row, fresh content,
    and the observed ln latency (truth mean plus N(0, sigma^2) noise).
    Returns (rows int32 [n], Content, y float32 [n])."""
    w = world.w
    rows = rng.integers(0, w.n_cfg, n).astype(np.int32)
    c = draw_content(rng, n)
    op = rows // 64
    mu = (np.log(w.lat[rows].astype(np.float64)) + world.a[op, w.hw[rows]] * np.log1p(c.n_obj)
          + world.b[op] * np.log(c.px / PX_720P))
    y = (mu + world.sigma * rng.standard_normal(n)).astype(np.float32)
    return rows, c, y


def c4_invocations(world, rng, n, slo=500_000):
    """n pending invocations of the C4 pipeline (as C1: SLO 500 ms, elapsed
    U[0, SLO]) with their content."""
    w = world.w
    inv_op = rng.integers(0, w.n_ops, n).astype(np.int32)
    elapsed = rng.integers(0, slo + 1, n).astype(np.int32)
    c = draw_content(rng, n)
    return w.with_invocations(inv_op, elapsed, np.full(n, slo, np.int32), name="c4-inference"), c


# ---------------------------------------------------------------------------
# Configuration 5: serving (Poisson arrivals over 1,024 uneven pipelines)
# ---------------------------------------------------------------------------

def make_c5(seed=6, n_pipelines=1024, n_inv=1_000_000, max_cfg=2048):
    """1,024 pipelines shaped as in C3 (op counts 3-200, 16-2048 configurations
    per op) with a pool of invocations as in C2."""
    w = make_c3(seed=seed, n_pipelines=n_pipelines, n_inv=n_inv, max_cfg=max_cfg)
    w.name = "c5-serving"
    return w


def poisson_arrivals(rng, rate_per_s, duration_s):
    """Arrival offsets in ns of a Poisson process of the given rate."""
    n = rng.poisson(rate_per_s * duration_s)
    t = np.sort(rng.uniform(0.0, duration_s, n))
    return (t * 1e9).astype(np.int64)
