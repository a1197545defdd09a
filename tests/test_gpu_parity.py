"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Everything is integer, so every comparison is bit-exact: targets, chosen
configuration index and flag, W for both slack modes, packed keys.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2102_01887_amd import binding as B
from paper_2102_01887_amd import workloads as wl

pytestmark = pytest.mark.gpu

PAPER, PROB = 0, 1
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a, torch):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


class Run:
    """A workload loaded into one context, with its invocations on the GPU."""

    def __init__(self, w):
        self.torch = torch = _torch()
        self.w = w
        self.L = B.Llama(0).load(w)
        self.op = dev(w.inv_op, torch)
        self.el = dev(w.elapsed, torch)
        self.slo = dev(w.slo, torch)
        self.P = oracle.Problem(w)

    def q(self, Q):
        return None if Q is None else dev(np.asarray(Q, np.int64), self.torch)

    def targets(self, mode, Q=None):
        t = self.L.targets(self.op, self.el, self.slo, self.q(Q), mode)
        self.torch.cuda.synchronize()
        return t.cpu().numpy()

    def decide(self, mode, scan, Q=None):
        c, f = self.L.decide(self.op, self.el, self.slo, self.q(Q), mode, scan)
        self.torch.cuda.synchronize()
        return c.cpu().numpy(), f.cpu().numpy()

    def select(self, target):
        c, f = self.L.select(self.op, dev(target.astype(np.int32), self.torch))
        self.torch.cuda.synchronize()
        return c.cpu().numpy(), f.cpu().numpy()


def assert_full_parity(r, Q=None, modes=(PAPER, PROB), scans=B.SCANS):
    say(f"parity {r.w.name}: n_ops={r.w.n_ops} n_cfg={r.w.n_cfg} n_inv={r.w.n_inv} Q={Q}")
    for mode in modes:
        assert np.array_equal(r.L.export("W_paper" if mode == PAPER else "W_prob"), r.P.W(mode))
        t_or = r.P.targets(mode, Q=Q)
        t_gpu = r.targets(mode, Q)
        assert np.array_equal(t_gpu, t_or), f"targets mode {mode}"
        c_or, f_or = r.P.decide(mode, Q=Q)
        for scan in scans:
            c, f = r.decide(mode, scan, Q)
            bad = np.nonzero((c != c_or) | (f != f_or))[0]
            assert bad.size == 0, f"mode {mode} scan {scan}: {bad.size} mismatches, first {bad[:5]}"
        # select given the oracle's own targets
        c, f = r.select(t_or)
        c2, f2 = r.P.select(t_or)
        assert np.array_equal(c, c2) and np.array_equal(f, f2), f"select mode {mode}"


def test_worked_example():
    torch = _torch()
    g = json.load(open(GOLDEN))
    s, t = g["tables"], g["succ"]
    so, si, sq = wl.csr_from_edges(4, t["src"], t["dst"], t["q16"])
    inv = g["invocations"]
    w = wl.Workload("worked", 2, np.array([0, 4], np.int32), so, si, sq,
                    np.array(s["cfg_off"], np.int32), np.array(s["hw"], np.int32),
                    np.array(s["batch"], np.int32), np.array(s["res"], np.int32),
                    np.array(s["lat"], np.int32), np.array(s["cost"], np.int64),
                    np.array([i["op"] for i in inv], np.int32),
                    np.array([i["elapsed"] for i in inv], np.int32),
                    np.array([i["slo"] for i in inv], np.int32))
    r = Run(w)
    assert r.L.export("W_paper").tolist() == g["W"]["paper"]
    assert r.L.export("W_prob").tolist() == g["W"]["prob"]
    assert r.L.export("ref").tolist() == g["ref"]
    assert r.L.export("key")[1:6].tolist() == g["dense_rank_op1"]["key"]
    tp, tq = r.targets(PAPER), r.targets(PROB)
    for i, c in enumerate(inv):
        assert tp[i].tolist() == [c["target_paper"]] * 2
        assert tq[i].tolist() == [c["target_prob"]] * 2
    for scan in B.SCANS:
        cfg, flag = r.decide(PAPER, scan)
        assert cfg[0] == inv[0]["cfg_paper"] and flag[0] == 1
    cases = g["select_op1"]
    n = len(cases)
    op = torch.ones(n, dtype=torch.int32, device="cuda")
    tg = dev(np.array([[c["target"]] * 2 for c in cases], np.int32), torch)
    cfg, flag = r.L.select(op, tg)
    torch.cuda.synchronize()
    assert cfg.cpu().tolist() == [c["cfg"] for c in cases]
    assert flag.cpu().tolist() == [c["flag"] for c in cases]


@pytest.mark.parametrize("queue", [False, True])
def test_c1_plain_tiny(queue):
    w = wl.make_c1(queue=queue)
    assert_full_parity(Run(w), Q=w.Q)


@pytest.mark.parametrize("queue", [False, True])
def test_c2_reduced(queue):
    # 16 pipelines, 20,001 invocations: several tiles plus a ragged tail
    w = wl.make_c2(seed=5, n_pipelines=16, n_inv=20_001, queue=queue)
    assert_full_parity(Run(w), Q=w.Q)


def test_c2_priced_costs():
    # paper-shaped costs (price * resource * latency): long frontiers
    w = wl.make_c2(seed=6, n_pipelines=8, n_inv=5_000, cost_model="priced")
    assert_full_parity(Run(w))


def test_c2_full_size():
    # the benchmark workload: 256 pipelines, 1M invocations, every decision
    w = wl.make_c2()
    r = Run(w)
    say("c2 full: oracle decide (1M invocations)")
    for mode in (PAPER, PROB):
        c_or, f_or = r.P.decide(mode)
        for scan in B.SCANS:
            c, f = r.decide(mode, scan)
            assert np.array_equal(c, c_or) and np.array_equal(f, f_or), (mode, scan)
    sl = slice(0, 200_000)
    t = r.targets(PAPER)[sl]
    assert np.array_equal(t, r.P.targets(PAPER, sl=sl))


def test_fuzz_small_dags_with_ties():
    rng = np.random.default_rng(99)
    for it in range(60):
        w = wl.random_small(rng, n_inv=int(rng.integers(1, 700)))
        Q = rng.integers(0, 5000, w.n_hw) if it % 3 == 0 else None
        assert_full_parity(Run(w), Q=Q)


def test_empty_batch_and_invalid_invocations():
    torch = _torch()
    w = wl.make_c1()
    r = Run(w)
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    c, f = r.L.decide(e, e, e)
    t = r.L.targets(e, e, e)
    torch.cuda.synchronize()
    assert c.numel() == 0 and t.numel() == 0
    r.L.stats(reset_error=True)
    bad = w.with_invocations([-1, 6, 1 << 30, 2, 2, 2, 3], [0, 0, 0, -1, 0, 9, 0],
                             [10, 10, 10, 10, -1, 5, 2**31 - 1])
    rb = Run(bad)
    rb.L.stats(reset_error=True)
    for scan in B.SCANS:
        c, f = rb.decide(PAPER, scan)
        c_or, f_or = rb.P.decide(PAPER)
        assert c.tolist() == c_or.tolist() and f.tolist() == f_or.tolist()
        assert c[:5].tolist() == [-1] * 5
    assert rb.L.stats()["device_error"] & B.DEVERR_INVALID_INVOCATION
    t = rb.targets(PAPER)
    assert np.array_equal(t, rb.P.targets(PAPER))
    assert (t[:5] == -1).all()
    assert rb.L.stats(reset_error=True)["device_error"] != 0
    assert rb.L.stats()["device_error"] == 0


def test_extreme_values():
    # maximal latencies, costs, batches, SLOs; zero costs; huge queueing time
    rng = np.random.default_rng(3)
    n_ops, n_hw = 3, 3
    so, si, sq = wl.csr_from_edges(n_ops, [0, 1], [1, 2], [1, 65536])
    counts = [5, 7, 4]
    cfg_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    n = int(cfg_off[-1])
    hw = rng.integers(0, n_hw, n).astype(np.int32)
    hw[cfg_off[:-1]] = 0
    batch = rng.choice([1, 2, 65536], n).astype(np.int32)
    batch[cfg_off[:-1]] = 1
    lat = rng.choice([1, 2, 2**31 - 1, 2**30, 99_999], n).astype(np.int32)
    cost = rng.choice([0, 1, 2**40, 2**40 - 1, 12345], n).astype(np.int64)
    inv_op = np.tile(np.arange(n_ops), 50).astype(np.int32)
    slo = rng.choice([0, 1, 2**31 - 1, 10**7], len(inv_op)).astype(np.int32)
    el = np.minimum(rng.choice([0, 1, 2**31 - 1, 5 * 10**6], len(inv_op)), slo).astype(np.int32)
    w = wl.Workload("extreme", n_hw, np.array([0, n_ops], np.int32), so, si, sq, cfg_off, hw,
                    batch, np.ones(n, np.int32), lat, cost, inv_op, el, slo)
    for Q in (None, [0, 2**40, 7], [-5, 0, 2**62]):
        assert_full_parity(Run(w), Q=Q)


def test_max_configs_per_op():
    # one op with 65,535 configurations (the packed-index limit)
    rng = np.random.default_rng(4)
    n = 65535
    so, si, sq = wl.csr_from_edges(2, [0], [1])
    cfg_off = np.array([0, n, n + 3], np.int32)
    hw = rng.integers(0, 4, n + 3).astype(np.int32)
    hw[[0, n]] = 0
    batch = rng.integers(1, 65, n + 3).astype(np.int32)
    batch[[0, n]] = 1
    lat = rng.integers(1, 10**6, n + 3).astype(np.int32)
    cost = rng.integers(0, 10**6, n + 3).astype(np.int64)
    inv_op = rng.integers(0, 2, 3000).astype(np.int32)
    slo = rng.integers(0, 10**7, 3000).astype(np.int32)
    el = (slo * rng.random(3000)).astype(np.int32)
    w = wl.Workload("maxcfg", 4, np.array([0, 2], np.int32), so, si, sq, cfg_off, hw, batch,
                    np.ones(n + 3, np.int32), lat, cost, inv_op, el, slo)
    assert_full_parity(Run(w))


def test_update_latencies_recomputes_everything():
    w = wl.make_c2(seed=8, n_pipelines=6, n_inv=4000)
    r = Run(w)
    rng = np.random.default_rng(1)
    lat2 = np.maximum(1, (w.lat * rng.uniform(0.5, 1.5, w.n_cfg))).astype(np.int32)
    r.L.update_latencies(lat2)
    w2 = wl.Workload(**{**w.__dict__, "lat": lat2})
    r.w, r.P = w2, oracle.Problem(w2)
    assert_full_parity(r)


@pytest.mark.parametrize("maker", ["c1", "c2", "c3", "c3w", "c3m"])
def test_full_scan_schedule_classes(maker):
    # every crossover of the full scan's schedule table (pure lanes =
    # configurations, pure lanes = invocations, mixed) and the autotuned one
    # decide bit-exactly like the oracle, with and without queueing times;
    # c1 has 8 configurations per op (16-lane groups), c2 64-512, c3 16-256
    # with up to ~300 invocations per op, c3w up to 2,048 (backend runs of up
    # to 512 configurations: one or two register pieces of every slot count;
    # test_max_configs_per_op has runs of ~16 K, 64 pieces); c3m has more ops
    # than one LDS histogram holds,
    # so its invocations are bucketed in two levels (groups of ops, then ops)
    w = {"c1": lambda: wl.make_c1(queue=True),
         "c2": lambda: wl.make_c2(seed=15, n_pipelines=24, n_inv=40_000),
         "c3": lambda: wl.make_c3(seed=16, n_pipelines=96, n_inv=60_000, max_cfg=256),
         "c3w": lambda: wl.make_c3(seed=17, n_pipelines=48, n_inv=30_000, max_cfg=2048),
         "c3m": lambda: wl.make_c3(seed=18, n_pipelines=320, n_inv=90_000, max_cfg=256)}[maker]()
    r = Run(w)
    Q = [700, 0, 25_000, 3][:w.n_hw]
    for mode in (PAPER, PROB):
        c_or, f_or = r.P.decide(mode)
        cq_or, fq_or = r.P.decide(mode, Q=Q)
        for num, den in ((0, 1), (1 << 20, 1), (1, 1), (1, 4), (4, 1)):
            r.L.set_full_schedule(num, den)
            c, f = r.decide(mode, B.SCAN_FULL)
            assert np.array_equal(c, c_or) and np.array_equal(f, f_or), (num, den)
            c, f = r.decide(mode, B.SCAN_FULL, Q)
            assert np.array_equal(c, cq_or) and np.array_equal(f, fq_or), (num, den)
        (num, den), us = r.L.autotune_full(r.op, r.el, r.slo, mode)
        say(f"{maker} mode {mode}: full-scan crossover {num}/{den}, {us:.1f} us")
        c, f = r.decide(mode, B.SCAN_FULL)
        assert np.array_equal(c, c_or) and np.array_equal(f, f_or)
    with pytest.raises(B.LlamaError):
        r.L.set_full_schedule(1, 0)


@pytest.mark.parametrize("maker", ["c2", "c3"])
def test_relax_one_slack_mode(maker):
    # records rebuilt for one slack mode: that mode stays bit-exact, the
    # record-reading path refuses the other, the paths that read W directly
    # serve both; a full relaxation restores both
    w = (wl.make_c2(seed=13, n_pipelines=24, n_inv=30_000) if maker == "c2"
         else wl.make_c3(seed=14, n_pipelines=48, n_inv=30_000))
    r = Run(w)
    rng = np.random.default_rng(2)
    lat2 = np.maximum(1, (w.lat * rng.uniform(0.6, 1.4, w.n_cfg))).astype(np.int32)
    r.L.update_latencies(lat2)
    w2 = wl.Workload(**{**w.__dict__, "lat": lat2})
    r.w, r.P = w2, oracle.Problem(w2)
    for keep, drop in ((PAPER, PROB), (PROB, PAPER), (PAPER, PROB)):
        r.L.relax(modes=1 << keep)
        c, f = r.decide(keep, B.SCAN_INDEXED)
        c_or, f_or = r.P.decide(keep)
        assert np.array_equal(c, c_or) and np.array_equal(f, f_or)
        with pytest.raises(B.LlamaError, match="slack mode"):
            r.decide(drop, B.SCAN_INDEXED)
        c, f = r.decide(drop, B.SCAN_WAVE)
        c_or, f_or = r.P.decide(drop)
        assert np.array_equal(c, c_or) and np.array_equal(f, f_or)
        c, f = r.decide(drop, B.SCAN_INDEXED, Q=[10, 0, 300, 7])   # per-call records
        c_or, f_or = r.P.decide(drop, Q=[10, 0, 300, 7])
        assert np.array_equal(c, c_or) and np.array_equal(f, f_or)
    with pytest.raises(B.LlamaError):
        r.L.relax(modes=4)
    r.L.relax()
    assert_full_parity(r, scans=(B.SCAN_INDEXED,))


def test_repeatable_and_order_independent():
    torch = _torch()
    w = wl.make_c2(seed=9, n_pipelines=10, n_inv=30_000)
    r = Run(w)
    c0, f0 = r.decide(PAPER, B.SCAN_INDEXED)
    for _ in range(3):
        c, f = r.decide(PAPER, B.SCAN_INDEXED)
        assert np.array_equal(c, c0) and np.array_equal(f, f0)
    perm = np.random.default_rng(0).permutation(w.n_inv)
    rp = Run(w.with_invocations(w.inv_op[perm], w.elapsed[perm], w.slo[perm]))
    for scan in B.SCANS:
        cp, fp = rp.decide(PAPER, scan)
        assert np.array_equal(cp, c0[perm]) and np.array_equal(fp, f0[perm])
    # growing and pre-sized full-scan scratch give the same answers
    rp.L.reserve(10)
    rp.L.reserve(w.n_inv * 2)
    cp, fp = rp.decide(PAPER, B.SCAN_FULL)
    assert np.array_equal(cp, c0[perm]) and np.array_equal(fp, f0[perm])


def test_ingest_errors():
    _torch()
    L = B.Llama(0)
    with pytest.raises(B.LlamaError) as e:
        L.set_profiles(1, [0, 1], [0], [1], [1], [5], [1])
    assert e.value.rc == B.E_STATE
    with pytest.raises(B.LlamaError) as e:
        L.set_dag([0, 3], [0, 1, 2, 3], [1, 2, 0])
    assert e.value.rc == B.E_CYCLE
    with pytest.raises(B.LlamaError) as e:
        L.set_dag([0, 2], [0, 1, 1], [1], [0])
    assert e.value.rc == B.E_RANGE
    with pytest.raises(B.LlamaError) as e:
        L.set_dag([0, 1, 2], [0, 1, 1], [1])  # edge crosses pipelines
    assert e.value.rc == B.E_RANGE
    L.set_dag([0, 2], [0, 1, 1], [1])
    with pytest.raises(B.LlamaError) as e:  # no hw-0 batch-1 configuration for op 1
        L.set_profiles(2, [0, 1, 2], [0, 1], [1, 1], [1, 1], [5, 5], [1, 1])
    assert e.value.rc == B.E_STATE
    with pytest.raises(B.LlamaError) as e:
        L.set_profiles(2, [0, 1, 2], [0, 0], [1, 1], [1, 1], [0, 5], [1, 1])
    assert e.value.rc == B.E_RANGE
    with pytest.raises(B.LlamaError) as e:
        L.set_profiles(2, [0, 1, 2], [0, 0], [1, 1], [1, 1], [5, 5], [1, 2**41])
    assert e.value.rc == B.E_RANGE
    with pytest.raises(B.LlamaError) as e:
        L.set_profiles(9, [0, 1, 2], [0, 0], [1, 1], [1, 1], [5, 5], [1, 1])
    assert e.value.rc == B.E_RANGE
    L.set_profiles(2, [0, 1, 2], [0, 0], [1, 1], [1, 1], [5, 5], [1, 1])
    import torch
    op = torch.zeros(4, dtype=torch.int32, device="cuda")
    with pytest.raises(B.LlamaError) as e:
        L.decide(op, op, op, mode=7)
    assert e.value.rc == B.E_ARG


def test_select_rows_matches_oracle():
    torch = _torch()
    rng = np.random.default_rng(17)
    for w in (wl.make_c2(seed=10, n_pipelines=6, n_inv=3001), wl.make_c1(n_inv=777)):
        r = Run(w)
        stride = int(np.diff(w.cfg_off).max()) + 3
        lat = rng.integers(1, 400_000, (w.n_inv, stride)).astype(np.int32)
        lat[:, :5] = rng.integers(1, 3, (w.n_inv, 5))  # ties among the fastest
        t = r.P.targets(PAPER)
        c_or, f_or = oracle.select_lat(w.inv_op, t, w.n_hw, w.cfg_off, w.hw, w.batch, lat, w.cost)
        c, f = r.L.select_rows(r.op, dev(t, torch), dev(lat, torch))
        torch.cuda.synchronize()
        assert np.array_equal(c.cpu().numpy(), c_or) and np.array_equal(f.cpu().numpy(), f_or)


def test_c3_reduced():
    # uneven pipelines (3-200 ops) and tables (16-2048 configurations per op)
    w = wl.make_c3(seed=12, n_pipelines=64, n_inv=40_001)
    assert_full_parity(Run(w), modes=(PAPER,))


def test_c3_full_size_sampled():
    # 4,096 pipelines, ~80M configurations, 4M invocations, decided in one call
    # per slack mode; the oracle checks a 200,000-invocation sample of each call
    torch = _torch()
    w = wl.make_c3()
    say(f"c3: {w.n_ops} ops, {w.n_cfg} configurations, {w.n_inv} invocations")
    L = B.Llama(0).load(w)
    op, el, slo = dev(w.inv_op, torch), dev(w.elapsed, torch), dev(w.slo, torch)
    idx = np.sort(np.random.default_rng(0).choice(w.n_inv, 200_000, replace=False))
    ws = w.with_invocations(w.inv_op[idx], w.elapsed[idx], w.slo[idx])
    P = oracle.Problem(ws)
    for mode in (PAPER, PROB):
        c_or, f_or = P.decide(mode)
        # the indexed decision, the full scan (two-level bucketing, both
        # schedule layouts) and the wave scan
        for scan in (B.SCAN_AUTO, B.SCAN_FULL, B.SCAN_WAVE):
            c, f = L.decide(op, el, slo, mode=mode, scan=scan)
            torch.cuda.synchronize()
            c, f = c.cpu().numpy(), f.cpu().numpy()
            assert np.array_equal(c[idx], c_or) and np.array_equal(f[idx], f_or), (mode, scan)


def test_full_scan_beyond_packed_indices():
    # more than 2^24 invocations over more ops than one LDS histogram holds:
    # the full scan buckets with global atomics instead of the two-level
    # sort (whose entries pack a 24-bit index); the oracle checks a sample
    torch = _torch()
    w = wl.make_c3(seed=19, n_pipelines=320, n_inv=(1 << 24) + 4096, max_cfg=64)
    L = B.Llama(0).load(w)
    op, el, slo = dev(w.inv_op, torch), dev(w.elapsed, torch), dev(w.slo, torch)
    idx = np.sort(np.random.default_rng(1).choice(w.n_inv, 50_000, replace=False))
    idx[-1] = w.n_inv - 1
    ws = w.with_invocations(w.inv_op[idx], w.elapsed[idx], w.slo[idx])
    c_or, f_or = oracle.Problem(ws).decide(PAPER)
    c, f = L.decide(op, el, slo, mode=PAPER, scan=B.SCAN_FULL)
    torch.cuda.synchronize()
    c, f = c.cpu().numpy(), f.cpu().numpy()
    assert np.array_equal(c[idx], c_or) and np.array_equal(f[idx], f_or)


@pytest.mark.parametrize("maker", ["c2", "c3"])
def test_autotuned_schedules_agree_with_oracle(maker):
    # llama_autotune runs every schedule of the indexed decision (1, 2, 4
    # invocations per thread with plain or non-temporal input loads, and the
    # LDS-staged persistent variant when the ops fit) and fails if any two
    # disagree; the chosen one is then checked
    # against the oracle, so all of them are.
    torch = _torch()
    w = (wl.make_c2(seed=31, n_pipelines=40, n_inv=100_003) if maker == "c2"
         else wl.make_c3(seed=32, n_pipelines=48, n_inv=50_001))
    r = Run(w)
    sched, us = r.L.autotune(r.op, r.el, r.slo)
    say(f"{maker}: autotuned schedule {sched} ({us:.2f} us)")
    c, f = r.decide(PAPER, B.SCAN_INDEXED)
    c_or, f_or = r.P.decide(PAPER)
    assert np.array_equal(c, c_or) and np.array_equal(f, f_or)


def test_pinned_schedules_agree_with_oracle():
    # llama_set_schedule pins each schedule in turn; every one must give the
    # oracle's decisions in both slack modes, flags included, on a batch with
    # a ragged tail and invalid invocations
    torch = _torch()
    w = wl.make_c2(seed=33, n_pipelines=30, n_inv=70_001)
    r = Run(w)
    for mode in (PAPER, PROB):
        c_or, f_or = r.P.decide(mode)
        for sched in range(len(B.SCHEDULE_NAMES)):
            r.L.set_schedule(sched)
            c, f = r.decide(mode, B.SCAN_INDEXED)
            assert np.array_equal(c, c_or) and np.array_equal(f, f_or), (mode, B.SCHEDULE_NAMES[sched])
    c_or, f_or = r.P.decide(PAPER)
    op = w.inv_op.copy()
    op[5::97] = -1
    for sched in range(len(B.SCHEDULE_NAMES)):
        r.L.set_schedule(sched)
        c, f = r.L.decide(dev(op, torch), r.el, r.slo, scan=B.SCAN_INDEXED)
        torch.cuda.synchronize()
        c, f = c.cpu().numpy(), f.cpu().numpy()
        assert (c[5::97] == -1).all() and (f[5::97] == 0).all()
        ok = np.ones(len(op), bool)
        ok[5::97] = False
        assert np.array_equal(c[ok], c_or[ok]) and np.array_equal(f[ok], f_or[ok])
        assert r.L.stats(reset_error=True)["device_error"] & B.DEVERR_INVALID_INVOCATION
    for bad in (-1, len(B.SCHEDULE_NAMES)):
        with pytest.raises(B.LlamaError):
            r.L.set_schedule(bad)


def test_lds_schedule_on_unaligned_arrays():
    # the LDS-staged schedule reads four invocations per 16-byte load only
    # when every array is aligned; views that start one element in take its
    # one-invocation-per-load form, which must give the same decisions
    torch = _torch()
    w = wl.make_c2(seed=34, n_pipelines=25, n_inv=50_003)
    r = Run(w)
    r.L.set_schedule(B.SCHEDULE_NAMES.index("lds-persistent"))
    n = w.n_inv

    def shifted(a):
        buf = torch.empty(len(a) + 1, dtype=torch.int32, device="cuda")
        buf[1:] = dev(a, torch)
        return buf[1:]

    op, el, slo = shifted(w.inv_op), shifted(w.elapsed), shifted(w.slo)
    cfg_buf = torch.full((n + 1,), -9, dtype=torch.int32, device="cuda")
    flag_buf = torch.full((n + 3,), 7, dtype=torch.uint8, device="cuda")
    cfg, flag = cfg_buf[1:], flag_buf[3:]
    assert op.data_ptr() % 16 != 0 and cfg.data_ptr() % 16 != 0 and flag.data_ptr() % 4 != 0
    for mode in (PAPER, PROB):
        r.L.decide(op, el, slo, None, mode, B.SCAN_INDEXED, cfg, flag)
        torch.cuda.synchronize()
        c_or, f_or = r.P.decide(mode)
        assert np.array_equal(cfg.cpu().numpy(), c_or) and np.array_equal(flag.cpu().numpy(), f_or), mode
    assert cfg_buf[0].item() == -9 and (flag_buf[:3].cpu().numpy() == 7).all()
