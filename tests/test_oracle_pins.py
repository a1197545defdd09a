"""Pins for the CPU oracle (no GPU).

The oracle is checked against things other than itself:
  * a worked example derived by hand from Alg. 1 and Eq. 1 (tests/golden);
  * closed forms: a single op gets the whole remaining time, a chain of n
    equal-reference ops gives floor(R/n), a symmetric fork equals one branch,
    PROB mode with every q = 65536 equals PAPER mode;
  * literal path enumeration with exact rationals (tests/brute.py) on every
    DAG over 5 labelled vertices whose edges go from lower to higher index
    (all 2^10 edge sets), and on random DAGs of up to 8 ops;
  * invariants I1-I7 on the tiny and scaled synthetic workloads.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import brute
import oracle
from paper_2102_01887_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")
PAPER, PROB = oracle.PAPER, oracle.PROB


def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def golden_workload(g):
    s, t = g["tables"], g["succ"]
    succ_off, succ_ids, succ_q16 = wl.csr_from_edges(4, s_src := t["src"], t["dst"], t["q16"])
    inv = g["invocations"]
    return wl.Workload(
        name="worked", n_hw=g["n_hw"], pipe_off=np.array([0, 4], np.int32),
        succ_off=succ_off, succ_ids=succ_ids, succ_q16=succ_q16,
        cfg_off=np.array(s["cfg_off"], np.int32), hw=np.array(s["hw"], np.int32),
        batch=np.array(s["batch"], np.int32), res=np.array(s["res"], np.int32),
        lat=np.array(s["lat"], np.int32), cost=np.array(s["cost"], np.int64),
        inv_op=np.array([i["op"] for i in inv], np.int32),
        elapsed=np.array([i["elapsed"] for i in inv], np.int32),
        slo=np.array([i["slo"] for i in inv], np.int32))


# ---------------------------------------------------------------------------
# worked example
# ---------------------------------------------------------------------------

def test_worked_example_relaxation_and_targets():
    g = golden()
    w = golden_workload(g)
    P = oracle.Problem(w)
    assert P.ref.tolist() == g["ref"]
    assert P.W(PAPER).tolist() == g["W"]["paper"]
    assert P.W(PROB).tolist() == g["W"]["prob"]
    tp, tq = P.targets(PAPER), P.targets(PROB)
    for i, inv in enumerate(g["invocations"]):
        assert tp[i].tolist() == [inv["target_paper"]] * 2
        assert tq[i].tolist() == [inv["target_prob"]] * 2
    cfg, flag = P.decide(PAPER)
    assert cfg[0] == g["invocations"][0]["cfg_paper"] and flag[0] == 1


def test_worked_example_select():
    g = golden()
    w = golden_workload(g)
    cases = g["select_op1"]
    n = len(cases)
    tgt = np.array([[c["target"]] * 2 for c in cases], np.int32)
    cfg, flag = oracle.select(np.ones(n, np.int32), tgt, 2, w.cfg_off, w.hw, w.batch,
                              w.lat, w.cost)
    assert cfg.tolist() == [c["cfg"] for c in cases]
    assert flag.tolist() == [c["flag"] for c in cases]


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------

def chain_workload(refs, R_list, q=None):
    n = len(refs)
    src, dst = list(range(n - 1)), list(range(1, n))
    succ_off, succ_ids, succ_q16 = wl.csr_from_edges(n, src, dst, q)
    cfg_off = np.arange(n + 1, dtype=np.int32)
    ones = np.ones(n, np.int32)
    inv_op = np.repeat(np.arange(n), len(R_list)).astype(np.int32)
    slo = np.tile(np.asarray(R_list, np.int32), n)
    return wl.Workload("chain", 1, np.array([0, n], np.int32), succ_off, succ_ids, succ_q16,
                       cfg_off, np.zeros(n, np.int32), ones, ones,
                       np.asarray(refs, np.int32), np.ones(n, np.int64),
                       inv_op, np.zeros_like(slo), slo)


@pytest.mark.parametrize("mode", [PAPER, PROB])
def test_single_op_gets_whole_remaining_time(mode):
    w = chain_workload([777], [0, 1, 999, 10**7, 2**31 - 1])
    assert oracle.Problem(w).targets(mode)[:, 0].tolist() == [0, 1, 999, 10**7, 2**31 - 1]


@pytest.mark.parametrize("n", [2, 3, 7])
def test_equal_reference_chain(n):
    Rs = [0, 1, 5, 1000, 999_983, 2**31 - 1]
    w = chain_workload([123] * n, Rs)
    t = oracle.Problem(w).targets(PAPER)[:, 0].reshape(n, len(Rs))
    for pos in range(n):
        assert t[pos].tolist() == [R // (n - pos) for R in Rs]


def test_prob_chain_closed_form():
    # chain a -> b with q: W_a = ref_a + floor(q * ref_b / 65536)
    refs, q = [300, 500], 19661
    w = chain_workload(refs, [10_000], q=[q])
    P = oracle.Problem(w)
    Wa = 300 + (q * 500) // 65536
    assert P.W(PROB).tolist() == [Wa, 500]
    assert P.targets(PROB)[0, 0] == (300 * 10_000) // Wa


def test_symmetric_fork_equals_one_branch():
    # 0 -> {1, 2} with equal references equals the chain 0 -> 1
    succ_off, succ_ids, succ_q16 = wl.csr_from_edges(3, [0, 0], [1, 2])
    refs = np.array([40, 70, 70], np.int32)
    Rs = np.array([0, 17, 1000, 123_457], np.int32)
    fork = wl.Workload("fork", 1, np.array([0, 3], np.int32), succ_off, succ_ids, succ_q16,
                       np.arange(4, dtype=np.int32), np.zeros(3, np.int32), np.ones(3, np.int32),
                       np.ones(3, np.int32), refs, np.ones(3, np.int64),
                       np.zeros(len(Rs), np.int32), np.zeros(len(Rs), np.int32), Rs)
    chain = chain_workload([40, 70], Rs.tolist())
    a = oracle.Problem(fork).targets(PAPER)[:, 0]
    b = oracle.Problem(chain).targets(PAPER)[: len(Rs), 0]
    assert a.tolist() == b.tolist() == [int(R) * 40 // 110 for R in Rs]


def test_prob_equals_paper_when_branches_certain():
    rng = np.random.default_rng(7)
    for _ in range(50):
        w = wl.random_small(rng, q_choices=[65536])
        P = oracle.Problem(w)
        assert P.W(PROB).tolist() == P.W(PAPER).tolist()
        assert np.array_equal(P.targets(PROB), P.targets(PAPER))


# ---------------------------------------------------------------------------
# brute force: every 5-vertex DAG, random DAGs up to 8 ops
# ---------------------------------------------------------------------------

def _brute_targets(w, mode, Q=None):
    tg, _, _ = brute.decide_all(w, prob=(mode == PROB), Q=Q)
    return np.array(tg, np.int64)


def test_all_five_op_dags_against_path_enumeration():
    rng = np.random.default_rng(11)
    n = 5
    Rs = np.array([0, 1, 7, 100, 4321, 99_991, 2**31 - 1], np.int32)
    for mask in range(1 << 10):
        src, dst = wl.dag_from_mask(n, mask)
        for draw in range(2):
            refs = rng.integers(1, 1000 if draw else 5, n)
            q = rng.integers(1, 65537, len(src))
            succ_off, succ_ids, succ_q16 = wl.csr_from_edges(n, src, dst, q)
            inv_op = np.repeat(np.arange(n), len(Rs)).astype(np.int32)
            slo = np.tile(Rs, n)
            w = wl.Workload("dag5", 1, np.array([0, n], np.int32), succ_off, succ_ids,
                            succ_q16, np.arange(n + 1, dtype=np.int32), np.zeros(n, np.int32),
                            np.ones(n, np.int32), np.ones(n, np.int32),
                            refs.astype(np.int32), np.ones(n, np.int64), inv_op,
                            np.zeros_like(slo), slo)
            P = oracle.Problem(w)
            for mode in (PAPER, PROB):
                got = P.targets(mode)[:, 0]
                want = _brute_targets(w, mode)[:, 0]
                assert got.tolist() == want.tolist(), (mask, draw, mode)


def test_random_dags_full_decision_against_brute_force():
    rng = np.random.default_rng(12)
    for it in range(300):
        w = wl.random_small(rng, n_inv=40)
        Q = rng.integers(0, 3000, w.n_hw) if it % 2 else None
        P = oracle.Problem(w)
        for mode in (PAPER, PROB):
            tg, cf, fl = brute.decide_all(w, prob=(mode == PROB), Q=Q)
            t = P.targets(mode, Q=Q)
            assert t.tolist() == tg, it
            cfg, flag = P.decide(mode, Q=Q)
            assert cfg.tolist() == cf, it
            assert flag.tolist() == fl, it


def test_select_against_exact_rationals_with_many_ties():
    rng = np.random.default_rng(13)
    for it in range(200):
        n_hw = int(rng.integers(1, 4))
        cfg_off, hw, batch, res, lat, cost = wl.random_table(
            rng, 3, n_hw, cfg_lo=1, cfg_hi=12, lat_hi=8, cost_hi=6, batch_hi=3)
        n_inv = 64
        inv_op = rng.integers(0, 3, n_inv).astype(np.int32)
        tgt = rng.integers(-2, 10, (n_inv, n_hw)).astype(np.int32)
        cfg, flag = oracle.select(inv_op, tgt, n_hw, cfg_off, hw, batch, lat, cost)
        for i in range(n_inv):
            k, f = brute.select(int(inv_op[i]), tgt[i], cfg_off, hw, batch, lat, cost)
            assert (cfg[i], flag[i]) == (k, f), (it, i)


def test_reference_rule():
    # hw 0 batch 1 with the smallest resource size; lowest index on a tie
    cfg_off = np.array([0, 5, 8], np.int32)
    hw = np.array([1, 0, 0, 0, 0, 0, 0, 1], np.int32)
    batch = np.array([1, 2, 1, 1, 1, 1, 1, 1], np.int32)
    res = np.array([1, 1, 4, 2, 2, 3, 3, 1], np.int32)
    assert oracle.reference_cfg(cfg_off, hw, batch, res).tolist() == [3, 0]
    with pytest.raises(oracle.OracleError) as e:
        oracle.reference_cfg(np.array([0, 2], np.int32), np.array([1, 0], np.int32),
                             np.array([1, 2], np.int32), np.array([1, 1], np.int32))
    assert e.value.rc == oracle.E_STATE


def test_cycle_is_rejected():
    succ_off, succ_ids, q = wl.csr_from_edges(3, [0, 1, 2], [1, 2, 0])
    with pytest.raises(oracle.OracleError) as e:
        oracle.worst_path(succ_off, succ_ids, q, np.array([1, 2, 3], np.int64), PAPER)
    assert e.value.rc == oracle.E_CYCLE


def test_invalid_invocations():
    w = wl.make_c1()
    P = oracle.Problem(w)
    inv_op = np.array([-1, 6, 2, 2, 2], np.int32)
    elapsed = np.array([0, 0, -5, 0, 10], np.int32)
    slo = np.array([10, 10, 10, -1, 5], np.int32)
    cfg, flag = oracle.decide(inv_op, elapsed, slo, 2, None, P.ref, P.W(PAPER), w.cfg_off,
                              w.hw, w.batch, w.lat, w.cost)
    assert cfg[:4].tolist() == [-1, -1, -1, -1]
    assert flag[:4].tolist() == [0, 0, 0, 0]
    # past the deadline: valid, slack 0, fallback to the fastest
    assert flag[4] == 0 and cfg[4] == int(np.argmin(w.lat[16:24]))


# ---------------------------------------------------------------------------
# invariants on the synthetic workloads
# ---------------------------------------------------------------------------

def _per_item(cost, batch, x):
    return Fraction(int(cost[x]), int(batch[x]))


@pytest.mark.parametrize("maker", ["c1", "c1q", "c2"])
def test_invariants(maker):
    if maker == "c1":
        w, Q = wl.make_c1(), None
    elif maker == "c1q":
        w = wl.make_c1(queue=True)
        Q = w.Q
    else:
        w = wl.make_c2(n_pipelines=12, n_inv=3000, queue=True)
        Q = w.Q
    P = oracle.Problem(w)
    t_paper = P.targets(PAPER, Q=Q).astype(np.int64)
    t_prob = P.targets(PROB, Q=Q).astype(np.int64)
    cfg, flag = P.decide(PAPER, Q=Q)
    Qv = np.zeros(w.n_hw, np.int64) if Q is None else np.asarray(Q, np.int64)
    R = np.clip(w.slo[:, None].astype(np.int64) - w.elapsed[:, None] - Qv[None, :], 0, 2**31 - 1)
    # I4: 0 <= target <= R ; I7: PROB >= PAPER
    assert (t_paper >= 0).all() and (t_paper <= R).all()
    assert (t_prob >= t_paper).all() and (t_prob <= R).all()
    # I2: targets times every remaining path's reference sum stay within ref*R
    succ, _ = brute.successors(w.succ_off, w.succ_ids, None)
    W = P.W(PAPER)
    ref = P.ref
    assert (t_paper * W[w.inv_op][:, None] <= ref[w.inv_op][:, None] * R).all()
    # ... and splitting R along the worst path with v's denominator never exceeds R
    split = (ref[w.inv_op][:, None] * R) // W[w.inv_op][:, None]
    assert (split <= R).all()
    # I1, I3 on a sample
    idx = np.random.default_rng(0).choice(w.n_inv, min(w.n_inv, 600), replace=False)
    for i in idx:
        v = int(w.inv_op[i])
        a, b = int(w.cfg_off[v]), int(w.cfg_off[v + 1])
        feas = [x for x in range(a, b) if w.lat[x] < t_paper[i, w.hw[x]]]
        x = a + int(cfg[i])
        assert flag[i] == (1 if feas else 0)
        if feas:
            assert x in feas
            assert all(_per_item(w.cost, w.batch, x) <= _per_item(w.cost, w.batch, y) for y in feas)
        else:
            assert all(w.lat[x] <= w.lat[y] for y in range(a, b))
    # I4 monotonicity: more elapsed time never raises the target
    w2 = w.with_invocations(w.inv_op, np.minimum(w.elapsed.astype(np.int64) + 1000, 2**31 - 1), w.slo)
    t2 = oracle.Problem(w2).targets(PAPER, Q=Q)
    assert (t2 <= t_paper).all()


def test_relabelling_ops_leaves_targets_unchanged():
    rng = np.random.default_rng(21)
    for _ in range(40):
        w = wl.random_small(rng, n_inv=30)
        n = w.n_ops
        perm = rng.permutation(n)          # new id of old op v is perm[v]
        inv = np.argsort(perm)
        src = np.repeat(np.arange(n), np.diff(w.succ_off))
        so, si, sq = wl.csr_from_edges(n, perm[src], perm[w.succ_ids], w.succ_q16)
        counts = np.diff(w.cfg_off)[inv]
        cfg_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
        take = np.concatenate([np.arange(w.cfg_off[v], w.cfg_off[v + 1]) for v in inv]).astype(np.int64)
        w2 = wl.Workload("relabel", w.n_hw, w.pipe_off, so, si, sq, cfg_off, w.hw[take],
                         w.batch[take], w.res[take], w.lat[take], w.cost[take],
                         perm[w.inv_op].astype(np.int32), w.elapsed, w.slo)
        for mode in (PAPER, PROB):
            assert np.array_equal(oracle.Problem(w).targets(mode), oracle.Problem(w2).targets(mode))


def test_parallel_decide_equals_single_threaded():
    """The host-threaded oracle leg (used to time the oracle on every host
    core) returns exactly the single-threaded decisions."""
    w = wl.make_c2(seed=5, n_pipelines=8, n_inv=20_001)
    P = oracle.Problem(w)
    for mode in (oracle.PAPER, oracle.PROB):
        c1, f1 = P.decide(mode)
        c4, f4 = P.decide_parallel(mode, 4)
        assert np.array_equal(c1, c4) and np.array_equal(f1, f4)
