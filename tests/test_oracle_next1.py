"""Pins for the oracle's Eq. 2 queueing time and finite-alpha Eq. 1 (CPU only).

Eq. 2 (Sec. 4.3): Q[h] = floor(sum over queued i on h of L(x_i) * R(x_i) / R_total(h)).
Pinned by closed forms (an empty queue; n identical entries; values whose sum
passes 2^64, where any 64-bit or floating-point accumulation is wrong), by
separability across backends with different R_total, by permutation
invariance, and by the cap at 2^62.

Finite-alpha Eq. 1 (Sec. 4.2): obj = C/B if L < slack, else
C/B + alpha * L * R / (B * R_total).  Pinned by:
  * a hand-worked example (below, derived in the comments);
  * brute force with Python's exact Fractions on small random tables, evaluating
    the two-term form of Eq. 1 directly (the oracle instead compares single
    combined fractions with 256-bit products);
  * closed forms: alpha = 0 gives the cheapest C/B over every configuration;
    all configurations feasible gives the plain Eq. 1 choice; zero costs with
    nothing feasible give the smallest L * R / (B * R_total);
  * large magnitudes (costs near 2^40, R_total near 2^40, alpha near 2^32),
    where products exceed 2^128, against Fractions.
Planted mistakes in the new oracle functions must each fail a pin.
"""
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import oracle


def table(rng, n_ops=3, n_hw=2, cfg_hi=7, lat_hi=40, cost_hi=30, res_hi=4, batch_hi=4):
    counts = rng.integers(1, cfg_hi + 1, n_ops)
    cfg_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    n = int(cfg_off[-1])
    return dict(cfg_off=cfg_off,
                hw=rng.integers(0, n_hw, n).astype(np.int32),
                batch=rng.integers(1, batch_hi + 1, n).astype(np.int32),
                res=rng.integers(1, res_hi + 1, n).astype(np.int32),
                lat=rng.integers(1, lat_hi + 1, n).astype(np.int32),
                cost=rng.integers(0, cost_hi + 1, n).astype(np.int64))


# ---------------------------------------------------------------------------
# Eq. 2
# ---------------------------------------------------------------------------

def qt(t, q_op, q_cfg, n_hw, r_total):
    return oracle.queue_time(q_op, q_cfg, n_hw, t["cfg_off"], t["hw"], t["res"], t["lat"], r_total)


def test_queue_time_empty_is_zero():
    t = table(np.random.default_rng(0))
    Q, skipped = qt(t, [], [], 2, [5, 7])
    assert Q.tolist() == [0, 0] and skipped == 0


@pytest.mark.parametrize("n,L,R,Rt", [(1, 10, 3, 4), (7, 1000, 8, 3), (5, 2**31 - 1, 2**31 - 1, 1),
                                      (12, 2**31 - 1, 2**30, 3)])
def test_queue_time_identical_entries_closed_form(n, L, R, Rt):
    # one op with a single configuration on backend 1: Q[1] = floor(n*L*R/Rt)
    t = dict(cfg_off=np.array([0, 1], np.int32), hw=np.array([1], np.int32),
             res=np.array([R], np.int32), lat=np.array([L], np.int32))
    Q, _ = qt(t, [0] * n, [0] * n, 2, [9, Rt])
    want = min(n * L * R // Rt, 2**62)
    assert Q.tolist() == [0, want]
    if n * L * R >= 2**64:
        # a 64-bit accumulator would have wrapped; double rounding would be inexact
        assert want != (n * L * R % 2**64) // Rt


def test_queue_time_cap():
    t = dict(cfg_off=np.array([0, 1], np.int32), hw=np.array([0], np.int32),
             res=np.array([2**31 - 1], np.int32), lat=np.array([2**31 - 1], np.int32))
    Q, _ = qt(t, [0] * 4, [0] * 4, 1, [1])
    assert Q.tolist() == [2**62]


def test_queue_time_separable_and_permutation_invariant():
    rng = np.random.default_rng(1)
    t = table(rng, n_ops=5, n_hw=3)
    n_q = 200
    q_op = rng.integers(0, 5, n_q)
    q_cfg = np.array([rng.integers(0, t["cfg_off"][v + 1] - t["cfg_off"][v]) for v in q_op])
    r_total = np.array([3, 5, 11])
    Q, skipped = qt(t, q_op, q_cfg, 3, r_total)
    assert skipped == 0
    perm = rng.permutation(n_q)
    assert np.array_equal(qt(t, q_op[perm], q_cfg[perm], 3, r_total)[0], Q)
    # each backend only sees its own entries: dropping every entry of backend
    # 0 leaves Q[1] and Q[2] unchanged and makes Q[0] zero
    x = t["cfg_off"][q_op] + q_cfg
    keep = t["hw"][x] != 0
    Q2, _ = qt(t, q_op[keep], q_cfg[keep], 3, r_total)
    assert Q2[0] == 0 and Q2[1] == Q[1] and Q2[2] == Q[2]
    # per backend the result is the single-backend closed form of its entries:
    # floor(total / R_total[h]) with total the exact integer sum
    for h in range(3):
        sel = t["hw"][x] == h
        tot = sum(int(t["lat"][j]) * int(t["res"][j]) for j in x[sel])
        assert Q[h] == tot // int(r_total[h])


def test_queue_time_skips_out_of_range_entries():
    t = table(np.random.default_rng(2), n_ops=2)
    n0 = int(t["cfg_off"][1])
    Q, skipped = qt(t, [0, 0, 5, -1, 1], [0, n0, 0, 0, 0], 2, [1, 1])
    want, _ = qt(t, [0, 1], [0, 0], 2, [1, 1])
    assert skipped == 3 and np.array_equal(Q, want)


# ---------------------------------------------------------------------------
# finite-alpha Eq. 1
# ---------------------------------------------------------------------------

def sel_alpha(t, inv_op, target, n_hw, r_total, a_num, a_den):
    return oracle.select_alpha(inv_op, target, n_hw, t["cfg_off"], t["hw"], t["batch"], t["res"],
                               t["lat"], t["cost"], r_total, a_num, a_den)


def brute_alpha(t, inv_op, target, r_total, a_num, a_den):
    """Eq. 1 as printed: C/B, plus alpha*L*R/(B*R_total) when the slack is missed."""
    alpha = Fraction(a_num, a_den)
    cfg, flag = [], []
    for i, v in enumerate(inv_op):
        a, b = int(t["cfg_off"][v]), int(t["cfg_off"][v + 1])
        best = None
        for x in range(a, b):
            h = int(t["hw"][x])
            meets = int(t["lat"][x]) < int(target[i][h])
            obj = Fraction(int(t["cost"][x]), int(t["batch"][x]))
            if not meets:
                obj += alpha * int(t["lat"][x]) * int(t["res"][x]) / (int(t["batch"][x]) * int(r_total[h]))
            if best is None or obj < best[0]:
                best = (obj, x - a, meets)
        cfg.append(best[1])
        flag.append(int(best[2]))
    return np.array(cfg), np.array(flag)


def test_fraction_comparison_over_the_full_128_bit_range():
    # the oracle's 256-bit cross-multiplication against Python integers, on
    # random operands up to 2^128 - 1 (carries between limbs are frequent)
    # and on pairs whose products differ by one
    rng = np.random.default_rng(11)
    top = 2**128 - 1
    for _ in range(3000):
        bits = rng.integers(1, 129, 4)
        n1, d1, n2, d2 = (int(rng.integers(0, 2**63)) * 2**65 % 2**int(b) + int(rng.integers(0, 2**63))
                          for b in bits)
        d1, d2 = d1 or 1, d2 or 1
        assert oracle.fraction_below(n1, d1, n2, d2) == (n1 * d2 < n2 * d1)
    # near ties: n2/d2 just at or above n1/d1, so the two 256-bit products
    # agree in their top limbs and the carries between limbs decide
    for _ in range(2000):
        n1, d1, d2 = (int.from_bytes(rng.bytes(16), "little") or 1 for _ in range(3))
        for delta in (0, 1):
            n2 = n1 * d2 // d1 + delta
            if n2 > top:
                continue
            assert oracle.fraction_below(n1, d1, n2, d2) == (n1 * d2 < n2 * d1)
            assert oracle.fraction_below(n2, d2, n1, d1) == (n2 * d1 < n1 * d2)
    for n1, d1, n2, d2 in ((top, top, top, top), (top - 1, top, top, top), (top, top - 1, top, top),
                           (2**127, 2**127 + 1, 2**127 - 1, 2**127), (2**64 - 1, 2**64 + 1, 2**64, 2**64)):
        assert oracle.fraction_below(n1, d1, n2, d2) == (n1 * d2 < n2 * d1)
        assert oracle.fraction_below(n2, d2, n1, d1) == (n2 * d1 < n1 * d2)


def test_alpha_worked_example():
    # one op, backends 0 and 1, R_total = [4, 8], alpha = 1/2:
    #   x0: hw 0, B 1, R 2, L 10, C 6   -> C/B = 6,   penalty 1/2*10*2/(1*4)  = 5/2
    #   x1: hw 1, B 2, R 4, L 30, C 8   -> C/B = 4,   penalty 1/2*30*4/(2*8)  = 15/4
    #   x2: hw 1, B 1, R 1, L 5,  C 9   -> C/B = 9,   penalty 1/2*5*1/(1*8)   = 5/16
    # targets (40, 40): all feasible -> objs 6, 4, 9 -> x1, flag 1
    # targets (20, 20): x1 misses    -> objs 6, 4 + 15/4 = 31/4, 9 -> x0, flag 1
    # targets (5, 5):   all miss     -> 6 + 5/2 = 17/2, 31/4, 9 + 5/16 -> x1, flag 0
    # targets (11, 5):  x0 meets     -> 6, 31/4, 9 + 5/16 -> x0, flag 1
    # targets (0, 31):  x0 misses, x1 and x2 meet -> 17/2, 4, 9 -> x1, flag 1
    t = dict(cfg_off=np.array([0, 3], np.int32), hw=np.array([0, 1, 1], np.int32),
             batch=np.array([1, 2, 1], np.int32), res=np.array([2, 4, 1], np.int32),
             lat=np.array([10, 30, 5], np.int32), cost=np.array([6, 8, 9], np.int64))
    target = np.array([[40, 40], [20, 20], [5, 5], [11, 5], [0, 31]], np.int32)
    cfg, flag = sel_alpha(t, [0] * 5, target, 2, [4, 8], 1, 2)
    assert cfg.tolist() == [1, 0, 1, 0, 1]
    assert flag.tolist() == [1, 1, 0, 1, 1]
    # a larger alpha (3): all miss -> 6 + 15 = 21, 4 + 22.5 = 26.5, 9 + 15/8 -> x2
    cfg, flag = sel_alpha(t, [0], target[2:3], 2, [4, 8], 3, 1)
    assert cfg.tolist() == [2] and flag.tolist() == [0]


@pytest.mark.parametrize("seed", range(6))
def test_alpha_against_fractions(seed):
    rng = np.random.default_rng(100 + seed)
    n_hw = int(rng.integers(1, 4))
    t = table(rng, n_ops=4, n_hw=n_hw)
    n_inv = 300
    inv_op = rng.integers(0, 4, n_inv)
    target = rng.integers(0, 45, (n_inv, n_hw))
    r_total = rng.integers(1, 9, n_hw)
    for a_num, a_den in ((0, 1), (1, 1), (1, 3), (7, 2), (1000, 1), (3, 1000)):
        got = sel_alpha(t, inv_op, target, n_hw, r_total, a_num, a_den)
        want = brute_alpha(t, inv_op, target, r_total, a_num, a_den)
        assert np.array_equal(got[0], want[0]), (a_num, a_den)
        assert np.array_equal(got[1], want[1]), (a_num, a_den)


def test_alpha_large_magnitudes_against_fractions():
    rng = np.random.default_rng(7)
    n_hw = 3
    t = table(rng, n_ops=3, n_hw=n_hw, cfg_hi=6)
    n = len(t["lat"])
    t["cost"] = rng.integers(2**40 - 1000, 2**40 + 1, n).astype(np.int64)
    t["batch"] = rng.integers(2**16 - 3, 2**16 + 1, n).astype(np.int32)
    t["lat"] = rng.integers(2**31 - 100, 2**31 - 1, n).astype(np.int32)
    t["res"] = rng.integers(2**31 - 100, 2**31 - 1, n).astype(np.int32)
    r_total = np.array([2**40, 2**40 - 1, 2**39 + 5])
    inv_op = rng.integers(0, 3, 200)
    target = np.where(rng.random((200, n_hw)) < 0.5, 0, 2**31 - 1).astype(np.int64)
    for a_num, a_den in ((2**32 - 1, 2**32 - 1), (2**32 - 1, 1), (1, 2**32 - 1), (12345, 67891)):
        got = sel_alpha(t, inv_op, target, n_hw, r_total, a_num, a_den)
        want = brute_alpha(t, inv_op, target, r_total, a_num, a_den)
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), (a_num, a_den)


def test_alpha_zero_is_cheapest_overall():
    rng = np.random.default_rng(3)
    t = table(rng, n_ops=5, n_hw=2, cost_hi=50)
    inv_op = rng.integers(0, 5, 400)
    target = rng.integers(0, 45, (400, 2))
    cfg, flag = sel_alpha(t, inv_op, target, 2, [3, 5], 0, 1)
    for i, v in enumerate(inv_op):
        a, b = t["cfg_off"][v], t["cfg_off"][v + 1]
        per_item = [Fraction(int(t["cost"][x]), int(t["batch"][x])) for x in range(a, b)]
        k = min(range(b - a), key=lambda j: (per_item[j], j))
        assert cfg[i] == k
        x = a + k
        assert flag[i] == int(t["lat"][x] < target[i][t["hw"][x]])


def test_alpha_all_feasible_is_plain_eq1():
    rng = np.random.default_rng(4)
    t = table(rng, n_ops=6, n_hw=2)
    inv_op = rng.integers(0, 6, 500)
    target = np.full((500, 2), 10**6, np.int32)
    plain = oracle.select(inv_op, target, 2, t["cfg_off"], t["hw"], t["batch"], t["lat"], t["cost"])
    for a in ((0, 1), (5, 1), (1, 9)):
        got = sel_alpha(t, inv_op, target, 2, [2, 3], *a)
        assert np.array_equal(got[0], plain[0]) and got[1].all()


def test_alpha_zero_cost_nothing_feasible_is_least_weighted_latency():
    rng = np.random.default_rng(5)
    t = table(rng, n_ops=6, n_hw=3)
    t["cost"][:] = 0
    r_total = np.array([2, 7, 5])
    inv_op = rng.integers(0, 6, 300)
    target = np.zeros((300, 3), np.int32)
    cfg, flag = sel_alpha(t, inv_op, target, 3, r_total, 4, 3)
    assert not flag.any()
    for i, v in enumerate(inv_op):
        a, b = t["cfg_off"][v], t["cfg_off"][v + 1]
        w = [Fraction(int(t["lat"][x]) * int(t["res"][x]), int(t["batch"][x]) * int(r_total[t["hw"][x]]))
             for x in range(a, b)]
        assert cfg[i] == min(range(b - a), key=lambda j: (w[j], j))


def test_alpha_decide_matches_targets_then_select():
    from paper_2102_01887_amd import workloads as wl
    w = wl.with_resource_totals(wl.make_c1(queue=True))
    P = oracle.Problem(w)
    for mode in (oracle.PAPER, oracle.PROB):
        tgt = P.targets(mode, w.Q)
        want = sel_alpha(vars(w), w.inv_op, tgt, w.n_hw, w.hw_res_total, 3, 2)
        got = P.decide_alpha(mode, 3, 2, Q=w.Q)
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


# ---------------------------------------------------------------------------
# planted mistakes in the new functions
# ---------------------------------------------------------------------------

MUTANTS = {
    "queue: latency squared": ("(unsigned __int128)(uint32_t)lat[x] * (unsigned __int128)(uint32_t)res[x]",
                               "(unsigned __int128)(uint32_t)lat[x] * (unsigned __int128)(uint32_t)lat[x]"),
    "queue: R_total of backend 0": ("sum[h] / (unsigned __int128)r_total[h]",
                                    "sum[h] / (unsigned __int128)r_total[0]"),
    "queue: 64-bit accumulator": ("unsigned __int128 sum[64];", "uint64_t sum[64];"),
    "alpha: penalty dropped": ("if (!meets)\n                num +=", "if (0)\n                num +="),
    "alpha: non-strict feasibility": ("int meets = lat[x] < target[i * n_hw + h];",
                                      "int meets = lat[x] <= target[i * n_hw + h];"),
    "alpha: penalty when feasible": ("if (!meets)\n                num +=", "if (meets)\n                num +="),
    "alpha: denominator without R_total": (
        "(unsigned __int128)(uint32_t)batch[x] * (uint64_t)r_total[h] * alpha_den",
        "(unsigned __int128)(uint32_t)batch[x] * alpha_den"),
    "alpha: comparison reversed": ("return p[k] < r[k];", "return p[k] > r[k];"),
    "alpha: ties to the highest index": ("if (best < 0 || fraction_below(num, den, best_n, best_d))",
                                         "if (best < 0 || !fraction_below(best_n, best_d, num, den))"),
    "alpha: lost carry in the wide product": (
        "out[3] = (uint64_t)(top >> 64) + (uint64_t)(hh >> 64);", "out[3] = (uint64_t)(hh >> 64);"),
}

CHECKS = [
    test_fraction_comparison_over_the_full_128_bit_range,
    lambda: test_queue_time_identical_entries_closed_form(12, 2**31 - 1, 2**30, 3),
    lambda: test_queue_time_identical_entries_closed_form(7, 1000, 8, 3),
    test_queue_time_separable_and_permutation_invariant,
    test_alpha_worked_example,
    lambda: test_alpha_against_fractions(0),
    lambda: test_alpha_against_fractions(1),
    test_alpha_large_magnitudes_against_fractions,
    test_alpha_zero_is_cheapest_overall,
    test_alpha_all_feasible_is_plain_eq1,
    test_alpha_zero_cost_nothing_feasible_is_least_weighted_latency,
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    with open(oracle.SRC_PATH) as f:
        src = f.read()
    assert src.count(old) == 1, f"mutation site for '{name}' not unique"
    c = tmp_path / "mutant.c"
    c.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", str(c), "-o", str(so)])
    caught = []
    with oracle.use(str(so)):
        for check in CHECKS:
            try:
                check()
            except (AssertionError, oracle.OracleError):
                caught.append(1)
    assert caught, f"no pin caught the planted mistake '{name}'"
