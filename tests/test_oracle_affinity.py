"""Pins for the oracle's Eq. 3 affinity (Sec. 4.4), CPU only.

affinity(op, h) = min obj over the op's configurations not on backend h
                  / min obj over its configurations on h,
obj = Eq. 1 with finite alpha, each configuration judged against the slack
of its own backend.  Pinned by a hand-worked example, by exact Fractions on
random small problems (objective written in Eq. 1's two-term form), by
closed forms (one backend: infinite affinity; a backend without
configurations: 0; mirrored backends: 1), and by planted mistakes.
"""
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2102_01887_amd import workloads as wl


def single_op(hw, batch, res, lat, cost, n_hw, r_total, slo, elapsed):
    """One pipeline of one op: W = ref, so every backend's target is the
    remaining time itself."""
    n = len(hw)
    return wl.Workload(
        name="one-op", n_hw=n_hw, pipe_off=np.array([0, 1], np.int32),
        succ_off=np.array([0, 0], np.int32), succ_ids=np.zeros(0, np.int32),
        succ_q16=np.zeros(0, np.uint32), cfg_off=np.array([0, n], np.int32),
        hw=np.asarray(hw, np.int32), batch=np.asarray(batch, np.int32),
        res=np.asarray(res, np.int32), lat=np.asarray(lat, np.int32),
        cost=np.asarray(cost, np.int64), inv_op=np.zeros(len(slo), np.int32),
        elapsed=np.asarray(elapsed, np.int32), slo=np.asarray(slo, np.int32),
        hw_res_total=np.asarray(r_total, np.int64))


def test_worked_example():
    # configurations (backend, B, R, L, C): x0 (0, 1, 2, 10, 6), x1 (1, 2, 4, 30, 8),
    # x2 (1, 1, 1, 5, 9); R_total = (4, 8); alpha = 1/2; remaining time 20 on
    # both backends: x0 meets (obj 6), x1 misses (4 + 1/2*30*4/(2*8) = 31/4),
    # x2 meets (9).  affinity(0) = min(31/4, 9) / 6 = 31/24,
    # affinity(1) = 6 / (31/4) = 24/31.
    # With remaining time 40 everything meets: objs 6, 4, 9 -> affinity(0) = 4/6,
    # affinity(1) = 6/4.  With 0 nothing meets: 17/2, 31/4, 149/16 ->
    # affinity(0) = (31/4)/(17/2) = 31/34, affinity(1) = (17/2)/(31/4) = 34/31.
    w = single_op([0, 1, 1], [1, 2, 1], [2, 4, 1], [10, 30, 5], [6, 8, 9], 2, [4, 8],
                  slo=[20, 40, 100], elapsed=[0, 0, 100])
    P = oracle.Problem(w)
    own, oth = oracle.affinity_terms(w.inv_op, w.elapsed, w.slo, 2, None, P.ref, P.W(0), w.cfg_off,
                                     w.hw, w.batch, w.res, w.lat, w.cost, w.hw_res_total, 1, 2)
    assert own[0] == [Fraction(6), Fraction(31, 4)] and oth[0] == [Fraction(31, 4), Fraction(6)]
    aff = P.affinity(0, 1, 2)
    assert aff[0].tolist() == [float(Fraction(31, 24)), float(Fraction(24, 31))]
    assert aff[1].tolist() == [float(Fraction(4, 6)), float(Fraction(6, 4))]
    assert aff[2].tolist() == [float(Fraction(31, 34)), float(Fraction(34, 31))]


def brute(w, target, a_num, a_den):
    alpha = Fraction(a_num, a_den)
    out = []
    for i, v in enumerate(w.inv_op):
        row = []
        for h in range(w.n_hw):
            own, oth = None, None
            for x in range(w.cfg_off[v], w.cfg_off[v + 1]):
                g = int(w.hw[x])
                obj = Fraction(int(w.cost[x]), int(w.batch[x]))
                if not int(w.lat[x]) < int(target[i][g]):
                    obj += alpha * int(w.lat[x]) * int(w.res[x]) / (int(w.batch[x]) * int(w.hw_res_total[g]))
                if g == h:
                    own = obj if own is None or obj < own else own
                else:
                    oth = obj if oth is None or obj < oth else oth
            row.append(oracle.affinity_value(own, oth))
        out.append(row)
    return np.array(out)


@pytest.mark.parametrize("seed", range(5))
def test_against_fractions(seed):
    rng = np.random.default_rng(200 + seed)
    w = wl.with_resource_totals(wl.random_small(rng, n_inv=150), slots=int(rng.integers(1, 5)))
    P = oracle.Problem(w)
    Q = rng.integers(0, 15_000, w.n_hw)  # per-backend queueing times: the targets differ
    for a in ((0, 1), (1, 1), (5, 3)):
        for mode in (0, 1):
            for q in (None, Q):
                got = P.affinity(mode, *a, Q=q)
                want = brute(w, P.targets(mode, Q=q), *a)
                assert np.array_equal(got, want), (a, mode, q)


def test_closed_forms():
    # a single backend: no alternative, infinite affinity
    w = single_op([0, 0], [1, 2], [1, 1], [10, 20], [5, 7], 1, [4], slo=[15, 100], elapsed=[0, 0])
    assert np.all(np.isinf(oracle.Problem(w).affinity(0, 1, 1)))
    # backend 2 has no configuration: affinity 0 to it
    w = single_op([0, 1], [1, 1], [1, 1], [10, 12], [5, 4], 3, [4, 4, 4], slo=[11, 100], elapsed=[0, 0])
    aff = oracle.Problem(w).affinity(0, 1, 1)
    assert (aff[:, 2] == 0).all() and (aff[:, :2] > 0).all()
    # mirrored backends (same configurations, same R_total): affinity 1
    w = single_op([0, 1, 0, 1], [1, 1, 2, 2], [1, 1, 3, 3], [10, 10, 30, 30], [5, 5, 8, 8], 2, [6, 6],
                  slo=[5, 11, 31, 1000], elapsed=[0, 0, 0, 0])
    assert np.all(oracle.Problem(w).affinity(0, 2, 1) == 1.0)
    # zero-cost configurations on both sides with every slack met: 0 / 0 -> 1
    w = single_op([0, 1], [1, 1], [1, 1], [10, 10], [0, 0], 2, [4, 4], slo=[100], elapsed=[0])
    assert np.all(oracle.Problem(w).affinity(0, 1, 1) == 1.0)


MUTANTS = {
    "own and other swapped": ("                if (g == h) {\n                    if (!have_own",
                              "                if (g != h) {\n                    if (!have_own"),
    "other side keeps the largest": ("} else if (!have_oth || fraction_below(num, den, tn, td)) {",
                                     "} else if (!have_oth || fraction_below(tn, td, num, den)) {"),
    "slack of backend h for every configuration": ("int meets = lat[x] < target_scratch[g];",
                                                   "int meets = lat[x] < target_scratch[h];"),
}

CHECKS = [test_worked_example, lambda: test_against_fractions(0), lambda: test_against_fractions(1),
          test_closed_forms]


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
    caught = 0
    with oracle.use(str(so)):
        for check in CHECKS:
            try:
                check()
            except (AssertionError, oracle.OracleError):
                caught += 1
    assert caught, f"no pin caught the planted mistake '{name}'"
