"""Pins for the oracle's safe delayed batching (Sec. 4.4), CPU only.

Readings (per invocation of op v; available, upstream and wait_us per op):
x* = Eq. 1 over every configuration; commit x* if B(x*) <= available; wait
(cfg -2) if x* meets its slack, available + upstream >= B(x*) and
wait_us + L(x*) < slack of x*'s backend; otherwise commit Eq. 1 over the
configurations with B <= max(available, 1), or x* if there is none.
Pinned by a hand-worked example, by the closed forms "plenty available ->
plain Eq. 1" and "nothing upstream -> never waits", by a Fraction brute force
of the readings on random problems, and by planted mistakes.
"""
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2102_01887_amd import workloads as wl
from test_oracle_affinity import single_op

WAIT = oracle.CFG_WAIT


def test_worked_example():
    # one op, backend 0 only; x0: B 1, L 10, C 10 (10 per item); x1: B 4, L 12,
    # C 8 (2 per item).  W = ref = L(x0) = 10, so the slack equals the remaining
    # time.  With remaining time 20 both meet it and x* = x1 (cheaper per item).
    w = single_op([0, 0], [1, 4], [1, 1], [10, 12], [10, 8], 1, [8],
                  slo=[20] * 5 + [11], elapsed=[0] * 6)
    P = oracle.Problem(w)
    avail = lambda a: np.array([a], np.int32)
    cases = [  # (available, upstream, wait_us) -> (cfg, flag)
        ((4, 0, 0), (1, 1)),    # enough available: commit x1
        ((2, 2, 5), (WAIT, 1)),  # 2 + 2 >= 4 and 5 + 12 < 20: wait
        ((2, 1, 5), (0, 1)),    # 2 + 1 < 4: best with B <= 2 is x0
        ((2, 5, 8), (0, 1)),    # 8 + 12 >= 20 would break the slack: x0
        ((0, 0, 0), (0, 1)),    # nothing upstream: B <= 1 -> x0
    ]
    for i, ((a, u, t), want) in enumerate(cases):
        c, f = P.decide_batching(0, avail(a), avail(u), avail(t), sl=slice(i, i + 1))
        assert (c[0], f[0]) == want, (a, u, t)
    # remaining time 11: only x0 meets (10 < 11), B 1 fits: commit x0
    c, f = P.decide_batching(0, avail(1), avail(100), avail(0), sl=slice(5, 6))
    assert (c[0], f[0]) == (0, 1)


def brute(w, target, avail, up, wait):
    out_c, out_f = [], []
    for i, v in enumerate(w.inv_op):
        xs = range(w.cfg_off[v], w.cfg_off[v + 1])

        def eq1(limit):
            ok = [x for x in xs if w.batch[x] <= limit]
            if not ok:
                return None, 0
            feas = [x for x in ok if w.lat[x] < target[i][w.hw[x]]]
            if feas:
                return min(feas, key=lambda x: (Fraction(int(w.cost[x]), int(w.batch[x])), x)), 1
            return min(ok, key=lambda x: (int(w.lat[x]), x)), 0

        x_star, m = eq1(10**9)
        a = int(avail[v])
        if w.batch[x_star] <= a:
            c, f = x_star, m
        elif m and a + int(up[v]) >= w.batch[x_star] and \
                int(wait[v]) + int(w.lat[x_star]) < int(target[i][w.hw[x_star]]):
            out_c.append(WAIT)
            out_f.append(1)
            continue
        else:
            xr, mr = eq1(max(a, 1))
            c, f = (x_star, m) if xr is None else (xr, mr)
        out_c.append(c - w.cfg_off[v])
        out_f.append(f)
    return np.array(out_c), np.array(out_f)


def inputs(rng, w, hi_avail=6, hi_up=6, hi_wait=3000):
    return (rng.integers(0, hi_avail, w.n_ops).astype(np.int32),
            rng.integers(0, hi_up, w.n_ops).astype(np.int32),
            rng.integers(0, hi_wait, w.n_ops).astype(np.int32))


@pytest.mark.parametrize("seed", range(6))
def test_against_brute_force(seed):
    rng = np.random.default_rng(300 + seed)
    w = wl.random_small(rng, n_inv=300)
    P = oracle.Problem(w)
    Q = rng.integers(0, 10_000, w.n_hw)
    for mode in (0, 1):
        for q in (None, Q):
            a, u, t = inputs(rng, w)
            got = P.decide_batching(mode, a, u, t, Q=q)
            want = brute(w, P.targets(mode, Q=q), a, u, t)
            assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), (mode, q)


def test_plenty_available_is_plain_eq1():
    w = wl.make_c1()
    P = oracle.Problem(w)
    big = np.full(w.n_ops, 10**6, np.int32)
    c, f = P.decide_batching(0, big, np.zeros(w.n_ops, np.int32), np.zeros(w.n_ops, np.int32))
    c0, f0 = P.decide(0)
    assert np.array_equal(c, c0) and np.array_equal(f, f0)


def test_nothing_upstream_never_waits_and_fits():
    rng = np.random.default_rng(7)
    w = wl.make_c1()
    P = oracle.Problem(w)
    a = rng.integers(1, 4, w.n_ops).astype(np.int32)
    c, f = P.decide_batching(0, a, np.zeros(w.n_ops, np.int32), np.zeros(w.n_ops, np.int32))
    assert (c != WAIT).all()
    # every op of C1 has a batch-1 configuration, so the committed batch fits
    x = w.cfg_off[w.inv_op] + c
    assert (w.batch[x] <= np.maximum(a[w.inv_op], 1)).all()


MUTANTS = {
    "wait breaks the slack": ("(int64_t)wait_us[v] + lat[xs] < target_scratch[hw[xs]]",
                              "(int64_t)wait_us[v] + lat[xs] <= target_scratch[hw[xs]]"),
    "upstream ignored": ("avail + (int64_t)upstream[v] >= batch[xs]", "avail + 1000000 >= batch[xs]"),
    "restricted scan ignores the batch": ("avail > 1 ? avail : 1,", "INT64_MAX,"),
    "waits for a configuration with no larger batch": ("if (batch[xs] <= avail) {", "if (batch[xs] < avail) {"),
}

CHECKS = [test_worked_example, lambda: test_against_brute_force(0), lambda: test_against_brute_force(1),
          test_plenty_available_is_plain_eq1, test_nothing_upstream_never_waits_and_fits]


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
