"""Pins for the learned form's judge in oracle/mlp.py, no GPU.

The surrogate's decisions are scored against the simulator's truth: the mean
of ln latency (truth_mean_log_latency), its 95th percentile (Z95,
truth_p95_latency) and the cost regret / miss rate of a choice against the
decision taken on the truth latencies (regret).  Each is pinned here by
something other than itself:

  * Z95 by the standard library's normal quantile;
  * the truth mean by closed forms (content that changes nothing, a case whose
    exponent is exactly ln 4000) and by the simulator's own samples: the
    residual of every simulated observation against the truth mean is
    N(0, sigma^2) and carries no content term;
  * the truth p95 by scipy's lognormal quantile and by the empirical 95th
    percentile of the simulator's latencies;
  * regret by a hand-worked six-invocation example (positive regrets, a zero
    regret, misses, one at a latency equal to its slack, an unscored
    invocation) and by its sign on random
    draws.

A planted mistake in each (a flipped ratio, a wrong quantile, a dropped
resolution or content term, a non-strict feasibility test, misses counted
over every invocation, the wrong backend's slack) must fail at least one of
these checks: see test_planted_mistake_in_judge_is_caught.
"""
import importlib.util
import math
import statistics

import numpy as np
import pytest
import scipy.stats

import oracle
from oracle import mlp
from paper_2102_01887_amd import workloads as wl

PX_720P = 1280 * 720


# ---------------------------------------------------------------------------
# checks, each taking the judge module so that planted mistakes can be run
# ---------------------------------------------------------------------------

def check_z95(m):
    assert abs(m.Z95 - statistics.NormalDist().inv_cdf(0.95)) < 1e-15


def check_truth_mean_closed_forms(m):
    # content at the reference (no objects, 720p): the profiled latency itself
    lat = np.array([1000, 55555, 1], np.int64)
    got = m.truth_mean_log_latency(lat, 0.6, 0.8, np.zeros(3), np.full(3, PX_720P))
    assert np.allclose(got, np.log(lat.astype(np.float64)), rtol=0, atol=1e-15)
    # 3 objects with a = 1/2 multiply by sqrt(4) = 2; four times the 720p
    # pixels with b = 1/2 multiply by sqrt(4) = 2: 1000 us becomes 4000 us
    got = m.truth_mean_log_latency(np.array([1000]), 0.5, 0.5, np.array([3]), np.array([4 * PX_720P]))
    assert abs(float(np.exp(got[0])) - 4000.0) < 1e-9
    # halving the pixels with b = 1 halves the latency
    got = m.truth_mean_log_latency(np.array([1000]), 0.3, 1.0, np.array([0]), np.array([PX_720P // 2]))
    assert abs(float(np.exp(got[0])) - 500.0) < 1e-9


def _simulated(n=400_000, seed=41):
    world = wl.make_c4_world(3)
    rows, content, y = wl.simulate_c4(world, np.random.default_rng(seed), n)
    return world, rows, content, y


def check_truth_mean_against_simulator(m, sim):
    """y = truth mean + N(0, sigma^2): the residual has mean 0, standard
    deviation sigma and no component along either content term."""
    world, rows, content, y = sim
    w = world.w
    op = rows // 64
    mu = m.truth_mean_log_latency(w.lat[rows], world.a[op, w.hw[rows]], world.b[op],
                                  content.n_obj, content.px)
    r = y.astype(np.float64) - mu
    n = len(r)
    # y is stored as float32 (relative 2^-24 of ~12): well below these bounds
    assert abs(r.mean()) < 5 * world.sigma / math.sqrt(n)
    assert abs(r.std() / world.sigma - 1.0) < 0.01
    # regress the residual on both content terms (and a constant)
    X = np.stack([np.ones(n), np.log1p(content.n_obj), np.log(content.px / PX_720P)], axis=1)
    coef, *_ = np.linalg.lstsq(X, r, rcond=None)
    assert np.all(np.abs(coef) < 0.01), coef


def check_truth_p95_against_lognormal(m):
    rng = np.random.default_rng(5)
    mu = rng.uniform(5.0, 12.0, 500)
    for sigma in (0.0, 0.1, 0.3, 1.0):
        got = m.truth_p95_latency(mu, sigma)
        q = scipy.stats.lognorm.ppf(0.95, s=sigma, scale=np.exp(mu)) if sigma > 0 else np.exp(mu)
        # ceil of the quantile; allow the quantile to sit within 1e-9 relative
        # of an integer (either side is then a correct ceiling)
        lo, hi = np.ceil(q * (1 - 1e-9)), np.ceil(q * (1 + 1e-9))
        assert np.all((got >= lo) & (got <= hi)), sigma
    # e = exp(1): mu = ln 1000 and sigma = 1 / Z gives ceil(1000 e) = 2719
    z = statistics.NormalDist().inv_cdf(0.95)
    assert m.truth_p95_latency(np.array([math.log(1000.0)]), 1.0 / z)[0] == 2719
    # capped at the int32 range
    assert m.truth_p95_latency(np.array([40.0]), 0.3)[0] == 2 ** 31 - 1


def check_truth_p95_against_simulator(m, sim):
    """Per content cell with many draws, the 95th percentile of the simulated
    latencies exp(y) matches truth_p95 of the cell's mean."""
    world, rows, content, y = sim
    w = world.w
    op = rows // 64
    mu = m.truth_mean_log_latency(w.lat[rows], world.a[op, w.hw[rows]], world.b[op],
                                  content.n_obj, content.px)
    # standardise: the 95th percentile of (y - mu) must be Z95 * sigma, which
    # truth_p95 of mu = 0 gives as ceil(exp(Z95 sigma) * 1e6) / 1e6 after scaling
    r = y.astype(np.float64) - mu
    emp = float(np.quantile(r, 0.95))
    want = math.log(float(m.truth_p95_latency(np.array([math.log(1e6)]), world.sigma)[0]) / 1e6)
    # sampling error of the 0.95 quantile with 4e5 draws: about 1e-3 (in ln us)
    assert abs(emp - want) < 4e-3, (emp, want)


# hand-worked example: one op with three configurations on two backends
#   k   hw  B   C    C/B
#   0   0   1   10   10
#   1   1   2   30   15
#   2   1   1   40   40
HW = np.array([0, 1, 1], np.int32)
BATCH = np.array([1, 2, 1], np.int32)
COST = np.array([10, 30, 40], np.int64)
#           truth latency (k0, k1, k2)   target (hw 0, hw 1)   surrogate choice
# A          100  50  20                  90  60              k2: feasible; truth k1 (15) -> regret 40/15 - 1
# B          100  50  20                  200 200             k0: the truth choice -> regret 0
# C          100  50  20                  200 30              k1: 50 >= 30 on backend 1 -> miss (truth k0)
# D          100  50  20                  50  10              k2: nothing truly feasible -> not scored
# E           30  50  20                  40  25              k2: feasible; truth k0 (10) -> regret 40/10 - 1
# F          100  50  20                  200 50              k1: 50 is not below 50 -> miss (truth k0)
TRUTH_LAT = np.array([[100, 50, 20], [100, 50, 20], [100, 50, 20], [100, 50, 20], [30, 50, 20],
                      [100, 50, 20]], np.int32)
TARGET = np.array([[90, 60], [200, 200], [200, 30], [50, 10], [40, 25], [200, 50]], np.int32)
SURR = np.array([2, 0, 1, 2, 2, 1], np.int32)
TRUTH_CHOICE = np.array([1, 0, 0, 2, 0, 0], np.int32)
TRUTH_FLAG = np.array([1, 1, 1, 0, 1, 1], np.uint8)
WANT_REGRET = (40 / 15 - 1 + 0 + 40 / 10 - 1) / 3      # = 14/9
WANT_MISS = 2 / 6


def check_regret_worked_example(m):
    r = m.regret(SURR, TRUTH_CHOICE, TRUTH_FLAG, TRUTH_LAT, TARGET, HW, COST, BATCH, np.zeros(6, np.int64))
    assert r["n_scored"] == 3 and r["n_feasible"] == 5
    assert abs(r["mean_regret"] - WANT_REGRET) < 1e-12
    assert abs(r["miss_rate"] - WANT_MISS) < 1e-12


def check_regret_nonnegative_and_zero_on_truth(m):
    rng = np.random.default_rng(6)
    n, n_cfg = 3000, 12
    hw = rng.integers(0, 3, n_cfg).astype(np.int32)
    batch = rng.integers(1, 9, n_cfg).astype(np.int32)
    cost = rng.integers(1, 1000, n_cfg).astype(np.int64)
    truth = rng.integers(10, 1000, (n, n_cfg)).astype(np.int32)
    target = rng.integers(0, 1100, (n, 3)).astype(np.int32)
    cfg_off = np.array([0, n_cfg], np.int32)
    t_c, t_f = oracle.select_lat(np.zeros(n, np.int32), target, 3, cfg_off, hw, batch, truth, cost)
    base = np.zeros(n, np.int64)
    r0 = m.regret(t_c, t_c, t_f, truth, target, hw, cost, batch, base)
    assert r0["mean_regret"] == 0.0 and r0["miss_rate"] == 0.0
    # any other choice: regret >= 0 and strictly positive on this draw
    other = rng.integers(0, n_cfg, n).astype(np.int32)
    r1 = m.regret(other, t_c, t_f, truth, target, hw, cost, batch, base)
    assert r1["mean_regret"] > 0.0 and r1["miss_rate"] > 0.0
    # misses are counted only where a truly feasible configuration existed
    assert r1["miss_rate"] <= float(np.mean(t_f == 1))


def run_all(m, sim):
    check_z95(m)
    check_truth_mean_closed_forms(m)
    check_truth_mean_against_simulator(m, sim)
    check_truth_p95_against_lognormal(m)
    check_truth_p95_against_simulator(m, sim)
    check_regret_worked_example(m)
    check_regret_nonnegative_and_zero_on_truth(m)


# ---------------------------------------------------------------------------
# tests
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def sim():
    return _simulated()


def test_z95_is_the_normal_quantile():
    check_z95(mlp)


def test_truth_mean_closed_forms():
    check_truth_mean_closed_forms(mlp)


def test_truth_mean_against_the_simulator(sim):
    check_truth_mean_against_simulator(mlp, sim)


def test_truth_p95_against_scipy_lognormal():
    check_truth_p95_against_lognormal(mlp)


def test_truth_p95_against_the_simulator(sim):
    check_truth_p95_against_simulator(mlp, sim)


def test_regret_worked_example():
    check_regret_worked_example(mlp)


def test_worked_example_truth_choices_follow_eq1():
    """The example's truth choices are what the plain oracle selects on the
    truth latencies (cheapest per item meeting its backend's slack, else the
    fastest)."""
    c, f = oracle.select_lat(np.zeros(6, np.int32), TARGET, 2, np.array([0, 3], np.int32), HW, BATCH,
                             TRUTH_LAT, COST)
    assert c.tolist() == TRUTH_CHOICE.tolist() and f.tolist() == TRUTH_FLAG.tolist()


def test_regret_nonnegative_and_zero_on_truth():
    check_regret_nonnegative_and_zero_on_truth(mlp)


JUDGE_MUTANTS = {
    "flipped regret ratio": ("per_item[x_c[ok]] / np.maximum(per_item[x_t[ok]], 1e-300)",
                             "per_item[x_t[ok]] / np.maximum(per_item[x_c[ok]], 1e-300)"),
    "0.975 quantile": ("Z95 = 1.6448536269514722", "Z95 = 1.959963984540054"),
    "0.90 quantile": ("Z95 = 1.6448536269514722", "Z95 = 1.2815515655446004"),
    "dropped resolution term": ("\n            + b_op * np.log(np.asarray(px, np.float64) / px_ref))", ")"),
    "dropped content term": ("a_hw * np.log1p(n_obj)", "0.0 * np.log1p(n_obj)"),
    "ln(n_obj) for ln(1 + n_obj)": ("a_hw * np.log1p(n_obj)", "a_hw * np.log(np.maximum(n_obj, 1))"),
    "mean instead of p95": ("np.exp(mu_star + Z95 * sigma)", "np.exp(mu_star)"),
    "floor instead of ceiling": ("np.ceil(np.exp(mu_star + Z95 * sigma))",
                                 "np.floor(np.exp(mu_star + Z95 * sigma))"),
    "non-strict truth feasibility": ("feas_c = truth_lat[idx, choice] < target",
                                     "feas_c = truth_lat[idx, choice] <= target"),
    "misses over every invocation": ("np.mean(has & ~feas_c)", "np.mean(~feas_c)"),
    "backend 0's slack for every configuration": ("target[idx, hw[x_c]]", "target[idx, 0]"),
    "regret against the choice itself": ("x_t = cfg_base + truth_choice", "x_t = cfg_base + choice"),
}


def _mutant_module(name, tmp_path):
    old, new = JUDGE_MUTANTS[name]
    src = open(mlp.__file__).read()
    assert src.count(old) == 1, f"mutation site for '{name}' not unique"
    path = tmp_path / "mlp_mutant.py"
    path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location("mlp_mutant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("name", sorted(JUDGE_MUTANTS))
def test_planted_mistake_in_judge_is_caught(name, tmp_path, sim):
    mod = _mutant_module(name, tmp_path)
    with pytest.raises(AssertionError):
        run_all(mod, sim)


def test_unmutated_judge_passes_every_check(sim):
    run_all(mlp, sim)
