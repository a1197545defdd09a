"""Pins for the oracle's feedback step (exponential smoothing of profiled
latencies, Sec. 3.3), CPU only.

Reading: the m observations of one configuration in a batch, with sum S, make
one step toward their mean: L' = L + floor(beta * (S/m - L)), clamped to
[1, 2^31 - 1], beta = beta_q16 / 65536.  Pinned by closed forms (beta = 0
keeps L; beta = 1 gives floor of the mean; one observation gives
floor((1 - beta) L + beta obs)), the bound min(L, mean) - 1 < L' <= max(L, mean),
exact Fractions on random batches (including negative steps, where a
truncating division would be wrong), untouched configurations, skipped
observations, and planted mistakes.
"""
import math
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import oracle


def table(rng, n_ops=5, cfg_hi=6, lat_hi=10_000):
    counts = rng.integers(1, cfg_hi + 1, n_ops)
    cfg_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    lat = rng.integers(1, lat_hi, int(cfg_off[-1])).astype(np.int32)
    return cfg_off, lat


def observations(rng, cfg_off, n_obs, lat_hi=20_000):
    n_ops = len(cfg_off) - 1
    op = rng.integers(0, n_ops, n_obs).astype(np.int32)
    k = np.array([rng.integers(0, cfg_off[v + 1] - cfg_off[v]) for v in op], np.int32)
    obs = rng.integers(1, lat_hi, n_obs).astype(np.int32)
    return op, k, obs


def test_beta_zero_keeps_latencies():
    rng = np.random.default_rng(0)
    cfg_off, lat = table(rng)
    op, k, obs = observations(rng, cfg_off, 300)
    new, skipped = oracle.feedback(op, k, obs, cfg_off, lat, 0)
    assert skipped == 0 and np.array_equal(new, lat)


def test_beta_one_gives_floor_of_the_mean():
    rng = np.random.default_rng(1)
    cfg_off, lat = table(rng)
    op, k, obs = observations(rng, cfg_off, 400)
    new, _ = oracle.feedback(op, k, obs, cfg_off, lat, 65536)
    x = cfg_off[op] + k
    for c in range(len(lat)):
        sel = obs[x == c]
        want = lat[c] if sel.size == 0 else int(sel.astype(np.int64).sum()) // sel.size
        assert new[c] == want


@pytest.mark.parametrize("beta", [1, 6554, 32768, 52429, 65535])
def test_single_observation_closed_form(beta):
    rng = np.random.default_rng(beta)
    cfg_off, lat = table(rng, n_ops=1, cfg_hi=1)
    for _ in range(200):
        obs = int(rng.integers(1, 20_000))
        new, _ = oracle.feedback([0], [0], [obs], cfg_off, lat, beta)
        b = Fraction(beta, 65536)
        assert new[0] == math.floor((1 - b) * int(lat[0]) + b * obs)
        lat = new


def test_against_fractions_and_bounds():
    rng = np.random.default_rng(2)
    for rep in range(20):
        cfg_off, lat = table(rng, n_ops=8, cfg_hi=8)
        op, k, obs = observations(rng, cfg_off, int(rng.integers(1, 400)))
        beta = int(rng.integers(0, 65537))
        new, _ = oracle.feedback(op, k, obs, cfg_off, lat, beta)
        x = cfg_off[op] + k
        for c in range(len(lat)):
            sel = obs[x == c].astype(np.int64)
            if sel.size == 0:
                assert new[c] == lat[c]
                continue
            mean = Fraction(int(sel.sum()), sel.size)
            want = math.floor(int(lat[c]) + Fraction(beta, 65536) * (mean - int(lat[c])))
            assert new[c] == max(1, want), (rep, c)
            assert min(int(lat[c]), mean) - 1 < new[c] <= max(int(lat[c]), mean)


def test_clamps_and_skips():
    cfg_off = np.array([0, 2, 3], np.int32)
    lat = np.array([5, 2**31 - 1, 1], np.int32)
    # a step below 1 is clamped to 1; the maximum stays representable
    new, skipped = oracle.feedback([0, 0, 1, 0, 9, 1, 0], [0, 1, 0, 5, 0, -1, 1],
                                   [1, 2**31 - 1, 1, 3, 3, 3, 0], cfg_off, lat, 65536)
    assert skipped == 4  # op 0 cfg 5, op 9, cfg -1, latency 0
    assert new.tolist() == [1, 2**31 - 1, 1]


MUTANTS = {
    "truncating division": ("            q -= 1; /* floor, not truncation */", "            q -= 0;"),
    "step from the sum, not the mean": ("__int128 den = (__int128)65536 * m[x];",
                                        "__int128 den = (__int128)65536;"),
    "wrong sign of the step": ("__int128 nl = (__int128)lat[x] + q;", "__int128 nl = (__int128)lat[x] - q;"),
    "beta ignored": ("__int128 num = (__int128)beta_q16 * (S[x] - (__int128)m[x] * lat[x]);",
                     "__int128 num = (__int128)65536 * (S[x] - (__int128)m[x] * lat[x]);"),
    "observations of the wrong configuration": ("int64_t x = cfg_off[v] + obs_cfg[i];",
                                                "int64_t x = cfg_off[v];"),
}

CHECKS = [test_beta_zero_keeps_latencies, test_beta_one_gives_floor_of_the_mean,
          lambda: test_single_observation_closed_form(32768), test_against_fractions_and_bounds,
          test_clamps_and_skips]


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
