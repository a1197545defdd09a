"""Pins of the CPU reference of the pipeline simulator (oracle.simulator).

Philox4x32-10 against the published known-answer vectors; the inversion
samplers against scipy's quantile functions; the Beta(3, 7) construction,
the Box-Muller normals and the row and resolution draws against their
distributions; the observed ln latency against the pinned truth mean of
oracle.mlp; and planted mistakes that must be caught.
"""
import numpy as np
import pytest
from scipy import stats

from oracle import mlp
from oracle import simulator as S


def test_philox_known_answers():
    # known-answer vectors of Philox4x32-10 (Salmon et al., SC 2011)
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
        ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
        ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
         (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
    ]
    for ctr, key, want in cases:
        got = S.philox4x32_10(np.array([ctr], np.uint64), key)[0]
        assert tuple(int(x) for x in got) == want


def test_philox_planted_round_count_fails():
    # nine rounds instead of ten would not reproduce the vectors
    ctr, key = np.zeros((1, 4), np.uint64), (0, 0)
    c = np.asarray(ctr, np.uint64)
    c0, c1, c2, c3 = (c[:, j].copy() for j in range(4))
    k0, k1 = np.uint64(0), np.uint64(0)
    for r in range(9):
        p0, p1 = np.uint64(S.PHILOX_M0) * c0, np.uint64(S.PHILOX_M1) * c2
        c0, c1, c2, c3 = ((p1 >> np.uint64(32)) ^ c1 ^ k0, p1 & np.uint64(S.M32),
                          (p0 >> np.uint64(32)) ^ c3 ^ k1, p0 & np.uint64(S.M32))
        k0 = (k0 + np.uint64(S.PHILOX_W0)) & np.uint64(S.M32)
        k1 = (k1 + np.uint64(S.PHILOX_W1)) & np.uint64(S.M32)
    assert int(c0[0]) != 0x6627E8D5


def test_inversion_samplers_match_scipy_quantiles():
    rng = np.random.default_rng(0)
    u = rng.uniform(size=4000)
    rate = np.exp(np.log(2.0) + rng.standard_normal(4000))
    k, margin = S.poisson_inv(u, rate, np.full(4000, 60))
    ok = margin > 1e-9
    want = np.minimum(stats.poisson.ppf(u, rate), 60)
    assert np.array_equal(k[ok], want[ok]) and ok.mean() > 0.999
    m = rng.integers(0, 61, 4000)
    kb, mb = S.binomial_inv(u, m, 0.6)
    okb = mb > 1e-9
    assert np.array_equal(kb[okb], stats.binom.ppf(u, m, 0.6)[okb]) and okb.mean() > 0.999
    # the cap applies: a cap of 0 gives 0, the people cap 60
    assert (S.poisson_inv(u[:10], rate[:10], np.zeros(10, np.int64))[0] == 0).all()
    assert S.poisson_inv(np.array([1 - 1e-12]), np.array([500.0]), np.array([60]))[0][0] == 60


def test_simulated_content_distributions():
    n = 200_000
    lat = np.full(64 * 2, 5000, np.int32)
    hw = np.tile(np.repeat([0, 1], 32), 2).astype(np.int32)
    a = np.array([[0.5, 0.2], [0.4, 0.1]])
    b = np.array([0.7, 0.9])
    d = S.simulate(n, 12345, 128, lat, hw, a, b, 0.3)
    f = d["feat64"]
    # rows uniform over the 128 rows, resolutions over three
    assert stats.chisquare(np.bincount(d["rows"], minlength=128)).pvalue > 1e-4
    assert stats.chisquare(np.bincount(d["res"], minlength=3)).pvalue > 1e-4
    # branch hit rate Beta(3, 7); motion, blur, brightness U(0, 1)
    assert stats.kstest(f[:20_000, 10], stats.beta(3, 7).cdf).pvalue > 1e-4
    for j in (7, 8, 9):
        assert stats.kstest(f[:20_000, j], "uniform").pvalue > 1e-4
    # the phase features lie on the unit circle
    assert np.allclose(f[:, 11] ** 2 + f[:, 12] ** 2, 1.0)
    # people: Poisson with a lognormal(ln 2, 1) rate (mixture mean 2 e^(1/2)), capped at 60
    assert abs(d["people"].mean() - 2 * np.exp(0.5)) < 0.05 and d["people"].max() <= 60
    assert (d["people"] + d["cars"] <= 60).all() and (d["faces"] <= d["people"]).all()
    assert abs(d["faces"].sum() / d["people"].sum() - 0.6) < 0.01
    # y: the pinned truth mean plus N(0, 0.3^2) noise
    op = d["rows"] // 64
    wh = np.asarray(S.RESOLUTIONS)[d["res"]]
    mu = mlp.truth_mean_log_latency(lat[d["rows"]], a[op, hw[d["rows"]]], b[op], d["people"] + d["cars"],
                                    wh[:, 0] * wh[:, 1])
    resid = d["y64"] - mu
    assert abs(resid.mean()) < 0.005 and abs(resid.std() - 0.3) < 0.005
    assert stats.kstest(resid[:20_000] / 0.3, "norm").pvalue > 1e-4
    # features are BF16 values
    assert np.array_equal(d["feat"], mlp.bf16(d["feat"]))


def test_samples_do_not_depend_on_the_split():
    lat = np.full(64, 5000, np.int32)
    hw = np.repeat([0, 1], 32).astype(np.int32)
    a, b = np.array([[0.5, 0.2]]), np.array([0.7])
    whole = S.simulate(1000, 7, 64, lat, hw, a, b, 0.3)
    part = S.simulate(300, 7, 64, lat, hw, a, b, 0.3, first=700)
    assert np.array_equal(whole["rows"][700:], part["rows"])
    assert np.array_equal(whole["y"][700:], part["y"])
    other = S.simulate(1000, 8, 64, lat, hw, a, b, 0.3)
    assert not np.array_equal(whole["rows"], other["rows"])
