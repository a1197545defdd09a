"""GPU parity of the feedback step: exponential smoothing of the profile from
observed latencies and the device rebuild of every latency-derived table,
through the C ABI, against the oracle.  Integer throughout: bit-exact.

After a feedback call the decisions of every scan mode, both slack modes, with
and without queueing times, must equal the oracle's decisions on the
oracle-smoothed profile, and so must W and the latencies themselves.
"""
import numpy as np
import pytest

import oracle
from paper_2102_01887_amd import binding as B
from paper_2102_01887_amd import workloads as wl
from test_gpu_parity import PAPER, PROB, Run, assert_full_parity, dev, say

pytestmark = pytest.mark.gpu


def observe(w, rng, n_obs, spread=(0.5, 2.0)):
    return wl.observations(w, rng, n_obs, spread)


def apply(r, op, cfg, lat, beta):
    torch = r.torch
    r.L.feedback(dev(op, torch), dev(cfg, torch), dev(lat, torch), beta)
    torch.cuda.synchronize()
    new, skipped = oracle.feedback(op, cfg, lat, r.w.cfg_off, r.w.lat, beta)
    w2 = r.w.with_invocations(r.w.inv_op, r.w.elapsed, r.w.slo, r.w.Q)
    w2.lat = new
    r.w = w2
    r.P = oracle.Problem(w2)
    return skipped


def check(r, Q=None, scans=B.SCANS):
    assert np.array_equal(r.L.export("lat"), r.w.lat)
    assert np.array_equal(r.L.export("ref"), r.P.ref)
    assert_full_parity(r, Q=Q, scans=scans)


@pytest.mark.parametrize("beta", [0, 16384, 65536])
def test_feedback_c1(beta):
    w = wl.make_c1(queue=True)
    r = Run(w)
    rng = np.random.default_rng(1)
    for step in range(3):
        apply(r, *observe(r.w, rng, 300), beta)
        check(r)
        check(r, Q=w.Q)


def test_feedback_c2_reduced_many_batches():
    w = wl.make_c2(seed=51, n_pipelines=20, n_inv=30_000)
    r = Run(w)
    rng = np.random.default_rng(2)
    for step in range(4):
        apply(r, *observe(r.w, rng, 20_000), 13107)
        say(f"c2 feedback step {step}: {np.mean(r.w.lat != w.lat):.3f} of latencies changed")
    check(r)
    check(r, Q=[20_000, 0, 300_000, 1_000_000], scans=(B.SCAN_INDEXED,))


def test_feedback_c3_reduced():
    w = wl.make_c3(seed=52, n_pipelines=24, n_inv=20_000)
    r = Run(w)
    rng = np.random.default_rng(3)
    apply(r, *observe(r.w, rng, 50_000, spread=(0.2, 5.0)), 32768)
    check(r, scans=(B.SCAN_INDEXED, B.SCAN_FULL))


def test_feedback_fuzz_small_tables_with_ties():
    rng = np.random.default_rng(4)
    for rep in range(10):
        w = wl.random_small(rng, n_inv=1500, name=f"fb{rep}")
        r = Run(w)
        for step in range(2):
            op, cfg, lat = observe(r.w, rng, int(rng.integers(1, 400)), spread=(0.3, 3.0))
            lat = np.minimum(lat, 60)  # small values: many equal latencies after smoothing
            apply(r, op, cfg, lat, int(rng.integers(0, 65537)))
        check(r)


def test_feedback_skips_bad_observations_and_flags_them():
    w = wl.make_c1()
    r = Run(w)
    rng = np.random.default_rng(5)
    op, cfg, lat = observe(w, rng, 200)
    op[::9] = w.n_ops
    cfg[4::13] = 999
    lat[7::11] = 0
    skipped = apply(r, op, cfg, lat, 40000)
    assert skipped > 0
    assert r.L.stats(reset_error=True)["device_error"] & B.DEVERR_INVALID_OBSERVATION
    check(r)


def test_feedback_then_latency_update_and_alpha():
    w = wl.with_resource_totals(wl.make_c2(seed=53, n_pipelines=8, n_inv=10_000))
    r = Run(w)
    rng = np.random.default_rng(6)
    apply(r, *observe(r.w, rng, 5000), 20000)
    # the finite-alpha tables were dropped; rebuilt from the smoothed profile
    with pytest.raises(B.LlamaError):
        r.L.decide_alpha(r.op, r.el, r.slo)
    r.L.set_alpha(3, 2)
    c, f = r.L.decide_alpha(r.op, r.el, r.slo)
    r.torch.cuda.synchronize()
    c_or, f_or = r.P.decide_alpha(PAPER, 3, 2)
    assert np.array_equal(c.cpu().numpy(), c_or) and np.array_equal(f.cpu().numpy(), f_or)
    # a host-side latency update replaces the smoothed profile entirely
    lat2 = np.maximum(1, (w.lat * rng.uniform(0.8, 1.2, w.n_cfg))).astype(np.int32)
    r.L.update_latencies(lat2)
    r.w.lat = lat2
    r.P = oracle.Problem(r.w)
    check(r, scans=(B.SCAN_INDEXED,))
