"""Serving loop: continuous batching, memory-based admission, latency.

Each decision depends only on its own invocation, so a request's result must
be the same decided alone as in any mix; this is checked bit-exactly in both
the plain and the learned modes, and every served decision is checked
against the CPU oracle: Alg. 1 + Eq. 1 in the plain form, Eq. 1 over the
GPU's own predicted latencies in the learned form.
"""
import math
import sys
import time

import numpy as np
import pytest

import oracle
from paper_2102_01887_amd import binding as B
from paper_2102_01887_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def serve_all(srv, op, el, slo, feat=None, rng=None):
    """Offer every request in random bursts, collecting as they finish."""
    rng = rng or np.random.default_rng(0)
    n = len(op)
    i = 0
    got_t, got_c, got_f = [], [], []
    while i < n or sum(len(x) for x in got_t) < n:
        if i < n:
            j = min(n, i + int(rng.integers(1, 3000)))
            k, _ = srv.submit(op[i:j], el[i:j], slo[i:j], None if feat is None else feat[i:j])
            i += k
        t, c, f, _ = srv.poll(wait_ms=1 if i >= n else 0)
        got_t.append(t)
        got_c.append(c)
        got_f.append(f)
    return np.concatenate(got_t), np.concatenate(got_c), np.concatenate(got_f)


def test_plain_mix_equals_alone():
    torch = _torch()
    w = wl.make_c2(seed=21, n_pipelines=32, n_inv=60_000)
    L = B.Llama(0).load(w)
    srv = B.Server(L, n_slots=4096, max_batch=1024, max_inflight=4)
    t, c, f = serve_all(srv, w.inv_op, w.elapsed, w.slo)
    st = srv.stats()
    srv.close()
    say(f"plain serving stats: {st}")
    assert np.array_equal(t, np.arange(w.n_inv))          # each request exactly once, in order
    assert st["batches"] > 1 and st["max_batch_seen"] <= 1024
    c_or, f_or = oracle.Problem(w).decide(0)
    assert np.array_equal(c, c_or) and np.array_equal(f, f_or)
    c_all, f_all = L.decide(dev(torch, w.inv_op), dev(torch, w.elapsed), dev(torch, w.slo))
    torch.cuda.synchronize()
    assert np.array_equal(c, c_all.cpu().numpy()) and np.array_equal(f, f_all.cpu().numpy())
    for i in np.random.default_rng(1).choice(w.n_inv, 50, replace=False):
        ca, fa = L.decide(dev(torch, w.inv_op[i:i + 1]), dev(torch, w.elapsed[i:i + 1]),
                          dev(torch, w.slo[i:i + 1]))
        torch.cuda.synchronize()
        assert (ca.item(), fa.item()) == (c[i], f[i])


def test_learned_mix_equals_alone():
    torch = _torch()
    world = wl.make_c4_world(3)
    L = B.Llama(0).load(world.w)
    L.surrogate_init(seed=5, mean_log_latency=10.5)
    w, content = wl.c4_invocations(world, np.random.default_rng(2), 20_000)
    feat_bits = (np.ascontiguousarray(content.feat, np.float32).view(np.uint32) >> 16).astype(np.uint16)
    srv = B.Server(L, n_slots=2048, max_batch=512, max_inflight=3, learned=True)
    t, c, f = serve_all(srv, w.inv_op, w.elapsed, w.slo, feat_bits)
    srv.close()
    assert np.array_equal(t, np.arange(w.n_inv))
    feat_t = dev(torch, feat_bits.view(np.int16))
    lat = torch.empty(w.n_inv * 64, dtype=torch.int32, device="cuda")
    c_all, f_all = L.decide_learned(dev(torch, w.inv_op), dev(torch, w.elapsed), dev(torch, w.slo),
                                    feat_t, lat_out=lat, lat_stride=64)
    torch.cuda.synchronize()
    assert np.array_equal(c, c_all.cpu().numpy()) and np.array_equal(f, f_all.cpu().numpy())
    # the oracle's Eq. 1 over the GPU's predicted latencies and the oracle's own targets
    tgt = oracle.Problem(w).targets(0)
    c_or, f_or = oracle.select_lat(w.inv_op, tgt, w.n_hw, w.cfg_off, w.hw, w.batch,
                                   lat.cpu().numpy().reshape(w.n_inv, 64), w.cost)
    assert np.array_equal(c, c_or) and np.array_equal(f, f_or)
    for i in np.random.default_rng(3).choice(w.n_inv, 20, replace=False):
        ca, fa = L.decide_learned(dev(torch, w.inv_op[i:i + 1]), dev(torch, w.elapsed[i:i + 1]),
                                  dev(torch, w.slo[i:i + 1]), feat_t[i:i + 1])
        torch.cuda.synchronize()
        assert (ca.item(), fa.item()) == (c[i], f[i])


def test_memory_admission():
    _torch()
    w = wl.make_c1(n_inv=1000)
    L = B.Llama(0).load(w)
    bpr = L._L.llama_serve_bytes_per_request(0)
    srv = B.Server(L, n_slots=4096, mem_budget_bytes=100 * bpr, max_batch=64)
    k, tickets = srv.submit(w.inv_op, w.elapsed, w.slo)
    assert k == 100 and np.array_equal(tickets, np.arange(100))
    k2, _ = srv.submit(w.inv_op[:5], w.elapsed[:5], w.slo[:5])
    assert k2 == 0                                       # budget full until results are collected
    done = 0
    while done < 100:
        t, _, _, _ = srv.poll(wait_ms=50)
        done += len(t)
    k3, t3 = srv.submit(w.inv_op[100:300], w.elapsed[100:300], w.slo[100:300])
    assert k3 == 100 and t3[0] == 100
    while done < 200:
        t, _, _, _ = srv.poll(wait_ms=50)
        done += len(t)
    st = srv.stats()
    srv.close()
    # the ring holds what the budget buys: 100 slots of the 4,096 asked for
    assert st["capacity"] == 100 and bpr == 32
    assert st["peak_bytes_in_use"] <= 100 * bpr and st["rejected"] == 900 + 5 + 100


def drive_poisson(srv, w, rate, duration, seed=0):
    """Offer w's invocations as a Poisson stream; returns latencies (ns) and
    the sustained rate."""
    rng = np.random.default_rng(seed)
    off = wl.poisson_arrivals(rng, rate, duration)
    n = min(len(off), w.n_inv)
    off = off[:n]
    t0 = time.monotonic_ns() + 2_000_000
    arr = t0 + off
    i = done = 0
    lats = []
    while done < n:
        now = time.monotonic_ns()
        j = int(np.searchsorted(arr, now, side="right"))
        if j > i:
            k, _ = srv.submit(w.inv_op[i:j], w.elapsed[i:j], w.slo[i:j], arrival_ns=arr[i:j])
            i += k
        t, _, _, lat = srv.poll(wait_ms=0)
        done += len(t)
        lats.append(lat)
    t_end = time.monotonic_ns()
    lat = np.concatenate(lats)
    return lat, n / ((t_end - t0) * 1e-9)


def test_poisson_stream_latency():
    _torch()
    w = wl.make_c2(seed=22, n_pipelines=64, n_inv=200_000)
    L = B.Llama(0).load(w)
    srv = B.Server(L, n_slots=65536, max_batch=65536, max_inflight=4)
    lat, rate = drive_poisson(srv, w, 100_000, 0.5)
    st = srv.stats()
    srv.close()
    p50, p99 = np.percentile(lat, [50, 99]) / 1e3
    say(f"poisson 100k/s: {len(lat)} decisions, p50 {p50:.1f} us, p99 {p99:.1f} us, sustained {rate:.0f}/s, {st}")
    assert len(lat) > 30_000 and (lat > 0).all() and p99 < 1e6


def test_relaunch_after_idle_exit():
    # the persistent kernel exits after 20 ms without work; requests published
    # later must start it again, and decisions keep matching the oracle
    _torch()
    w = wl.make_c2(seed=23, n_pipelines=16, n_inv=3000)
    L = B.Llama(0).load(w)
    srv = B.Server(L, n_slots=1024, max_batch=64, max_inflight=2)
    got_c, got_f = [], []
    for part in range(3):
        sl = slice(1000 * part, 1000 * (part + 1))
        k, _ = srv.submit(w.inv_op[sl], w.elapsed[sl], w.slo[sl])
        assert k == 1000
        n = 0
        while n < 1000:
            t, c, f, lat = srv.poll(wait_ms=100)
            assert (lat > 0).all() and (lat < 1_000_000_000).all()
            n += len(t)
            got_c.append(c)
            got_f.append(f)
        time.sleep(0.06)
    st = srv.stats()
    srv.close()
    say(f"relaunch: {st}")
    assert st["kernel_launches"] >= 3 and st["decided"] == 3000 and st["in_flight_batches"] == 0
    assert 0 <= st["clock_rtt_ns"] < 1_000_000
    c_or, f_or = oracle.Problem(w).decide(0)
    assert np.array_equal(np.concatenate(got_c), c_or) and np.array_equal(np.concatenate(got_f), f_or)


def test_latency_clock_does_not_drift():
    # isolated requests for 0.6 s: the device-stamped latency must not grow
    # with the time since open (the device clock is re-anchored to the host's
    # while the kernel runs), and every latency is positive
    _torch()
    w = wl.make_c2(seed=24, n_pipelines=16, n_inv=2000)
    L = B.Llama(0).load(w)
    srv = B.Server(L, n_slots=1024, max_batch=64, max_inflight=2)
    lat, when = [], []
    t_start = time.monotonic_ns()
    i = 0
    while time.monotonic_ns() - t_start < 6e8:
        t0 = time.monotonic_ns()
        k, _ = srv.submit(w.inv_op[i:i + 1], w.elapsed[i:i + 1], w.slo[i:i + 1])
        assert k == 1
        n = 0
        while n == 0:
            t, c, f, l = srv.poll(wait_ms=100)
            n = len(t)
            lat.extend(l.tolist())
        when.append((t0 - t_start) * 1e-9)
        i = (i + 1) % 2000
        while time.monotonic_ns() - t0 < 1_000_000:
            pass
    st = srv.stats()
    srv.close()
    lat, when = np.asarray(lat) / 1e3, np.asarray(when)
    early, late = np.median(lat[when < 0.15]), np.median(lat[when > 0.45])
    say(f"isolated requests: {len(lat)}, p50 first 0.15 s {early:.1f} us, last 0.15 s {late:.1f} us; {st}")
    assert (lat > 0).all()
    assert abs(late - early) < 15.0
    assert st["clock_anchors"] >= 10 and abs(st["clock_rate_ppb"]) < 2_000_000
