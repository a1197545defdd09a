"""GPU parity of Eq. 2 (queueing time) and the finite-alpha Eq. 1 objective
against the CPU oracle, through the C ABI.  Everything is integer: bit-exact.
"""
import numpy as np
import pytest

import oracle
from paper_2102_01887_amd import binding as B
from paper_2102_01887_amd import workloads as wl
from test_gpu_parity import PAPER, PROB, Run, _torch, dev, say

pytestmark = pytest.mark.gpu

ALPHAS = ((0, 1), (1, 1), (1, 1000), (7, 3), (2**32 - 1, 1), (1, 2**32 - 1))


def queue_case(r, q_op, q_cfg):
    torch = r.torch
    Q = r.L.queue_time(dev(q_op, torch), dev(q_cfg, torch))
    torch.cuda.synchronize()
    return Q.cpu().numpy()


@pytest.mark.parametrize("maker", ["c1", "c2", "c3"])
def test_queue_time_matches_oracle(maker):
    w = {"c1": lambda: wl.make_c1(),
         "c2": lambda: wl.make_c2(seed=41, n_pipelines=32, n_inv=50_000),
         "c3": lambda: wl.make_c3(seed=42, n_pipelines=40, n_inv=50_000)}[maker]()
    w = wl.with_resource_totals(w)
    r = Run(w)
    rng = np.random.default_rng(5)
    for n_q in (0, 1, 63, 64, 65, 1000, 250_001):
        q_op, q_cfg = wl.queue_snapshot(w, rng, n_q)
        got = queue_case(r, q_op, q_cfg)
        want, skipped = r.P.queue_time(q_op, q_cfg)
        assert skipped == 0
        assert np.array_equal(got, want), (n_q, got, want)
    say(f"{maker}: Q = {got.tolist()}")
    assert r.L.stats()["device_error"] == 0


def test_queue_time_exact_beyond_64_bits_and_cap():
    # one op with two configurations whose L * R is close to 2^62: a few
    # thousand queued copies exceed 2^64 (and, on backend 0 with R_total 1,
    # the 2^62 cap)
    w = wl.make_c1()
    w.lat = np.full(w.n_cfg, 2**31 - 1, np.int32)
    w.res = np.full(w.n_cfg, 2**31 - 7, np.int32)
    w = wl.with_resource_totals(w, per_hw=[1, 3])
    r = Run(w)
    rng = np.random.default_rng(6)
    for n_q in (3, 5000, 70_000):
        q_op, q_cfg = wl.queue_snapshot(w, rng, n_q)
        got = queue_case(r, q_op, q_cfg)
        want, _ = r.P.queue_time(q_op, q_cfg)
        assert np.array_equal(got, want), (n_q, got, want)
    assert got[0] == 2**62


def test_queue_time_invalid_entries_are_skipped_and_flagged():
    w = wl.with_resource_totals(wl.make_c1())
    r = Run(w)
    rng = np.random.default_rng(7)
    q_op, q_cfg = wl.queue_snapshot(w, rng, 500)
    bad_op, bad_cfg = q_op.copy(), q_cfg.copy()
    bad_op[::7] = w.n_ops + 3
    bad_cfg[3::11] = 999
    bad_op[5::13] = -2
    got = queue_case(r, bad_op, bad_cfg)
    want, skipped = r.P.queue_time(bad_op, bad_cfg)
    assert skipped > 0 and np.array_equal(got, want)
    assert r.L.stats(reset_error=True)["device_error"] & B.DEVERR_INVALID_QUEUE_ENTRY


def test_queue_time_needs_resource_totals():
    r = Run(wl.make_c1())
    with pytest.raises(B.LlamaError):
        r.L.queue_time(dev(np.zeros(3, np.int32), r.torch), dev(np.zeros(3, np.int32), r.torch))
    with pytest.raises(B.LlamaError):
        r.L.set_alpha(1, 1)


def alpha_parity(r, Q=None, modes=(PAPER, PROB), alphas=ALPHAS):
    torch = r.torch
    q = None if Q is None else dev(np.asarray(Q, np.int64), torch)
    for a in alphas:
        r.L.set_alpha(*a)
        for mode in modes:
            c, f = r.L.decide_alpha(r.op, r.el, r.slo, q, mode)
            torch.cuda.synchronize()
            c, f = c.cpu().numpy(), f.cpu().numpy()
            c_or, f_or = r.P.decide_alpha(mode, *a, Q=Q)
            bad = np.nonzero((c != c_or) | (f != f_or))[0]
            assert bad.size == 0, f"alpha {a} mode {mode}: {bad.size} mismatches, first {bad[:5]}"
            say(f"{r.w.name} alpha {a} mode {mode}: {f.mean():.3f} meet their slack")


def test_alpha_c1_with_and_without_queue():
    w = wl.with_resource_totals(wl.make_c1(queue=True))
    r = Run(w)
    alpha_parity(r)
    alpha_parity(r, Q=w.Q)


def test_alpha_c2_reduced():
    w = wl.with_resource_totals(wl.make_c2(seed=43, n_pipelines=24, n_inv=40_000))
    r = Run(w)
    alpha_parity(r, alphas=ALPHAS[:4])
    alpha_parity(r, Q=[30_000, 0, 200_000, 5_000_000], modes=(PAPER,), alphas=ALPHAS[1:3])


def test_alpha_c3_reduced():
    w = wl.with_resource_totals(wl.make_c3(seed=44, n_pipelines=30, n_inv=30_000))
    r = Run(w)
    alpha_parity(r, modes=(PAPER,), alphas=((1, 1), (3, 2)))


def test_alpha_c3_many_ops_grouped():
    # more ops than one LDS histogram holds and far more configurations than
    # invocations: with queueing times the per-backend counts (no per-call
    # merge) after grouping the invocations by op in two levels; without,
    # one search per invocation in the op's merged run
    w = wl.with_resource_totals(wl.make_c3(seed=47, n_pipelines=320, n_inv=20_000, max_cfg=2048))
    assert w.n_ops > 12288 and 8 * w.n_inv < w.n_cfg
    r = Run(w)
    alpha_parity(r, modes=(PAPER,), alphas=((1, 1), (3, 2)))
    alpha_parity(r, Q=[30_000, 0, 200_000, 5_000_000], alphas=((1, 1),))


def test_alpha_captured_before_any_scratch():
    # captured into a graph on a fresh context, before any call has grown the
    # scratch that grouping by op needs: with queueing times one thread per
    # invocation instead (no allocation under capture), and the merged search
    # without; every replay checked
    torch = _torch()
    w = wl.with_resource_totals(wl.make_c3(seed=49, n_pipelines=40, n_inv=2000, max_cfg=512))
    assert 8 * w.n_inv < w.n_cfg
    r = Run(w)
    r.L.set_alpha(1, 1)
    n = w.n_inv
    s = torch.cuda.Stream()
    for Q in (None, [30_000, 0, 200_000, 5_000_000]):
        q = None if Q is None else dev(np.asarray(Q, np.int64), torch)
        cfg = torch.empty(n, dtype=torch.int32, device="cuda")
        flag = torch.empty(n, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            r.L.decide_alpha(r.op, r.el, r.slo, q, PAPER, cfg=cfg, flag=flag, stream=s)
        c_or, f_or = r.P.decide_alpha(PAPER, 1, 1, Q=Q)
        for _ in range(2):
            cfg.fill_(-7)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(cfg.cpu().numpy(), c_or) and np.array_equal(flag.cpu().numpy(), f_or), Q


def test_grouping_with_few_invocations_over_many_ops():
    # five invocations (one invalid) over more ops than one LDS histogram
    # holds: the two-level counting sort with nearly every op empty, for the
    # full scan, the finite-alpha decision with queueing times and the
    # affinities
    from test_gpu_affinity import close
    torch = _torch()
    base = wl.with_resource_totals(wl.make_c3(seed=50, n_pipelines=320, n_inv=1000, max_cfg=256))
    assert base.n_ops > 12288
    op = np.array([base.n_ops - 1, 0, base.n_ops // 2, base.n_ops + 3, 12288], np.int32)
    slo = np.array([900_000, 50_000, 2_000_000, 10, 400_000], np.int32)
    el = np.array([1000, 40_000, 0, 0, 399_000], np.int32)
    w = base.with_invocations(op, el, slo)
    L = B.Llama(0).load(w)
    P = oracle.Problem(w)
    ok = np.arange(5) != 3
    d_op, d_el, d_slo = dev(op, torch), dev(el, torch), dev(slo, torch)
    c, f = L.decide(d_op, d_el, d_slo, mode=PAPER, scan=B.SCAN_FULL)
    c_or, f_or = P.decide(PAPER, sl=np.flatnonzero(ok))
    c, f = c.cpu().numpy(), f.cpu().numpy()
    assert c[3] == -1 and np.array_equal(c[ok], c_or) and np.array_equal(f[ok], f_or)
    L.set_alpha(1, 1)
    Q = [30_000, 0, 200_000, 5_000_000]
    c, f = L.decide_alpha(d_op, d_el, d_slo, dev(np.asarray(Q, np.int64), torch), PAPER)
    c_or, f_or = P.decide_alpha(PAPER, 1, 1, Q=Q, sl=np.flatnonzero(ok))
    c, f = c.cpu().numpy(), f.cpu().numpy()
    assert c[3] == -1 and np.array_equal(c[ok], c_or) and np.array_equal(f[ok], f_or)
    aff, order = L.affinity(d_op, d_el, d_slo)
    aff, order = aff.cpu().numpy(), order.cpu().numpy()
    assert (aff[3] == 0).all()
    close(aff[ok], P.affinity(PAPER, 1, 1, sl=np.flatnonzero(ok)))
    assert all(sorted(order[h]) == list(range(5)) for h in range(w.n_hw))
    L.stats(reset_error=True)


def test_alpha_fuzz_small_tables():
    rng = np.random.default_rng(8)
    for rep in range(12):
        w = wl.with_resource_totals(wl.random_small(rng, n_inv=2000, name=f"fuzz{rep}"),
                                    per_hw=None, slots=int(rng.integers(1, 6)))
        r = Run(w)
        alpha_parity(r, alphas=((0, 1), (1, 2), (5, 1)))
        Q = rng.integers(0, 40, w.n_hw)
        alpha_parity(r, Q=Q, modes=(PAPER,), alphas=((1, 1),))


def test_alpha_invalid_invocations_and_empty_batch():
    w = wl.with_resource_totals(wl.make_c1())
    r = Run(w)
    r.L.set_alpha(1, 1)
    torch = r.torch
    op = w.inv_op.copy()
    el = w.elapsed.copy()
    op[::5] = w.n_ops
    el[1::7] = -1
    c, f = r.L.decide_alpha(dev(op, torch), dev(el, torch), r.slo)
    torch.cuda.synchronize()
    c, f = c.cpu().numpy(), f.cpu().numpy()
    P = oracle.Problem(w.with_invocations(op, el, w.slo))
    c_or, f_or = P.decide_alpha(PAPER, 1, 1)
    assert np.array_equal(c, c_or) and np.array_equal(f, f_or)
    assert (c[::5] == -1).all()
    assert r.L.stats(reset_error=True)["device_error"] & B.DEVERR_INVALID_INVOCATION
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    r.L.decide_alpha(e, e, e)


def test_alpha_tables_follow_latency_updates():
    w = wl.with_resource_totals(wl.make_c2(seed=45, n_pipelines=8, n_inv=20_000))
    r = Run(w)
    r.L.set_alpha(2, 1)
    rng = np.random.default_rng(9)
    lat2 = np.maximum(1, (w.lat * rng.uniform(0.5, 1.5, w.n_cfg))).astype(np.int32)
    r.L.update_latencies(lat2)
    w2 = w.with_invocations(w.inv_op, w.elapsed, w.slo)
    w2.lat = lat2
    r.P = oracle.Problem(w2)
    c, f = r.L.decide_alpha(r.op, r.el, r.slo)
    r.torch.cuda.synchronize()
    c_or, f_or = r.P.decide_alpha(PAPER, 2, 1)
    assert np.array_equal(c.cpu().numpy(), c_or) and np.array_equal(f.cpu().numpy(), f_or)


def test_queue_time_feeds_decide_alpha_on_device():
    # the chain of Sec. 4.3: Q from the queued invocations' configurations,
    # then Alg. 1 with that Q and the finite-alpha Eq. 1, without leaving the GPU
    w = wl.with_resource_totals(wl.make_c2(seed=46, n_pipelines=16, n_inv=30_000), slots=256)
    r = Run(w)
    torch = r.torch
    rng = np.random.default_rng(10)
    q_op, q_cfg = wl.queue_snapshot(w, rng, 200)
    r.L.set_alpha(1, 4)
    Q = r.L.queue_time(dev(q_op, torch), dev(q_cfg, torch))
    c, f = r.L.decide_alpha(r.op, r.el, r.slo, Q)
    torch.cuda.synchronize()
    Q_or, _ = r.P.queue_time(q_op, q_cfg)
    assert np.array_equal(Q.cpu().numpy(), Q_or)
    c_or, f_or = r.P.decide_alpha(PAPER, 1, 4, Q=Q_or)
    assert np.array_equal(c.cpu().numpy(), c_or) and np.array_equal(f.cpu().numpy(), f_or)
    say(f"chained: Q = {Q_or.tolist()}, {f_or.mean():.3f} meet their slack")


def test_alpha_queue_extremes_and_c3():
    # the per-call merged order with queueing times at the clamp's edges:
    # negative (always within reach), zero, just under and at 2^31 (never)
    w = wl.with_resource_totals(wl.make_c2(seed=45, n_pipelines=12, n_inv=20_000))
    r = Run(w)
    for Q in ([-(1 << 40), 0, (1 << 31) - 5, 1 << 31], [7, -3, 123_456, 1 << 62]):
        alpha_parity(r, Q=Q, modes=(PAPER, PROB), alphas=((1, 1),))
    w3 = wl.with_resource_totals(wl.make_c3(seed=46, n_pipelines=20, n_inv=20_000))
    alpha_parity(Run(w3), Q=[100_000, 0, 2_000_000, 40_000], modes=(PAPER,), alphas=((2, 1),))


def test_alpha_queue_fallback_for_large_ops():
    # an op with more configurations than the per-call merge takes (4,096):
    # one search per backend instead; same decisions
    from test_oracle_affinity import single_op
    rng = np.random.default_rng(47)
    n = 5000
    w = single_op(rng.integers(0, 3, n), rng.integers(1, 9, n), rng.integers(1, 5, n),
                  rng.integers(1, 400_000, n), rng.integers(1, 10_000, n), 3, [40, 30, 20],
                  slo=rng.integers(1, 800_000, 3000), elapsed=rng.integers(0, 1000, 3000))
    r = Run(w)
    alpha_parity(r, Q=[50_000, 0, 300_000], modes=(PAPER,), alphas=((1, 1),))
    alpha_parity(r, alphas=((1, 1),))
