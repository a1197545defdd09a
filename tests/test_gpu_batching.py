"""GPU parity of safe delayed batching against the oracle, through the C ABI
(bit-exact: the decision is integer)."""
import numpy as np
import pytest

import oracle
from paper_2102_01887_amd import binding as B
from paper_2102_01887_amd import workloads as wl
from test_gpu_parity import PAPER, PROB, Run, _torch, dev, say

pytestmark = pytest.mark.gpu


def per_op(rng, w, hi_avail, hi_up, hi_wait):
    return (rng.integers(0, hi_avail, w.n_ops).astype(np.int32),
            rng.integers(0, hi_up, w.n_ops).astype(np.int32),
            rng.integers(0, hi_wait, w.n_ops).astype(np.int32))


def case(r, avail, up, wait, Q=None, modes=(PAPER, PROB)):
    torch = r.torch
    q = None if Q is None else dev(np.asarray(Q, np.int64), torch)
    for mode in modes:
        c, f = r.L.decide_batching(r.op, r.el, r.slo, dev(avail, torch), dev(up, torch), dev(wait, torch),
                                   q, mode)
        torch.cuda.synchronize()
        c, f = c.cpu().numpy(), f.cpu().numpy()
        c_or, f_or = r.P.decide_batching(mode, avail, up, wait, Q=Q)
        bad = np.nonzero((c != c_or) | (f != f_or))[0]
        assert bad.size == 0, f"mode {mode}: {bad.size} mismatches, first {bad[:5]}"
        say(f"{r.w.name} mode {mode}: {np.mean(c == B.CFG_WAIT):.3f} wait")


def test_batching_c1():
    w = wl.make_c1(queue=True)
    r = Run(w)
    rng = np.random.default_rng(1)
    for _ in range(3):
        a = per_op(rng, w, 9, 9, 300_000)
        case(r, *a)
        case(r, *a, Q=w.Q, modes=(PAPER,))


def test_batching_c2_reduced():
    w = wl.make_c2(seed=71, n_pipelines=16, n_inv=40_000)
    r = Run(w)
    rng = np.random.default_rng(2)
    case(r, *per_op(rng, w, 65, 65, 2_000_000))
    case(r, *per_op(rng, w, 8, 200, 500_000), Q=[10_000, 0, 100_000, 900_000], modes=(PAPER,))


def test_batching_c3_reduced():
    w = wl.make_c3(seed=72, n_pipelines=20, n_inv=20_000)
    r = Run(w)
    rng = np.random.default_rng(3)
    case(r, *per_op(rng, w, 65, 65, 2_000_000), modes=(PAPER,))


def test_batching_c3_many_ops():
    # more ops than one LDS histogram holds: the queued invocations are
    # grouped by op in two levels before the per-op scan
    w = wl.make_c3(seed=75, n_pipelines=320, n_inv=30_000, max_cfg=512)
    assert w.n_ops > 12288
    r = Run(w)
    rng = np.random.default_rng(5)
    case(r, *per_op(rng, w, 65, 65, 2_000_000))
    case(r, *per_op(rng, w, 8, 200, 500_000), Q=[10_000, 0, 100_000, 900_000], modes=(PAPER,))


def test_batching_beyond_packed_slots():
    # more sub-queue slots than a packed 24-bit position holds, over many ops:
    # the batch-limited scan takes one wavefront per slot instead of grouping
    # by op; the oracle checks a sample
    torch = _torch()
    w = wl.make_c3(seed=76, n_pipelines=320, n_inv=(1 << 24) + 4096, max_cfg=64)
    L = B.Llama(0).load(w)
    op, el, slo = dev(w.inv_op, torch), dev(w.elapsed, torch), dev(w.slo, torch)
    rng = np.random.default_rng(6)
    avail, up, wait = per_op(rng, w, 65, 65, 2_000_000)
    idx = np.sort(np.random.default_rng(1).choice(w.n_inv, 50_000, replace=False))
    idx[-1] = w.n_inv - 1
    c_or, f_or = oracle.Problem(w).decide_batching(PAPER, avail, up, wait, sl=idx)
    c, f = L.decide_batching(op, el, slo, dev(avail, torch), dev(up, torch), dev(wait, torch), None, PAPER)
    torch.cuda.synchronize()
    c, f = c.cpu().numpy(), f.cpu().numpy()
    assert np.array_equal(c[idx], c_or) and np.array_equal(f[idx], f_or)


def test_batching_fuzz_small_tables():
    rng = np.random.default_rng(4)
    for rep in range(10):
        w = wl.random_small(rng, n_inv=1000, name=f"sdb{rep}")
        r = Run(w)
        case(r, *per_op(rng, w, 6, 6, 3000))
        case(r, *per_op(rng, w, 6, 6, 3000), Q=rng.integers(0, 10_000, w.n_hw), modes=(PAPER,))


def test_batching_plenty_available_is_plain_decide_and_invalid():
    w = wl.make_c2(seed=73, n_pipelines=6, n_inv=5000)
    r = Run(w)
    torch = r.torch
    big = np.full(w.n_ops, 1 << 20, np.int32)
    zero = np.zeros(w.n_ops, np.int32)
    c, f = r.L.decide_batching(r.op, r.el, r.slo, dev(big, torch), dev(zero, torch), dev(zero, torch))
    c0, f0 = r.L.decide(r.op, r.el, r.slo, scan=B.SCAN_INDEXED)
    torch.cuda.synchronize()
    assert np.array_equal(c.cpu().numpy(), c0.cpu().numpy()) and np.array_equal(f.cpu().numpy(), f0.cpu().numpy())
    op = w.inv_op.copy()
    op[::5] = -3
    c, f = r.L.decide_batching(dev(op, torch), r.el, r.slo, dev(big, torch), dev(zero, torch), dev(zero, torch))
    torch.cuda.synchronize()
    assert (c.cpu().numpy()[::5] == -1).all()
    assert r.L.stats(reset_error=True)["device_error"] & B.DEVERR_INVALID_INVOCATION


def test_batching_scratch_grows_on_one_context():
    # the queue scratch is sized by the first call and grows with a larger
    # batch; each call's decisions must match the oracle's
    w = wl.make_c2(seed=74, n_pipelines=10, n_inv=30_001)
    r = Run(w)
    torch = r.torch
    rng = np.random.default_rng(5)
    avail, up, wait = per_op(rng, w, 40, 40, 1_000_000)
    for n in (1000, 30_001, 257):
        ws = w.with_invocations(w.inv_op[:n], w.elapsed[:n], w.slo[:n])
        c, f = r.L.decide_batching(dev(ws.inv_op, torch), dev(ws.elapsed, torch), dev(ws.slo, torch),
                                   dev(avail, torch), dev(up, torch), dev(wait, torch))
        torch.cuda.synchronize()
        c_or, f_or = oracle.Problem(ws).decide_batching(PAPER, avail, up, wait)
        assert np.array_equal(c.cpu().numpy(), c_or) and np.array_equal(f.cpu().numpy(), f_or), n
