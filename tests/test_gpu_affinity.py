"""GPU parity of Eq. 3 (affinity) and the commit order, through the C ABI.

Tolerance: each objective value is rounded to double once (three roundings of
relative size 2^-53: numerator, denominator, quotient) and the ratio once
more, so the GPU's ratio is within 7 * 2^-53 of the exact one and within
8 * 2^-53 < 1e-15 of the oracle's correctly rounded value; the special values
(0, 1, infinity) are exact.  The commit order is a permutation whose GPU
affinities never increase, ties in index order, and whose exact affinities
never increase by more than the tolerance.
"""
import numpy as np
import pytest

from paper_2102_01887_amd import binding as B
from paper_2102_01887_amd import workloads as wl
from test_gpu_parity import PAPER, PROB, Run, _torch, dev, say

pytestmark = pytest.mark.gpu
RTOL = 1e-15


def close(got, want):
    special = ~np.isfinite(want) | (want == 0) | (want == 1)
    assert np.array_equal(got[special], want[special])
    f = ~special
    rel = np.abs(got[f] - want[f]) / np.abs(want[f])
    assert rel.size == 0 or rel.max() <= RTOL, rel.max()


def check_order(order, aff_gpu, aff_or):
    n = aff_gpu.shape[0]
    for h in range(order.shape[0]):
        o = order[h]
        assert np.array_equal(np.sort(o), np.arange(n))
        a = aff_gpu[o, h]
        assert (a[:-1] >= a[1:]).all()
        ties = a[:-1] == a[1:]
        assert (o[:-1][ties] < o[1:][ties]).all()
        e = aff_or[o, h]
        fin = np.isfinite(e[:-1]) & np.isfinite(e[1:])
        assert (e[:-1][fin] >= e[1:][fin] * (1 - 2 * RTOL)).all()


def run_case(r, a, Q=None, modes=(PAPER, PROB), n_check=None):
    torch = r.torch
    q = None if Q is None else dev(np.asarray(Q, np.int64), torch)
    r.L.set_alpha(*a)
    for mode in modes:
        aff, order = r.L.affinity(r.op, r.el, r.slo, q, mode)
        torch.cuda.synchronize()
        aff, order = aff.cpu().numpy(), order.cpu().numpy()
        sl = slice(None) if n_check is None else slice(0, n_check)
        want = r.P.affinity(mode, *a, Q=Q, sl=sl)
        close(aff[sl], want)
        if n_check is None:
            check_order(order, aff, want)
        say(f"{r.w.name} alpha {a} mode {mode}: median affinity {np.median(aff):.3f}")


def test_affinity_c1():
    w = wl.with_resource_totals(wl.make_c1(queue=True))
    r = Run(w)
    for a in ((0, 1), (1, 1), (7, 3)):
        run_case(r, a)
        run_case(r, a, Q=w.Q, modes=(PAPER,))


def test_affinity_c2_reduced():
    w = wl.with_resource_totals(wl.make_c2(seed=61, n_pipelines=12, n_inv=4_000))
    r = Run(w)
    run_case(r, (1, 1))
    run_case(r, (1, 2), Q=[50_000, 0, 400_000, 2_000_000], modes=(PAPER,))


def test_affinity_fuzz_small_tables():
    rng = np.random.default_rng(11)
    for rep in range(8):
        w = wl.with_resource_totals(wl.random_small(rng, n_inv=600, name=f"aff{rep}"),
                                    slots=int(rng.integers(1, 5)))
        r = Run(w)
        run_case(r, (int(rng.integers(0, 6)), int(rng.integers(1, 4))))
        run_case(r, (1, 1), Q=rng.integers(0, 15_000, w.n_hw), modes=(PAPER,))


def test_affinity_without_order_and_invalid_invocations():
    w = wl.with_resource_totals(wl.make_c1())
    r = Run(w)
    r.L.set_alpha(1, 1)
    torch = r.torch
    op = w.inv_op.copy()
    op[::6] = w.n_ops
    aff, order = r.L.affinity(dev(op, torch), r.el, r.slo, with_order=False)
    torch.cuda.synchronize()
    assert order is None
    aff = aff.cpu().numpy()
    assert (aff[::6] == 0).all()
    assert r.L.stats(reset_error=True)["device_error"] & B.DEVERR_INVALID_INVOCATION
    ok = np.ones(len(op), bool)
    ok[::6] = False
    want = r.P.affinity(PAPER, 1, 1)
    close(aff[ok], want[ok])


def test_affinity_order_with_invalid_invocations():
    # invalid invocations get zero affinities, and the commit order still
    # holds every invocation once, affinities non-increasing, ties by index
    w = wl.with_resource_totals(wl.make_c2(seed=62, n_pipelines=8, n_inv=3_000))
    r = Run(w)
    r.L.set_alpha(1, 1)
    torch = r.torch
    op = w.inv_op.copy()
    op[::7] = -1
    aff, order = r.L.affinity(dev(op, torch), r.el, r.slo)
    torch.cuda.synchronize()
    aff, order = aff.cpu().numpy(), order.cpu().numpy()
    assert r.L.stats(reset_error=True)["device_error"] & B.DEVERR_INVALID_INVOCATION
    want = r.P.affinity(PAPER, 1, 1)
    want[::7] = 0.0
    close(aff, want)
    check_order(order, aff, want)


def test_affinity_c3_many_ops_grouped():
    # more ops than one LDS histogram holds, far more configurations than
    # invocations: the invocations are grouped by op in two levels and
    # counted per backend, with and without queueing times
    w = wl.with_resource_totals(wl.make_c3(seed=63, n_pipelines=320, n_inv=20_000, max_cfg=2048))
    assert w.n_ops > 12288 and 8 * w.n_inv < w.n_cfg
    r = Run(w)
    run_case(r, (1, 1), modes=(PAPER,))
    run_case(r, (3, 2), Q=[50_000, 0, 400_000, 2_000_000], modes=(PAPER,))


def test_affinity_captured_before_any_scratch():
    # captured into a graph on a fresh context, before any call has grown the
    # grouping scratch: the static merged order without queueing times, one
    # thread per invocation with them (no allocation under capture); every
    # replay checked
    torch = _torch()
    w = wl.with_resource_totals(wl.make_c3(seed=64, n_pipelines=40, n_inv=2000, max_cfg=512))
    assert 8 * w.n_inv < w.n_cfg
    r = Run(w)
    r.L.set_alpha(1, 1)
    s = torch.cuda.Stream()
    for Q in (None, [50_000, 0, 400_000, 2_000_000]):
        q = None if Q is None else dev(np.asarray(Q, np.int64), torch)
        aff = torch.empty((w.n_inv, w.n_hw), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            r.L.affinity(r.op, r.el, r.slo, q, PAPER, aff=aff, with_order=False, stream=s)
        want = r.P.affinity(PAPER, 1, 1, Q=Q)
        for _ in range(2):
            aff.fill_(-1.0)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            close(aff.cpu().numpy(), want)


def test_affinity_needs_alpha():
    r = Run(wl.with_resource_totals(wl.make_c1()))
    with pytest.raises(B.LlamaError):
        r.L.affinity(r.op, r.el, r.slo)


def test_affinity_large_op_fallback_and_static_order():
    # one op with more configurations than the per-call merge takes (4,096):
    # with queueing times the per-backend searches, without them the static
    # merged order; both must match the oracle
    from test_oracle_affinity import single_op
    rng = np.random.default_rng(12)
    n = 5000
    w = single_op(rng.integers(0, 3, n), rng.integers(1, 9, n), rng.integers(1, 5, n),
                  rng.integers(1, 400_000, n), rng.integers(1, 10_000, n), 3, [40, 30, 20],
                  slo=rng.integers(1, 800_000, 2000), elapsed=rng.integers(0, 1000, 2000))
    r = Run(w)
    run_case(r, (1, 1), Q=[50_000, 0, 300_000], modes=(PAPER,))
    run_case(r, (2, 3))
