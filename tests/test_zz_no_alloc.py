"""The allocation-free full-scan decision against llama_decide's FULL mode.

llama_decide_full_noalloc takes its bucketing scratch from a static per-GPU
array; its outputs must equal llama_decide(scan=FULL) bit for bit, on two
calls in a row with the second smaller, in both bucketing layouts (few ops:
per-chunk LDS histograms; many ops: global counters), and a batch beyond the
array's limit must be rejected before anything runs.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2102_01887_amd import binding as B
from paper_2102_01887_amd import workloads as wl

pytestmark = pytest.mark.gpu

PAPER, PROB = 0, 1


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def check_two_calls(w, sizes, Q=None):
    torch = _torch()
    L = B.Llama(0).load(w)
    q = None if Q is None else dev(torch, np.asarray(Q, np.int64))
    P = oracle.Problem(w)
    rng = np.random.default_rng(7)
    for mode in (PAPER, PROB):
        for n in sizes:  # the second call is smaller and must not see the first's scratch
            say(f"noalloc: n_ops {w.n_ops}, n {n}, mode {mode}, queue {Q is not None}")
            a = int(rng.integers(0, w.n_inv - n + 1))
            op, el, slo = (dev(torch, x[a:a + n]) for x in (w.inv_op, w.elapsed, w.slo))
            cfg = torch.full((n,), -7, dtype=torch.int32, device="cuda")
            flag = torch.full((n,), 9, dtype=torch.uint8, device="cuda")
            L.decide_full_noalloc(op, el, slo, cfg, flag, queue=q, mode=mode)
            c_ref, f_ref = L.decide(op, el, slo, q, mode, B.SCAN_FULL)
            torch.cuda.synchronize()
            assert np.array_equal(cfg.cpu().numpy(), c_ref.cpu().numpy())
            assert np.array_equal(flag.cpu().numpy(), f_ref.cpu().numpy())
            sl = slice(a, a + min(n, 5000))
            c_or, f_or = P.decide(mode, Q=Q, sl=sl)
            assert np.array_equal(cfg.cpu().numpy()[:len(c_or)], c_or)
            assert np.array_equal(flag.cpu().numpy()[:len(f_or)], f_or)
    L.close()


def test_noalloc_few_ops_matches_full_scan():
    # about 1,600 ops: the per-chunk LDS histogram layout, several chunks and a ragged tail
    w = wl.make_c2(seed=41, n_pipelines=64, n_inv=120_000)
    check_two_calls(w, (100_001, 17_389), Q=[300, 0, 12_000, 70])


def test_noalloc_many_ops_matches_full_scan():
    # more than 12,288 ops: counts by global atomics, scatter by cursors
    w = wl.make_c3(seed=42, n_pipelines=320, n_inv=90_000, max_cfg=256)
    assert w.n_ops > 12_288
    check_two_calls(w, (80_003, 1_111))


def test_noalloc_rejects_batches_beyond_the_limit():
    torch = _torch()
    w = wl.make_c1(n_inv=1000)
    L = B.Llama(0).load(w)
    lib = L._L
    per = lib.llama_decide_full_noalloc_words(1, w.n_ops)
    n = 1
    while lib.llama_decide_full_noalloc_words(n, w.n_ops) * 4 <= 32 << 20:
        n *= 2
    assert per > 0 and n <= 1 << 24
    op = torch.zeros(n, dtype=torch.int32, device="cuda")
    cfg = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    with pytest.raises(B.LlamaError, match="limit"):
        L.decide_full_noalloc(op, op, op, cfg)
    torch.cuda.synchronize()
    assert int((cfg != -7).sum()) == 0     # nothing was launched
    # a batch within the limit still works afterwards
    c, f = L.decide_full_noalloc(*(dev(torch, x) for x in (w.inv_op, w.elapsed, w.slo)),
                                 torch.empty(w.n_inv, dtype=torch.int32, device="cuda"),
                                 torch.empty(w.n_inv, dtype=torch.uint8, device="cuda"))
    torch.cuda.synchronize()
    c_or, f_or = oracle.Problem(w).decide(PAPER)
    assert np.array_equal(c.cpu().numpy(), c_or) and np.array_equal(f.cpu().numpy(), f_or)
    L.close()
