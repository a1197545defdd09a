"""The GPU pipeline simulator (llama_simulate) against its CPU reference.

Both sides draw the same Philox4x32-10 words and apply the same transforms in
FP64, so every sample is compared one by one: configuration rows and
resolutions exactly; object counts exactly wherever the uniform is not
within 1e-9 of the cdf value it was compared with (the two sides' exp and
log may differ in the last bit); BF16 features exactly, or by one BF16 step
where the FP64 value sits at a rounding boundary; y within 1e-5.  Then the
split invariance, and training on GPU-simulated executions.
"""
import sys

import numpy as np
import pytest

from oracle import mlp
from oracle import simulator as S
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


def bits_to_f32(b):
    return (np.asarray(b).astype(np.uint16).astype(np.uint32) << 16).view(np.float32)


def test_simulator_matches_cpu_reference():
    torch = _torch()
    world = wl.make_c4_world(3)
    w = world.w
    L = B.Llama(0).load(w)
    L.set_simulator(world.a, world.b, world.sigma)
    n, seed, first = 200_000, 0x1234_5678_9ABC, 1_000_000
    rows, feat, y = L.simulate(n, seed, first)
    torch.cuda.synchronize()
    rows, feat, y = rows.cpu().numpy(), bits_to_f32(feat.cpu().numpy().view(np.uint16)), y.cpu().numpy()
    ref = S.simulate(n, seed, w.n_cfg, w.lat, w.hw, world.a, world.b, world.sigma, first=first)
    assert np.array_equal(rows, ref["rows"])
    clear = ref["margin"] > 1e-9
    say(f"simulator: {n} samples, {np.count_nonzero(~clear)} within 1e-9 of a cdf value")
    assert clear.mean() > 0.9999
    same = np.all(feat == ref["feat"], axis=1)
    # where they differ: one BF16 step, at most 1e-4 of the samples
    diff = ~same & clear
    assert diff.mean() < 1e-4
    if diff.any():
        step = np.abs(feat[diff] - ref["feat"][diff]) / np.maximum(np.abs(ref["feat"][diff]), 1e-30)
        assert (step <= 2.0 ** -7).all()
    assert np.allclose(y[clear], ref["y"][clear], rtol=0, atol=1e-5)
    # the truth mean plus noise: residuals about N(0, sigma^2)
    op = rows // 64
    resid = y.astype(np.float64) - mlp.truth_mean_log_latency(
        w.lat[rows], world.a[op, w.hw[rows]], world.b[op], ref["people"] + ref["cars"],
        np.asarray(S.RESOLUTIONS)[ref["res"]].prod(axis=1))
    assert abs(resid.mean()) < 0.01 and abs(resid.std() - world.sigma) < 0.01
    L.close()


def test_simulator_split_and_errors():
    torch = _torch()
    world = wl.make_c4_world(3)
    L = B.Llama(0).load(world.w)
    with pytest.raises(B.LlamaError):
        L.simulate(10, 1)                      # no simulator set
    L.set_simulator(world.a, world.b, world.sigma)
    r1, f1, y1 = L.simulate(5000, 99)
    r2, f2, y2 = L.simulate(3000, 99, first=2000)
    torch.cuda.synchronize()
    assert torch.equal(r1[2000:], r2) and torch.equal(f1[2000:], f2) and torch.equal(y1[2000:], y2)
    with pytest.raises(B.LlamaError):
        L.set_simulator(world.a, world.b, -1.0)
    with pytest.raises(B.LlamaError):
        L.simulate(10, 1, first=(1 << 32) - 5)
    L.close()


def test_training_on_gpu_simulated_executions():
    # the learned form trained on executions drawn on the device beats the
    # static profile on misses, as it does with host-drawn executions; the
    # training set is the 10M-sample one of the host-drawn test (with 4M
    # samples the regret sat near the bound)
    from test_gpu_surrogate import check_inference, evaluate, inference_case, setup_world
    torch, world, L = setup_world()
    L.set_simulator(world.a, world.b, world.sigma)
    L.surrogate_init(seed=15, mean_log_latency=10.5)
    n, batch = 10_000_000, 4096
    rows, feat, y = L.simulate(n, 2024)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    L.surrogate_fit(rows, feat, y, epochs=3, batch=batch, lr_max=5e-3, weight_decay=1e-4, loss_sum=loss)
    torch.cuda.synchronize()
    final = loss.item() / ((((n // batch) + 9) // 10) * batch)
    say(f"training on device-simulated executions: final loss {final:.4f}")
    w, c, tgt, cfg, flag, lat = inference_case(torch, world, L, 20_000, seed=8)
    check_inference(world, L, w, c, tgt, cfg, flag, lat)
    r_s, r_p = evaluate(world, w, c, tgt, cfg)
    say(f"surrogate: {r_s}\nplain:     {r_p}")
    assert r_s["mean_regret"] <= 0.03
    assert r_s["miss_rate"] < r_p["miss_rate"]
    L.close()
