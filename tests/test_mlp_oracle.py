"""Pins for the surrogate oracle (oracle/mlp.py), no GPU.

  * BF16 rounding equals torch's float32 -> bfloat16 conversion;
  * the tanh-form GELU stays within its known approximation error of the exact
    erf-form GELU, and its derivative matches central differences;
  * the backward pass (without rounding emulation) matches central finite
    differences of the loss in FP64, for every parameter tensor;
  * the pinball-loss gradient has the right sign convention;
  * AdamW matches torch.optim.AdamW step for step;
  * decisions: a perfect surrogate has zero regret and no misses; the
    spread rule falls back to the profile.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import mlp


def test_bf16_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10 ** rng.uniform(-8, 8, 20000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 3.0e38, -3.0e38, 1e-40]])
    want = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    got = mlp.bf16(x)
    assert np.array_equal(got, want)
    bits = mlp.bf16_bits(x)
    assert np.array_equal(mlp.from_bf16_bits(bits), want)


def test_gelu_tanh_form_against_erf_form():
    xs = np.linspace(-8, 8, 20001)
    exact = np.array([0.5 * x * (1 + math.erf(x / math.sqrt(2))) for x in xs])
    assert np.max(np.abs(mlp.gelu(xs) - exact)) < 1e-3
    # and it is not a cruder approximation
    assert np.max(np.abs(mlp.gelu(xs) - exact)) < 5e-4


def test_gelu_grad_against_central_differences():
    xs = np.linspace(-6, 6, 1001)
    h = 1e-6
    fd = (mlp.gelu(xs + h) - mlp.gelu(xs - h)) / (2 * h)
    assert np.max(np.abs(mlp.gelu_grad(xs) - fd)) < 1e-7


def small_params(rng, n_rows=5, scale=0.3):
    p = {k: rng.standard_normal(s) * scale for k, s in mlp.shapes(n_rows).items()}
    p["b3"] = np.array([2.0, 2.4])
    return p


def test_backward_against_finite_differences():
    rng = np.random.default_rng(1)
    n_rows = 5
    p = small_params(rng, n_rows)
    B = 7
    rows = rng.integers(0, n_rows, B)
    feat = rng.uniform(0, 1, (B, mlp.FEAT))
    y = rng.uniform(1.0, 3.5, B)
    _, g = mlp.loss_and_grads(p, rows, feat, y, emulate=False)
    h = 1e-6
    for k in mlp.NAMES:
        flat = p[k].ravel()
        for idx in rng.choice(flat.size, min(flat.size, 12), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = mlp.loss_and_grads(p, rows, feat, y, emulate=False)
            flat[idx] = old - h
            lm, _ = mlp.loss_and_grads(p, rows, feat, y, emulate=False)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(g[k].ravel()[idx] - fd) <= 1e-6 + 1e-5 * abs(fd), (k, idx)


def test_pinball_gradient_sign():
    # one row, q below y: increasing q lowers the loss (gradient -tau);
    # q above y: gradient 1 - tau
    out = np.array([[1.0, 0.5]])
    d = lambda q: (mlp.loss_terms(np.array([[1.0, q + 1e-7]]), np.array([1.0]))
                   - mlp.loss_terms(np.array([[1.0, q - 1e-7]]), np.array([1.0])))[0] / 2e-7
    assert abs(d(0.5) - (-0.95)) < 1e-6
    assert abs(d(1.5) - 0.05) < 1e-6
    assert mlp.loss_terms(out, np.array([1.0]))[0] == pytest.approx(0.5 * 0.95)


def test_adamw_matches_torch():
    rng = np.random.default_rng(2)
    n_rows = 4
    p = small_params(rng, n_rows)
    tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    lr, wd = 3e-3, 0.1
    opt = torch.optim.AdamW([{"params": [tp[k] for k in mlp.DECAYED], "weight_decay": wd},
                             {"params": [tp[k] for k in mlp.NAMES if k not in mlp.DECAYED],
                              "weight_decay": 0.0}], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(x) for k, x in p.items()}
    for step in range(1, 6):
        g = {k: rng.standard_normal(x.shape) for k, x in p.items()}
        for k in mlp.NAMES:
            tp[k].grad = torch.tensor(g[k])
        opt.step()
        mlp.adamw_step(p, g, m, v, step, lr, wd)
        for k in mlp.NAMES:
            assert np.allclose(p[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-14), (step, k)


def test_zero_output_weights_give_the_bias():
    rng = np.random.default_rng(3)
    p = small_params(rng)
    p["W3"][:] = 0.0
    c = mlp.forward(p, rng.integers(0, 5, 9), rng.uniform(0, 1, (9, 16)))
    assert np.all(c["out"] == p["b3"])


def test_spread_rule_and_perfect_surrogate():
    out = np.array([[5.0, 5.5], [5.0, 4.0], [5.0, 9.0], [np.nan, 5.0]])
    L, ok = mlp.predicted_latency(out, np.array([7, 8, 9, 10]), spread_max=math.log(4))
    assert ok.tolist() == [True, False, False, False]
    assert L.tolist() == [math.ceil(math.exp(5.5)), 8, 9, 10]
    # perfect surrogate: decisions made on the truth latencies have zero regret
    rng = np.random.default_rng(4)
    n, n_cfg = 200, 8
    cost = rng.integers(1, 100, n_cfg).astype(np.int64)
    batch = rng.integers(1, 4, n_cfg).astype(np.int32)
    hw = rng.integers(0, 2, n_cfg).astype(np.int32)
    truth = rng.integers(10, 1000, (n, n_cfg)).astype(np.int32)
    target = rng.integers(0, 1200, (n, 2)).astype(np.int32)
    cfg_off = np.array([0, n_cfg], np.int32)
    c, f = oracle.select_lat(np.zeros(n, np.int32), target, 2, cfg_off, hw, batch, truth, cost)
    r = mlp.regret(c, c, f, truth, target, hw, cost, batch, np.zeros(n, np.int64))
    assert r["mean_regret"] == 0.0 and r["miss_rate"] == 0.0 and r["n_feasible"] == int(f.sum())
    # a deliberately content-blind choice (all configurations assumed 10 us) misses
    blind, _ = oracle.select_lat(np.zeros(n, np.int32), target, 2, cfg_off, hw, batch,
                                 np.full((n, n_cfg), 10, np.int32), cost)
    r2 = mlp.regret(blind, c, f, truth, target, hw, cost, batch, np.zeros(n, np.int64))
    assert r2["miss_rate"] > 0.0


def test_select_lat_matches_select_for_constant_rows():
    w = __import__("paper_2102_01887_amd.workloads", fromlist=["x"]).make_c1()
    P = oracle.Problem(w)
    t = P.targets(0)
    lat_rows = np.stack([w.lat[w.cfg_off[v]:w.cfg_off[v + 1]] for v in w.inv_op])
    a = oracle.select_lat(w.inv_op, t, w.n_hw, w.cfg_off, w.hw, w.batch, lat_rows, w.cost)
    b = P.select(t)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_grad_magnitudes_bound_the_gradients():
    """The magnitude sums are at least |g| for every element and equal |g|
    where every term has one sign (a single row, one sample per embedding
    row, all-positive weights and inputs in the last layer)."""
    rng = np.random.default_rng(7)
    n_rows = 6
    p = small_params(rng, n_rows)
    rows = rng.integers(0, n_rows, 40)
    feat = rng.uniform(0, 1, (40, mlp.FEAT))
    y = rng.uniform(1.0, 3.5, 40)
    _, g = mlp.loss_and_grads(p, rows, feat, y)
    mag = mlp.grad_magnitudes(p, rows, feat, y)
    for k in mlp.NAMES:
        assert mag[k].shape == g[k].shape
        assert np.all(mag[k] >= np.abs(g[k]) * (1 - 1e-12)), k
    # one sample: the last layer's terms are single products, so equality
    _, g1 = mlp.loss_and_grads(p, rows[:1], feat[:1], y[:1])
    m1 = mlp.grad_magnitudes(p, rows[:1], feat[:1], y[:1])
    for k in ("W3", "b3"):
        assert np.allclose(m1[k], np.abs(g1[k]), rtol=1e-12, atol=0), k
