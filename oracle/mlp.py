"""Oracle for the learned latency surrogate (test infrastructure only).

The paper profiles each configuration once and corrects profiles through a
feedback loop, noting that other estimators can replace exponential smoothing
(Sec. 3.3, Manager) and that input content changes operation latency (Sec. 2,
Fig. 3: 17.2x on CPU and 4x on GPU between 0 and 60 faces).  The surrogate is
such an estimator: a 2-hidden-layer MLP that predicts, per
(invocation, configuration) row, the mean and the 95th percentile of ln(latency
in microseconds) from a per-row embedding and 16 content features.  Nothing in
the paper fixes the network; its form, loss and optimiser are stated here.

Everything is FP64 numpy.  Where the GPU rounds to BF16 (weights, embedding,
features, both hidden activations, and the backward's output gradient and
pre-activation gradients) the oracle rounds at the same points
(round-to-nearest-even of the FP32 value), unless emulate=False.

    x   = [E[row] (16), f (16)]
    h1  = GELU(W1 x + b1)          (256)
    h2  = GELU(W2 h1 + b2)         (256)
    out = W3 h2 + b3               (2: mu, q = mean and p95 of ln L)
    loss per row = (mu - y)^2 + rho_0.95(y - q),  rho_t(u) = u (t - [u < 0])

GELU is the tanh form of Hendrycks & Gimpel (2016).
"""
import math

import numpy as np

EMB = 16
FEAT = 16
IN = EMB + FEAT
HID = 256
OUT = 2
TAU = 0.95
Z95 = 1.6448536269514722  # standard normal 0.95 quantile
GELU_C = math.sqrt(2.0 / math.pi)
GELU_A = 0.044715


# ---------------------------------------------------------------------------
# BF16
# ---------------------------------------------------------------------------

def bf16(x):
    """Round to bfloat16 (via FP32, round to nearest even); returns float64."""
    x32 = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = x32.view(np.uint32).astype(np.uint64)
    bias = 0x7FFF + ((u >> 16) & 1)
    r = ((u + bias) & 0xFFFF0000).astype(np.uint32)
    nan = np.isnan(x32)
    r = np.where(nan, u.astype(np.uint32) | 0x00400000, r)
    return r.view(np.float32).astype(np.float64)


def bf16_bits(x):
    """BF16 bit patterns (uint16) of bf16(x)."""
    return (np.ascontiguousarray(bf16(x).astype(np.float32)).view(np.uint32) >> 16).astype(np.uint16)


def from_bf16_bits(b):
    return (np.asarray(b, np.uint32) << 16).astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# GELU (tanh form) and its derivative
# ---------------------------------------------------------------------------

def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(GELU_C * (x + GELU_A * x ** 3)))


def gelu_grad(x):
    t = np.tanh(GELU_C * (x + GELU_A * x ** 3))
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * GELU_C * (1.0 + 3.0 * GELU_A * x * x)


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------

NAMES = ("E", "W1", "b1", "W2", "b2", "W3", "b3")


def shapes(n_rows):
    return {"E": (n_rows, EMB), "W1": (HID, IN), "b1": (HID,), "W2": (HID, HID), "b2": (HID,),
            "W3": (OUT, HID), "b3": (OUT,)}


def n_params(n_rows):
    return sum(int(np.prod(s)) for s in shapes(n_rows).values())


def unflatten(flat, n_rows):
    out, o = {}, 0
    for k, s in shapes(n_rows).items():
        n = int(np.prod(s))
        out[k] = np.asarray(flat[o:o + n], np.float64).reshape(s)
        o += n
    return out


def flatten(p):
    return np.concatenate([np.asarray(p[k], np.float64).ravel() for k in NAMES])


# ---------------------------------------------------------------------------
# forward / backward
# ---------------------------------------------------------------------------

def forward(p, rows, feat, emulate=True):
    r = bf16 if emulate else (lambda a: np.asarray(a, np.float64))
    E, W1, W2, W3 = r(p["E"]), r(p["W1"]), r(p["W2"]), r(p["W3"])
    X = np.concatenate([E[np.asarray(rows)], r(feat)], axis=1)
    z1 = X @ W1.T + p["b1"]
    h1 = r(gelu(z1))
    z2 = h1 @ W2.T + p["b2"]
    h2 = r(gelu(z2))
    out = h2 @ W3.T + p["b3"]
    return {"X": X, "z1": z1, "h1": h1, "z2": z2, "h2": h2, "out": out,
            "W1": W1, "W2": W2, "W3": W3}


def loss_terms(out, y, tau=TAU):
    mu, q = out[:, 0], out[:, 1]
    u = y - q
    return (mu - y) ** 2 + u * (tau - (u < 0))


def loss_and_grads(p, rows, feat, y, emulate=True, tau=TAU):
    """Mean loss over the batch and the gradient of every parameter (the
    straight-through gradient of the BF16 rounding points)."""
    r = bf16 if emulate else (lambda a: np.asarray(a, np.float64))
    c = forward(p, rows, feat, emulate)
    y = np.asarray(y, np.float64)
    B = len(y)
    out = c["out"]
    loss = float(np.mean(loss_terms(out, y, tau)))
    dmu = 2.0 * (out[:, 0] - y) / B
    dq = (((y - out[:, 1]) < 0).astype(np.float64) - tau) / B
    dout = r(np.stack([dmu, dq], axis=1))
    g = {}
    g["W3"] = dout.T @ c["h2"]
    g["b3"] = dout.sum(0)
    dh2 = dout @ c["W3"]
    dz2 = r(dh2 * gelu_grad(c["z2"]))
    g["W2"] = dz2.T @ c["h1"]
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ c["W2"]
    dz1 = r(dh1 * gelu_grad(c["z1"]))
    g["W1"] = dz1.T @ c["X"]
    g["b1"] = dz1.sum(0)
    dX = dz1 @ c["W1"]
    g["E"] = np.zeros_like(p["E"])
    np.add.at(g["E"], np.asarray(rows), dX[:, :EMB])
    return loss, g


def grad_magnitudes(p, rows, feat, y, emulate=True, tau=TAU):
    """Per gradient element, the sum of the absolute values of the terms the
    backward adds up for it: the same chain as loss_and_grads with every
    factor replaced by its absolute value.  Any rounding of the terms (FP32
    accumulation, one-ulp BF16 flips of an operand) changes a gradient element
    by a fraction of this sum, so it scales element-wise tolerances; it is at
    least |g| everywhere (triangle inequality)."""
    r = bf16 if emulate else (lambda a: np.asarray(a, np.float64))
    c = forward(p, rows, feat, emulate)
    y = np.asarray(y, np.float64)
    B = len(y)
    out = c["out"]
    dmu = 2.0 * (out[:, 0] - y) / B
    dq = (((y - out[:, 1]) < 0).astype(np.float64) - tau) / B
    a_out = np.abs(r(np.stack([dmu, dq], axis=1)))
    m = {}
    m["W3"] = a_out.T @ np.abs(c["h2"])
    m["b3"] = a_out.sum(0)
    a_z2 = (a_out @ np.abs(c["W3"])) * np.abs(gelu_grad(c["z2"]))
    m["W2"] = a_z2.T @ np.abs(c["h1"])
    m["b2"] = a_z2.sum(0)
    a_z1 = (a_z2 @ np.abs(c["W2"])) * np.abs(gelu_grad(c["z1"]))
    m["W1"] = a_z1.T @ np.abs(c["X"])
    m["b1"] = a_z1.sum(0)
    a_X = a_z1 @ np.abs(c["W1"])
    m["E"] = np.zeros_like(p["E"])
    np.add.at(m["E"], np.asarray(rows), a_X[:, :EMB])
    return m


# ---------------------------------------------------------------------------
# AdamW (decoupled weight decay; decay on E, W1, W2, W3, not on biases)
# ---------------------------------------------------------------------------

DECAYED = ("E", "W1", "W2", "W3")


def adamw_step(p, g, m, v, step, lr, wd, beta1=0.9, beta2=0.999, eps=1e-8):
    """One AdamW update in place; `step` is the 1-based step number."""
    for k in NAMES:
        if k in DECAYED:
            p[k] = p[k] * (1.0 - lr * wd)
        m[k] = beta1 * m[k] + (1.0 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k]
        mh = m[k] / (1.0 - beta1 ** step)
        vh = v[k] / (1.0 - beta2 ** step)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


# ---------------------------------------------------------------------------
# latency prediction and decisions
# ---------------------------------------------------------------------------

def predicted_latency(out, lat_profile, spread_max):
    """Per row: ceil(exp(q)) (capped at 2^31-1) when the predicted spread
    q - mu is finite and in [0, spread_max], else the profiled latency."""
    mu, q = out[:, 0], out[:, 1]
    s = q - mu
    ok = np.isfinite(mu) & np.isfinite(q) & (s >= 0) & (s <= spread_max)
    with np.errstate(over="ignore"):
        L = np.minimum(np.ceil(np.exp(np.where(ok, q, 0.0))), 2.0 ** 31 - 1)
    return np.where(ok, L, lat_profile).astype(np.int64), ok


def truth_mean_log_latency(lat, a_hw, b_op, n_obj, px, px_ref=1280 * 720):
    """The simulator's truth model of mean ln latency (used for training
    data and to judge decisions): ln L_profile + a * ln(1 + n_obj) + b * ln(px / px_720p)."""
    return (np.log(np.asarray(lat, np.float64)) + a_hw * np.log1p(n_obj)
            + b_op * np.log(np.asarray(px, np.float64) / px_ref))


def truth_p95_latency(mu_star, sigma):
    return np.minimum(np.ceil(np.exp(mu_star + Z95 * sigma)), 2.0 ** 31 - 1).astype(np.int64)


def regret(choice, truth_choice, truth_flag, truth_lat, target, hw, cost, batch, cfg_base):
    """Mean cost regret of `choice` against the truth decision, over
    invocations whose truth decision is feasible and whose chosen
    configuration is truly feasible; plus the miss rate (chosen configuration
    truly infeasible while a feasible one existed).  truth_lat is
    [n_inv, n_cfg_op]; hw/cost/batch are the profile arrays; cfg_base[i] is
    the first row of invocation i's op."""
    n = len(choice)
    idx = np.arange(n)
    x_c = cfg_base + choice
    x_t = cfg_base + truth_choice
    feas_c = truth_lat[idx, choice] < target[idx, hw[x_c]]
    has = truth_flag == 1
    ok = has & feas_c
    per_item = cost.astype(np.float64) / batch.astype(np.float64)
    reg = per_item[x_c[ok]] / np.maximum(per_item[x_t[ok]], 1e-300) - 1.0
    return {"mean_regret": float(reg.mean()) if reg.size else 0.0,
            "miss_rate": float(np.mean(has & ~feas_c)) if n else 0.0,
            "n_scored": int(ok.sum()), "n_feasible": int(has.sum())}
