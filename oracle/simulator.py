"""Test infrastructure: CPU reference of the GPU pipeline simulator.

Not part of the product path: only tests and bench.py's cpu_baseline may use
it.  The GPU simulator (llama_simulate) draws the training executions of the
learned latency surrogate on the device; this module computes the same
draws on the CPU from the same counter-based random numbers, in FP64, so that
the GPU's samples can be checked one by one.

Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC 2011): a 128-bit counter and a 64-bit key
give four 32-bit words after ten rounds of two 32x32->64-bit multiplications
with the key bumped by the Weyl constants between rounds.  Sample i uses the
counters (i, k, 0, 0), k = 0..5, under key (seed low word, seed high word):
24 words, used in this order:
  w0           configuration row: floor(w0 * n_rows / 2^32)
  w1..w4       two Box-Muller pairs: N_people, N_cars (rates), N_noise, unused
  w5, w6       people, cars: inversion of Poisson(rate), rate =
               exp(ln 2 + N), capped (people at 60, cars at 60 - people)
  w7           faces: inversion of Binomial(people, 0.6)
  w8           resolution: floor(w8 * 3 / 2^32) -> 480p, 720p, 1080p
  w9..w11      motion, blur, brightness U(0, 1)
  w12..w21     Beta(3, 7) = G3 / (G3 + G7), G3 = -ln(u12 u13 u14),
               G7 = -ln(u15 ... u21) (sums of unit exponentials)
  w22          frame phase 2 pi u
with u = (w + 0.5) / 2^32.  The observed ln latency of row x is the truth mean
ln L[x] + a[op, hw(x)] ln(1 + n_obj) + b[op] ln(px / px_720p) plus sigma N_noise.
"""
import numpy as np

PHILOX_M0, PHILOX_M1 = 0xD2511F53, 0xCD9E8D57
PHILOX_W0, PHILOX_W1 = 0x9E3779B9, 0xBB67AE85
M32 = 0xFFFFFFFF
RESOLUTIONS = ((854, 480), (1280, 720), (1920, 1080))
PX_720P = 1280 * 720
N_FEAT = 16


def philox4x32_10(ctr, key):
    """Philox4x32-10 of counters ctr [n, 4] (uint32) under key (2 uint32):
    [n, 4] uint32.  One round: the products of words 0 and 2 with the two
    multipliers give the new words (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)."""
    c = np.asarray(ctr, np.uint64) & M32
    c0, c1, c2, c3 = (c[:, j].copy() for j in range(4))
    k0, k1 = np.uint64(key[0] & M32), np.uint64(key[1] & M32)
    for r in range(10):
        p0 = np.uint64(PHILOX_M0) * c0
        p1 = np.uint64(PHILOX_M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(M32)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(M32)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        if r < 9:
            k0 = (k0 + np.uint64(PHILOX_W0)) & np.uint64(M32)
            k1 = (k1 + np.uint64(PHILOX_W1)) & np.uint64(M32)
    return np.stack([c0, c1, c2, c3], axis=1).astype(np.uint32)


def words(n, seed, first=0):
    """The 24 words of samples first .. first + n - 1: [n, 24] uint32."""
    i = np.arange(first, first + n, dtype=np.uint64)
    key = (int(seed) & M32, (int(seed) >> 32) & M32)
    out = np.empty((n, 24), np.uint32)
    for k in range(6):
        ctr = np.zeros((n, 4), np.uint64)
        ctr[:, 0] = i & np.uint64(M32)
        ctr[:, 1] = np.uint64(k)
        out[:, 4 * k:4 * k + 4] = philox4x32_10(ctr, key)
    return out


def uniform(w):
    """(w + 1/2) / 2^32 in (0, 1), exact in FP64."""
    return (w.astype(np.float64) + 0.5) * (1.0 / 4294967296.0)


def poisson_inv(u, rate, cap):
    """Smallest k with u < P(X <= k) for X ~ Poisson(rate), at most cap
    (the pmf by its recurrence p_k = p_{k-1} rate / k); also the distance of u
    from the nearest cdf value the search compared it with."""
    n = len(u)
    k = np.zeros(n, np.int64)
    p = np.exp(-rate)
    cdf = p.copy()
    margin = np.abs(u - cdf)
    done = (u < cdf) | (k >= cap)
    for j in range(1, int(np.max(cap)) + 1 if n else 1):
        act = ~done
        if not act.any():
            break
        p = np.where(act, p * rate / j, p)
        cdf = np.where(act, cdf + p, cdf)
        k = np.where(act, j, k)
        margin = np.where(act, np.minimum(margin, np.abs(u - cdf)), margin)
        done = done | (u < cdf) | (k >= cap)
    return k, margin


def binomial_inv(u, m, p):
    """Smallest k with u < P(X <= k) for X ~ Binomial(m, p) (at most m),
    from the pmf recurrence; and the margin as in poisson_inv."""
    n = len(u)
    q = 1.0 - p
    pk = q ** m.astype(np.float64)
    cdf = pk.copy()
    k = np.zeros(n, np.int64)
    margin = np.abs(u - cdf)
    done = (u < cdf) | (k >= m)
    for j in range(1, int(np.max(m)) + 1 if n else 1):
        act = ~done
        if not act.any():
            break
        pk = np.where(act, pk * (m - j + 1) / j * (p / q), pk)
        cdf = np.where(act, cdf + pk, cdf)
        k = np.where(act, j, k)
        margin = np.where(act, np.minimum(margin, np.abs(u - cdf)), margin)
        done = done | (u < cdf) | (k >= m)
    return k, margin


def to_bf16(x):
    """Round to nearest even BF16, returned as float32 values."""
    b = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + np.uint64(0x7FFF) + ((b >> np.uint64(16)) & np.uint64(1))) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32)


def simulate(n, seed, n_rows, lat, hw, a, b, sigma, cfg_per_op=64, first=0):
    """n executions (samples first ..): rows, features (BF16 values as float32
    [n, 16]), y (float32), and the integer draws with their decision margins
    (for the comparison with the GPU)."""
    w = words(n, seed, first)
    rows = ((w[:, 0].astype(np.uint64) * np.uint64(n_rows)) >> np.uint64(32)).astype(np.int64)
    u = uniform(w)
    r1 = np.sqrt(-2.0 * np.log(u[:, 1]))
    z_people = r1 * np.cos(2.0 * np.pi * u[:, 2])
    z_cars = r1 * np.sin(2.0 * np.pi * u[:, 2])
    r2 = np.sqrt(-2.0 * np.log(u[:, 3]))
    z_noise = r2 * np.cos(2.0 * np.pi * u[:, 4])
    people, m_p = poisson_inv(u[:, 5], np.exp(np.log(2.0) + z_people), np.full(n, 60))
    cars, m_c = poisson_inv(u[:, 6], np.exp(np.log(2.0) + z_cars), 60 - people)
    faces, m_f = binomial_inv(u[:, 7], people, 0.6)
    res = ((w[:, 8].astype(np.uint64) * np.uint64(3)) >> np.uint64(32)).astype(np.int64)
    wh = np.asarray(RESOLUTIONS, np.int64)[res]
    px = wh[:, 0] * wh[:, 1]
    g3 = -np.log(u[:, 12] * u[:, 13] * u[:, 14])
    g7 = -np.log(u[:, 15] * u[:, 16] * u[:, 17] * u[:, 18] * u[:, 19] * u[:, 20] * u[:, 21])
    phase = 2.0 * np.pi * u[:, 22]
    n_obj = people + cars
    f = np.zeros((n, N_FEAT), np.float64)
    f[:, 0] = people / 60.0
    f[:, 1] = cars / 60.0
    f[:, 2] = faces / 60.0
    f[:, 3] = np.log1p(n_obj) / np.log(61.0)
    f[:, 4] = wh[:, 0] / 1920.0
    f[:, 5] = wh[:, 1] / 1080.0
    f[:, 6] = px / (1920.0 * 1080.0)
    f[:, 7] = u[:, 9]
    f[:, 8] = u[:, 10]
    f[:, 9] = u[:, 11]
    f[:, 10] = g3 / (g3 + g7)
    f[:, 11] = np.sin(phase)
    f[:, 12] = np.cos(phase)
    op = rows // cfg_per_op
    h = np.asarray(hw)[rows]
    mu = (np.log(np.asarray(lat, np.float64)[rows]) + np.asarray(a)[op, h] * np.log1p(n_obj)
          + np.asarray(b)[op] * np.log(px / PX_720P))
    y = mu + sigma * z_noise
    return {"rows": rows.astype(np.int32), "feat": to_bf16(f.astype(np.float32)), "feat64": f,
            "y": y.astype(np.float32), "y64": y, "people": people, "cars": cars, "faces": faces,
            "res": res, "margin": np.minimum(np.minimum(m_p, m_c), m_f)}
