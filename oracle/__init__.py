"""CPU oracle for the Llama decision path (arXiv 2102.01887, Alg. 1 and Eq. 1).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use this package.  The product (``paper_2102_01887_amd``)
never imports it, and it imports nothing from the product.

``liboracle.so`` is built from ``oracle.c`` by ``build()`` (plain gcc).  The
wrappers below only marshal numpy arrays; all arithmetic is in the C file.
The learned-surrogate oracle (FP64 MLP with BF16 rounding emulation) is in
``oracle/mlp.py``.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "oracle.c")

PAPER = 0
PROB = 1

OK, E_ARG, E_RANGE, E_CYCLE, E_STATE = 0, -1, -2, -3, -4


def build(verbose=False):
    """Compile oracle.c into liboracle.so with gcc (no GPU code)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
           SRC_PATH, "-o", LIB_PATH + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def load(path):
    """Load an oracle library from ``path`` and declare its signatures."""
    L = ctypes.CDLL(path)
    p = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    L.oracle_reference_cfg.argtypes = [i32, p, p, p, p, p]
    L.oracle_worst_path.argtypes = [i32, p, p, p, p, i32, p]
    L.oracle_targets.argtypes = [i64, p, p, p, i32, p, i32, p, p, p]
    L.oracle_select.argtypes = [i64, p, p, i32, i32, p, p, p, p, p, p, p]
    L.oracle_decide.argtypes = [i64, p, p, p, i32, p, i32, p, p, p, p, p,
                                p, p, p, p, p]
    L.oracle_select_lat.argtypes = [i64, p, p, i32, i32, p, p, p, p, i64, p, p, p]
    L.oracle_queue_time.argtypes = [i64, p, p, i32, i32, p, p, p, p, p, p, p]
    u32 = ctypes.c_uint32
    L.oracle_select_alpha.argtypes = [i64, p, p, i32, i32, p, p, p, p, p, p, p, u32, u32, p, p]
    L.oracle_decide_alpha.argtypes = [i64, p, p, p, i32, p, i32, p, p, p, p, p, p, p, p, p,
                                      u32, u32, p, p, p]
    L.oracle_fraction_below.argtypes = [p, p, p, p]
    L.oracle_feedback.argtypes = [i64, p, p, p, i32, p, p, ctypes.c_uint32, p]
    L.oracle_decide_batching.argtypes = [i64, p, p, p, i32, p, i32, p, p, p, p, p, p, p, p, p, p,
                                         p, p, p]
    L.oracle_affinity_terms.argtypes = [i64, p, p, p, i32, p, i32, p, p, p, p, p, p, p, p, p,
                                        ctypes.c_uint32, ctypes.c_uint32, p, p, p, p, p]
    for f in (L.oracle_reference_cfg, L.oracle_worst_path, L.oracle_targets,
              L.oracle_select, L.oracle_decide, L.oracle_select_lat, L.oracle_queue_time,
              L.oracle_select_alpha, L.oracle_decide_alpha, L.oracle_fraction_below,
              L.oracle_feedback, L.oracle_affinity_terms, L.oracle_decide_batching):
        f.restype = ctypes.c_int
    return L


class use:
    """Context manager: route the wrappers below through another build of the
    oracle (the test suite uses it to check that planted mistakes are caught)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.prev = _lib
        _lib = load(self.path)
        return _lib

    def __exit__(self, *exc):
        global _lib
        _lib = self.prev
        return False


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = load(LIB_PATH)
    return _lib


class OracleError(RuntimeError):
    def __init__(self, fn, rc):
        super().__init__(f"{fn} returned {rc}")
        self.rc = rc


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _arr(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def _check(fn, rc):
    if rc != OK:
        raise OracleError(fn, rc)


def reference_cfg(cfg_off, hw, batch, res):
    cfg_off = _arr(cfg_off, np.int32)
    n_ops = len(cfg_off) - 1
    out = np.empty(n_ops, np.int32)
    a = [_arr(x, np.int32) for x in (hw, batch, res)]
    _check("oracle_reference_cfg",
           lib().oracle_reference_cfg(n_ops, _ptr(cfg_off), *map(_ptr, a), _ptr(out)))
    return out


def reference_latency(cfg_off, lat, ref_k):
    """ref[v] = lat of the op's reference configuration (int64)."""
    cfg_off = np.asarray(cfg_off, np.int64)
    return np.asarray(lat, np.int64)[cfg_off[:-1] + np.asarray(ref_k, np.int64)]


def worst_path(succ_off, succ_ids, succ_q16, ref_lat, mode):
    succ_off = _arr(succ_off, np.int32)
    n_ops = len(succ_off) - 1
    ids = _arr(succ_ids, np.int32)
    q = _arr(succ_q16, np.uint32)
    ref = _arr(ref_lat, np.int64)
    W = np.empty(n_ops, np.int64)
    _check("oracle_worst_path",
           lib().oracle_worst_path(n_ops, _ptr(succ_off), _ptr(ids), _ptr(q),
                                   _ptr(ref), mode, _ptr(W)))
    return W


def targets(inv_op, elapsed, slo, n_hw, Q, ref_lat, W):
    inv_op, elapsed, slo = (_arr(x, np.int32) for x in (inv_op, elapsed, slo))
    n = len(inv_op)
    Q = _arr(Q, np.int64)
    ref = _arr(ref_lat, np.int64)
    Wa = _arr(W, np.int64)
    out = np.empty((n, n_hw), np.int32)
    _check("oracle_targets",
           lib().oracle_targets(n, _ptr(inv_op), _ptr(elapsed), _ptr(slo), n_hw,
                                _ptr(Q), len(ref), _ptr(ref), _ptr(Wa), _ptr(out)))
    return out


def select(inv_op, target, n_hw, cfg_off, hw, batch, lat, cost):
    inv_op = _arr(inv_op, np.int32)
    n = len(inv_op)
    target = _arr(target, np.int32).reshape(n, n_hw)
    cfg_off = _arr(cfg_off, np.int32)
    hw, batch, lat = (_arr(x, np.int32) for x in (hw, batch, lat))
    cost = _arr(cost, np.int64)
    cfg = np.empty(n, np.int32)
    flag = np.empty(n, np.uint8)
    _check("oracle_select",
           lib().oracle_select(n, _ptr(inv_op), _ptr(target), n_hw, len(cfg_off) - 1,
                               _ptr(cfg_off), _ptr(hw), _ptr(batch), _ptr(lat),
                               _ptr(cost), _ptr(cfg), _ptr(flag)))
    return cfg, flag


def select_lat(inv_op, target, n_hw, cfg_off, hw, batch, lat_inv, cost):
    """Eq. 1 with a latency per (invocation, configuration): lat_inv is
    [n_inv, stride] holding the op's configurations in caller order."""
    inv_op = _arr(inv_op, np.int32)
    n = len(inv_op)
    target = _arr(target, np.int32).reshape(n, n_hw)
    cfg_off = _arr(cfg_off, np.int32)
    hw, batch = (_arr(x, np.int32) for x in (hw, batch))
    lat_inv = _arr(lat_inv, np.int32).reshape(n, -1)
    cost = _arr(cost, np.int64)
    cfg = np.empty(n, np.int32)
    flag = np.empty(n, np.uint8)
    _check("oracle_select_lat",
           lib().oracle_select_lat(n, _ptr(inv_op), _ptr(target), n_hw, len(cfg_off) - 1,
                                   _ptr(cfg_off), _ptr(hw), _ptr(batch), _ptr(lat_inv),
                                   lat_inv.shape[1], _ptr(cost), _ptr(cfg), _ptr(flag)))
    return cfg, flag


def decide(inv_op, elapsed, slo, n_hw, Q, ref_lat, W, cfg_off, hw, batch, lat, cost):
    inv_op, elapsed, slo = (_arr(x, np.int32) for x in (inv_op, elapsed, slo))
    n = len(inv_op)
    Q = _arr(Q, np.int64)
    ref = _arr(ref_lat, np.int64)
    Wa = _arr(W, np.int64)
    cfg_off = _arr(cfg_off, np.int32)
    hw, batch, lat = (_arr(x, np.int32) for x in (hw, batch, lat))
    cost = _arr(cost, np.int64)
    cfg = np.empty(n, np.int32)
    flag = np.empty(n, np.uint8)
    scratch = np.empty(n_hw, np.int32)
    _check("oracle_decide",
           lib().oracle_decide(n, _ptr(inv_op), _ptr(elapsed), _ptr(slo), n_hw,
                               _ptr(Q), len(ref), _ptr(ref), _ptr(Wa), _ptr(cfg_off),
                               _ptr(hw), _ptr(batch), _ptr(lat), _ptr(cost),
                               _ptr(cfg), _ptr(flag), _ptr(scratch)))
    return cfg, flag


def queue_time(q_op, q_cfg, n_hw, cfg_off, hw, res, lat, r_total):
    """Eq. 2 per backend from the queued invocations' (op, configuration);
    returns (Q int64 [n_hw], number of skipped out-of-range entries)."""
    q_op, q_cfg = _arr(q_op, np.int32), _arr(q_cfg, np.int32)
    cfg_off = _arr(cfg_off, np.int32)
    hw, res, lat = (_arr(x, np.int32) for x in (hw, res, lat))
    r_total = _arr(r_total, np.int64)
    Q = np.empty(n_hw, np.int64)
    skipped = ctypes.c_int64()
    _check("oracle_queue_time",
           lib().oracle_queue_time(len(q_op), _ptr(q_op), _ptr(q_cfg), n_hw, len(cfg_off) - 1,
                                   _ptr(cfg_off), _ptr(hw), _ptr(res), _ptr(lat), _ptr(r_total),
                                   _ptr(Q), ctypes.byref(skipped)))
    return Q, skipped.value


def feedback(obs_op, obs_cfg, obs_lat, cfg_off, lat, beta_q16):
    """Exponential smoothing of the profile latencies from observations;
    returns (new latencies, number of skipped observations)."""
    obs_op, obs_cfg, obs_lat = (_arr(x, np.int32) for x in (obs_op, obs_cfg, obs_lat))
    cfg_off = _arr(cfg_off, np.int32)
    out = np.array(lat, dtype=np.int32, copy=True)
    skipped = ctypes.c_int64()
    _check("oracle_feedback",
           lib().oracle_feedback(len(obs_op), _ptr(obs_op), _ptr(obs_cfg), _ptr(obs_lat),
                                 len(cfg_off) - 1, _ptr(cfg_off), _ptr(out), beta_q16,
                                 ctypes.byref(skipped)))
    return out, skipped.value


CFG_WAIT = -2


def decide_batching(inv_op, elapsed, slo, n_hw, Q, ref_lat, W, cfg_off, hw, batch, lat, cost,
                    available, upstream, wait_us):
    """Safe delayed batching: (cfg, flag), cfg = CFG_WAIT for a wait."""
    inv_op, elapsed, slo = (_arr(x, np.int32) for x in (inv_op, elapsed, slo))
    n = len(inv_op)
    Q = _arr(Q, np.int64)
    ref = _arr(ref_lat, np.int64)
    Wa = _arr(W, np.int64)
    cfg_off = _arr(cfg_off, np.int32)
    hw, batch, lat = (_arr(x, np.int32) for x in (hw, batch, lat))
    cost = _arr(cost, np.int64)
    available, upstream, wait_us = (_arr(x, np.int32) for x in (available, upstream, wait_us))
    cfg = np.empty(n, np.int32)
    flag = np.empty(n, np.uint8)
    scratch = np.empty(n_hw, np.int32)
    _check("oracle_decide_batching",
           lib().oracle_decide_batching(n, _ptr(inv_op), _ptr(elapsed), _ptr(slo), n_hw, _ptr(Q),
                                        len(ref), _ptr(ref), _ptr(Wa), _ptr(cfg_off), _ptr(hw),
                                        _ptr(batch), _ptr(lat), _ptr(cost), _ptr(available),
                                        _ptr(upstream), _ptr(wait_us), _ptr(cfg), _ptr(flag),
                                        _ptr(scratch)))
    return cfg, flag


def affinity_terms(inv_op, elapsed, slo, n_hw, Q, ref_lat, W, cfg_off, hw, batch, res, lat, cost,
                   r_total, alpha_num, alpha_den):
    """Eq. 3's two minima per (invocation, backend) as exact Python Fractions
    (None for a side without configurations): (own [n][n_hw], other [n][n_hw])."""
    from fractions import Fraction
    inv_op, elapsed, slo = (_arr(x, np.int32) for x in (inv_op, elapsed, slo))
    n = len(inv_op)
    Q = _arr(Q, np.int64)
    ref = _arr(ref_lat, np.int64)
    Wa = _arr(W, np.int64)
    cfg_off = _arr(cfg_off, np.int32)
    hw, batch, res, lat = (_arr(x, np.int32) for x in (hw, batch, res, lat))
    cost, r_total = _arr(cost, np.int64), _arr(r_total, np.int64)
    bufs = [np.zeros(n * n_hw * 2, np.uint64) for _ in range(4)]
    scratch = np.empty(n_hw, np.int32)
    _check("oracle_affinity_terms",
           lib().oracle_affinity_terms(n, _ptr(inv_op), _ptr(elapsed), _ptr(slo), n_hw, _ptr(Q),
                                       len(ref), _ptr(ref), _ptr(Wa), _ptr(cfg_off), _ptr(hw),
                                       _ptr(batch), _ptr(res), _ptr(lat), _ptr(cost), _ptr(r_total),
                                       alpha_num, alpha_den, *(_ptr(b) for b in bufs), _ptr(scratch)))
    big = [b.reshape(n, n_hw, 2) for b in bufs]

    def frac(num, den, i, h):
        d = int(den[i, h, 0]) | (int(den[i, h, 1]) << 64)
        if d == 0:
            return None
        return Fraction(int(num[i, h, 0]) | (int(num[i, h, 1]) << 64), d)

    own = [[frac(big[0], big[1], i, h) for h in range(n_hw)] for i in range(n)]
    oth = [[frac(big[2], big[3], i, h) for h in range(n_hw)] for i in range(n)]
    return own, oth


def affinity_value(own, oth):
    """Eq. 3 from its two minima, with the readings for empty sides and zero
    objectives: no configuration on the backend -> 0; none elsewhere -> inf;
    zero own minimum -> inf (1 when the other minimum is zero as well)."""
    if own is None:
        return 0.0
    if oth is None:
        return float("inf")
    if own == 0:
        return 1.0 if oth == 0 else float("inf")
    return float(oth / own)


def fraction_below(n1, d1, n2, d2):
    """n1/d1 < n2/d2 as the oracle decides it (operands below 2^128)."""
    limbs = [np.array([x & (2**64 - 1), x >> 64], np.uint64) for x in (n1, d1, n2, d2)]
    return bool(lib().oracle_fraction_below(*(_ptr(a) for a in limbs)))


def select_alpha(inv_op, target, n_hw, cfg_off, hw, batch, res, lat, cost, r_total,
                 alpha_num, alpha_den):
    """Eq. 1 with the finite weight alpha = alpha_num / alpha_den."""
    inv_op = _arr(inv_op, np.int32)
    n = len(inv_op)
    target = _arr(target, np.int32).reshape(n, n_hw)
    cfg_off = _arr(cfg_off, np.int32)
    hw, batch, res, lat = (_arr(x, np.int32) for x in (hw, batch, res, lat))
    cost, r_total = _arr(cost, np.int64), _arr(r_total, np.int64)
    cfg = np.empty(n, np.int32)
    flag = np.empty(n, np.uint8)
    _check("oracle_select_alpha",
           lib().oracle_select_alpha(n, _ptr(inv_op), _ptr(target), n_hw, len(cfg_off) - 1,
                                     _ptr(cfg_off), _ptr(hw), _ptr(batch), _ptr(res), _ptr(lat),
                                     _ptr(cost), _ptr(r_total), alpha_num, alpha_den,
                                     _ptr(cfg), _ptr(flag)))
    return cfg, flag


def decide_alpha(inv_op, elapsed, slo, n_hw, Q, ref_lat, W, cfg_off, hw, batch, res, lat, cost,
                 r_total, alpha_num, alpha_den):
    inv_op, elapsed, slo = (_arr(x, np.int32) for x in (inv_op, elapsed, slo))
    n = len(inv_op)
    Q = _arr(Q, np.int64)
    ref = _arr(ref_lat, np.int64)
    Wa = _arr(W, np.int64)
    cfg_off = _arr(cfg_off, np.int32)
    hw, batch, res, lat = (_arr(x, np.int32) for x in (hw, batch, res, lat))
    cost, r_total = _arr(cost, np.int64), _arr(r_total, np.int64)
    cfg = np.empty(n, np.int32)
    flag = np.empty(n, np.uint8)
    scratch = np.empty(n_hw, np.int32)
    _check("oracle_decide_alpha",
           lib().oracle_decide_alpha(n, _ptr(inv_op), _ptr(elapsed), _ptr(slo), n_hw, _ptr(Q),
                                     len(ref), _ptr(ref), _ptr(Wa), _ptr(cfg_off), _ptr(hw),
                                     _ptr(batch), _ptr(res), _ptr(lat), _ptr(cost), _ptr(r_total),
                                     alpha_num, alpha_den, _ptr(cfg), _ptr(flag), _ptr(scratch)))
    return cfg, flag


class Problem:
    """Bundle of one workload's arrays with the oracle's derived quantities.

    Holds exactly the caller's inputs (DAG CSR, profile table, invocations);
    ``ref``/``W``/``targets``/``decide`` are computed by the oracle above.
    """

    def __init__(self, w):
        self.w = w
        self.ref_k = (reference_cfg(w.cfg_off, w.hw, w.batch, w.res)
                      if w.ref_cfg is None else np.asarray(w.ref_cfg, np.int32))
        self.ref = reference_latency(w.cfg_off, w.lat, self.ref_k)
        self._W = {}

    def W(self, mode):
        if mode not in self._W:
            w = self.w
            self._W[mode] = worst_path(w.succ_off, w.succ_ids, w.succ_q16, self.ref, mode)
        return self._W[mode]

    def targets(self, mode, Q=None, sl=slice(None)):
        w = self.w
        return targets(w.inv_op[sl], w.elapsed[sl], w.slo[sl], w.n_hw, Q,
                       self.ref, self.W(mode))

    def decide(self, mode, Q=None, sl=slice(None)):
        w = self.w
        return decide(w.inv_op[sl], w.elapsed[sl], w.slo[sl], w.n_hw, Q, self.ref,
                      self.W(mode), w.cfg_off, w.hw, w.batch, w.lat, w.cost)

    def decide_parallel(self, mode, threads, Q=None):
        """decide() over every invocation on `threads` host threads: the
        invocations are cut into that many contiguous parts and each part is
        one single-threaded oracle call (ctypes releases the GIL), so the
        result is the same as decide()'s."""
        from concurrent.futures import ThreadPoolExecutor
        n = self.w.n_inv
        self.W(mode)
        cuts = [n * k // threads for k in range(threads + 1)]
        parts = [slice(cuts[k], cuts[k + 1]) for k in range(threads)]
        with ThreadPoolExecutor(threads) as ex:
            res = list(ex.map(lambda sl: self.decide(mode, Q, sl), parts))
        return np.concatenate([r[0] for r in res]), np.concatenate([r[1] for r in res])

    def select(self, target, sl=slice(None)):
        w = self.w
        return select(w.inv_op[sl], target, w.n_hw, w.cfg_off, w.hw, w.batch,
                      w.lat, w.cost)

    def queue_time(self, q_op, q_cfg):
        w = self.w
        return queue_time(q_op, q_cfg, w.n_hw, w.cfg_off, w.hw, w.res, w.lat, w.hw_res_total)

    def decide_batching(self, mode, available, upstream, wait_us, Q=None, sl=slice(None)):
        w = self.w
        return decide_batching(w.inv_op[sl], w.elapsed[sl], w.slo[sl], w.n_hw, Q, self.ref,
                               self.W(mode), w.cfg_off, w.hw, w.batch, w.lat, w.cost, available,
                               upstream, wait_us)

    def affinity(self, mode, alpha_num, alpha_den, Q=None, sl=slice(None)):
        """Eq. 3 per (invocation, backend) as floats (correctly rounded from
        the exact ratio), with the readings of affinity_value."""
        w = self.w
        own, oth = affinity_terms(w.inv_op[sl], w.elapsed[sl], w.slo[sl], w.n_hw, Q, self.ref,
                                  self.W(mode), w.cfg_off, w.hw, w.batch, w.res, w.lat, w.cost,
                                  w.hw_res_total, alpha_num, alpha_den)
        return np.array([[affinity_value(o, t) for o, t in zip(ro, rt)] for ro, rt in zip(own, oth)])

    def decide_alpha(self, mode, alpha_num, alpha_den, Q=None, sl=slice(None)):
        w = self.w
        return decide_alpha(w.inv_op[sl], w.elapsed[sl], w.slo[sl], w.n_hw, Q, self.ref,
                            self.W(mode), w.cfg_off, w.hw, w.batch, w.res, w.lat, w.cost,
                            w.hw_res_total, alpha_num, alpha_den)
