"""ctypes binding of libllama (include/llama.h).

Argument marshalling only: host tables are passed as numpy arrays, device
buffers as torch CUDA tensors (their data_ptr()), streams as torch streams
(their HIP handle).  Every step of the decision runs in the library's HIP
kernels; there is no Python or CPU fallback, and a missing library is an
ImportError.
"""
import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libllama.so")

OK, E_ARG, E_RANGE, E_CYCLE, E_STATE, E_DEVICE, E_NOMEM = 0, -1, -2, -3, -4, -5, -6
SLACK_PAPER, SLACK_PROB = 0, 1
SCAN_AUTO, SCAN_INDEXED, SCAN_FULL, SCAN_WAVE = 0, 1, 2, 3
SCANS = (SCAN_INDEXED, SCAN_FULL, SCAN_WAVE)
# decision schedules that llama_autotune chooses among (index = its *chosen)
SCHEDULE_NAMES = ("direct-1", "direct-2", "direct-4", "lds-persistent", "direct-1-nt", "direct-2-nt",
                  "direct-4-nt")
DEVERR_INVALID_INVOCATION = 1
DEVERR_INVALID_QUEUE_ENTRY = 2
DEVERR_INVALID_OBSERVATION = 4
CFG_WAIT = -2

EXPORTS = ["llama_create", "llama_destroy", "llama_last_error", "llama_set_dag",
           "llama_set_profiles", "llama_relax", "llama_update_latencies", "llama_targets",
           "llama_select", "llama_decide", "llama_reserve", "llama_get_stats",
           "llama_debug_export", "llama_surrogate_param_count", "llama_surrogate_init",
           "llama_surrogate_set", "llama_surrogate_get", "llama_surrogate_grads",
           "llama_surrogate_reserve", "llama_surrogate_forward", "llama_surrogate_train_step",
           "llama_surrogate_save", "llama_surrogate_load", "llama_decide_learned",
           "llama_surrogate_fit", "llama_select_rows", "llama_serve_bytes_per_request",
           "llama_serve_open", "llama_serve_submit", "llama_serve_poll", "llama_serve_stats_get",
           "llama_serve_close", "llama_autotune", "llama_set_schedule", "llama_queue_time", "llama_set_alpha",
           "llama_decide_alpha", "llama_feedback", "llama_affinity", "llama_decide_batching",
           "llama_decide_full_noalloc", "llama_decide_full_noalloc_words", "llama_relax_modes",
           "llama_autotune_full", "llama_set_full_schedule",
           "llama_set_simulator", "llama_simulate"]


class LlamaStats(ctypes.Structure):
    _fields_ = [("n_ops", ctypes.c_int32), ("n_hw", ctypes.c_int32),
                ("n_pipelines", ctypes.c_int32), ("max_depth", ctypes.c_int32),
                ("n_cfg", ctypes.c_int64), ("n_edges", ctypes.c_int64),
                ("frontier_entries", ctypes.c_int64), ("device_error", ctypes.c_uint32),
                ("device_bytes", ctypes.c_int64)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("n_slots", ctypes.c_int32), ("mem_budget_bytes", ctypes.c_int64),
                ("max_batch", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("learned", ctypes.c_int32), ("slack_mode", ctypes.c_int32),
                ("spread_max", ctypes.c_float)]


class ServeStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "submitted", "admitted", "rejected", "decided", "collected", "batches", "bytes_in_use",
        "peak_bytes_in_use", "max_batch_seen", "in_flight_batches", "capacity", "kernel_launches",
        "clock_rtt_ns", "clock_anchors", "clock_rate_ppb", "clock_probes", "clock_probe_timeouts",
        "clock_probe_rtt_min_ns", "clock_probe_rtt_last_ns")]


_lib = None


def load_library(path=LIB_PATH):
    """Load libllama.so and declare the C signatures."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2102_01887_amd.build`")
    L = ctypes.CDLL(path)
    p, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "llama_create": [ctypes.POINTER(p), i32],
        "llama_destroy": [p],
        "llama_last_error": [p],
        "llama_set_dag": [p, i32, p, p, p, p],
        "llama_set_profiles": [p, i32, i32, p, p, p, p, p, p, p, p],
        "llama_relax": [p, p],
        "llama_relax_modes": [p, i32, p],
        "llama_autotune_full": [p, i64, p, p, p, i32, p, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                ctypes.POINTER(ctypes.c_float), p],
        "llama_set_full_schedule": [p, i32, i32],
        "llama_set_simulator": [p, p, p, ctypes.c_double],
        "llama_simulate": [p, i64, ctypes.c_uint64, i64, p, p, p, p],
        "llama_update_latencies": [p, p],
        "llama_targets": [p, i64, p, p, p, p, i32, p, p],
        "llama_select": [p, i64, p, p, p, p, p],
        "llama_decide": [p, i64, p, p, p, p, i32, i32, p, p, p],
        "llama_reserve": [p, i64],
        "llama_decide_full_noalloc": [p, i64, p, p, p, p, i32, p, p, p],
        "llama_decide_full_noalloc_words": [i64, i32],
        "llama_select_rows": [p, i64, p, p, p, i64, p, p, p],
        "llama_serve_bytes_per_request": [i32],
        "llama_autotune": [p, i64, p, p, p, p, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float), p],
        "llama_queue_time": [p, i64, p, p, p, p],
        "llama_set_alpha": [p, ctypes.c_uint32, ctypes.c_uint32],
        "llama_decide_alpha": [p, i64, p, p, p, p, i32, p, p, p],
        "llama_feedback": [p, i64, p, p, p, ctypes.c_uint32, p],
        "llama_affinity": [p, i64, p, p, p, p, i32, p, p, p],
        "llama_decide_batching": [p, i64, p, p, p, p, i32, p, p, p, p, p, p],
        "llama_serve_open": [p, ctypes.POINTER(ServeConfig), ctypes.POINTER(p)],
        "llama_serve_submit": [p, i32, p, p, p, p, p, p, ctypes.POINTER(i32)],
        "llama_serve_poll": [p, i32, p, p, p, p, ctypes.POINTER(i32), i32],
        "llama_serve_stats_get": [p, ctypes.POINTER(ServeStats)],
        "llama_serve_close": [p],
        "llama_set_schedule": [p, i32],
        "llama_get_stats": [p, ctypes.POINTER(LlamaStats), i32],
        "llama_debug_export": [p, i32, p, i64],
        "llama_surrogate_param_count": [i64],
        "llama_surrogate_init": [p, ctypes.c_uint64, ctypes.c_float],
        "llama_surrogate_set": [p, p, i64],
        "llama_surrogate_get": [p, p, i64],
        "llama_surrogate_grads": [p, p, i64],
        "llama_surrogate_reserve": [p, i64],
        "llama_surrogate_forward": [p, i64, p, p, p, p],
        "llama_surrogate_train_step": [p, i64, p, p, p, ctypes.c_float, ctypes.c_float, i32, p, p],
        "llama_surrogate_fit": [p, i64, p, p, p, i32, i64, ctypes.c_float, ctypes.c_float, p, p],
        "llama_surrogate_save": [p, ctypes.c_char_p],
        "llama_surrogate_load": [p, ctypes.c_char_p],
        "llama_decide_learned": [p, i64, p, p, p, p, i32, p, ctypes.c_float, p, p, p, i64, p],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.llama_destroy.restype = None
    L.llama_surrogate_param_count.restype = ctypes.c_int64
    L.llama_serve_bytes_per_request.restype = ctypes.c_int64
    L.llama_decide_full_noalloc_words.restype = ctypes.c_int64
    L.llama_last_error.restype = ctypes.c_char_p
    if path == LIB_PATH:
        _lib = L
    return L


class LlamaError(RuntimeError):
    def __init__(self, fn, rc, msg):
        super().__init__(f"{fn} failed ({rc}): {msg}")
        self.rc = rc


def _np(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def _hp(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _dp(t, dtype_name, n=None):
    """Device pointer of a contiguous CUDA tensor of the given dtype."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if str(t.dtype) != "torch." + dtype_name:
        raise ValueError(f"expected torch.{dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if n is not None and t.numel() < n:
        raise ValueError(f"tensor has {t.numel()} elements, need {n}")
    return ctypes.c_void_p(t.data_ptr())


def _dp16(t, n=None):
    """Device pointer of a contiguous 2-byte tensor holding BF16 bit patterns."""
    if t is None:
        return None
    if not t.is_cuda or t.element_size() != 2 or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor of bfloat16 (or 16-bit) elements")
    if n is not None and t.numel() < n:
        raise ValueError(f"tensor has {t.numel()} elements, need {n}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Llama:
    """One library context on one device."""

    def __init__(self, device=0):
        self._L = load_library()
        self._ctx = ctypes.c_void_p()
        rc = self._L.llama_create(ctypes.byref(self._ctx), int(device))
        if rc != OK:
            raise LlamaError("llama_create", rc, "no usable HIP device")
        self.device = device
        self.n_ops = self.n_hw = None
        self._keep = None

    def close(self):
        if self._ctx:
            self._L.llama_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, fn, rc):
        if rc != OK:
            raise LlamaError(fn, rc, self._L.llama_last_error(self._ctx).decode())

    # -- ingest -------------------------------------------------------------
    def set_dag(self, pipe_off, succ_off, succ_ids, succ_q16=None):
        pipe_off, succ_off, succ_ids = (_np(x, np.int32) for x in (pipe_off, succ_off, succ_ids))
        q = _np(succ_q16, np.uint32)
        self._check("llama_set_dag", self._L.llama_set_dag(
            self._ctx, len(pipe_off) - 1, _hp(pipe_off), _hp(succ_off), _hp(succ_ids), _hp(q)))
        self.n_ops = int(pipe_off[-1])

    def set_profiles(self, n_hw, cfg_off, hw, batch, res, lat, cost, ref_cfg=None,
                     hw_res_total=None):
        cfg_off, hw, batch, res, lat = (_np(x, np.int32) for x in (cfg_off, hw, batch, res, lat))
        cost = _np(cost, np.int64)
        ref = _np(ref_cfg, np.int32)
        tot = _np(hw_res_total, np.int64)
        self._check("llama_set_profiles", self._L.llama_set_profiles(
            self._ctx, len(cfg_off) - 1, int(n_hw), _hp(cfg_off), _hp(hw), _hp(batch), _hp(res),
            _hp(lat), _hp(cost), _hp(ref), _hp(tot)))
        self.n_hw = int(n_hw)
        self.n_cfg = int(cfg_off[-1])

    def load(self, w):
        """set_dag + set_profiles from a workloads.Workload."""
        self.set_dag(w.pipe_off, w.succ_off, w.succ_ids, w.succ_q16)
        self.set_profiles(w.n_hw, w.cfg_off, w.hw, w.batch, w.res, w.lat, w.cost, w.ref_cfg,
                          w.hw_res_total)
        return self

    def update_latencies(self, lat):
        lat = _np(lat, np.int32)
        self._check("llama_update_latencies", self._L.llama_update_latencies(self._ctx, _hp(lat)))

    def autotune(self, op, elapsed, slo, stream=None):
        """Pick the fastest decision schedule on this batch; returns (schedule index, us)."""
        import torch
        n = op.numel()
        scratch = torch.empty(n, dtype=torch.int32, device=op.device)
        k, us = ctypes.c_int32(), ctypes.c_float()
        self._check("llama_autotune", self._L.llama_autotune(
            self._ctx, n, _dp(op, "int32"), _dp(elapsed, "int32", n), _dp(slo, "int32", n),
            _dp(scratch, "int32", n), ctypes.byref(k), ctypes.byref(us), _stream(stream)))
        return k.value, us.value

    def set_schedule(self, schedule):
        """Pin the indexed decision's schedule (0..6, as numbered by autotune)."""
        self._check("llama_set_schedule", self._L.llama_set_schedule(self._ctx, int(schedule)))

    def autotune_full(self, op, elapsed, slo, mode=SLACK_PAPER, stream=None):
        """Pick the full scan's schedule crossover on this batch; returns
        ((num, den), us per call)."""
        import torch
        n = op.numel()
        scratch = torch.empty(n, dtype=torch.int32, device=op.device)
        num, den, us = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_float()
        self._check("llama_autotune_full", self._L.llama_autotune_full(
            self._ctx, n, _dp(op, "int32"), _dp(elapsed, "int32", n), _dp(slo, "int32", n), int(mode),
            _dp(scratch, "int32", n), ctypes.byref(num), ctypes.byref(den), ctypes.byref(us),
            _stream(stream)))
        return (num.value, den.value), us.value

    def set_full_schedule(self, num, den):
        """Pin the full scan's schedule crossover (the table autotune_full returns)."""
        self._check("llama_set_full_schedule", self._L.llama_set_full_schedule(self._ctx, int(num), int(den)))

    def reserve(self, max_inv):
        self._check("llama_reserve", self._L.llama_reserve(self._ctx, int(max_inv)))

    def relax(self, stream=None, modes=3):
        """Relaxation; `modes` = bit mask of the slack modes whose records are
        rebuilt (3 = both, llama_relax)."""
        if modes == 3:
            self._check("llama_relax", self._L.llama_relax(self._ctx, _stream(stream)))
        else:
            self._check("llama_relax_modes", self._L.llama_relax_modes(self._ctx, int(modes), _stream(stream)))

    # -- decisions (device tensors) --------------------------------------------
    def targets(self, op, elapsed, slo, queue=None, mode=SLACK_PAPER, out=None, stream=None):
        import torch
        n = op.numel()
        if out is None:
            out = torch.empty((n, self.n_hw), dtype=torch.int32, device=op.device)
        self._check("llama_targets", self._L.llama_targets(
            self._ctx, n, _dp(op, "int32"), _dp(elapsed, "int32", n), _dp(slo, "int32", n),
            _dp(queue, "int64", self.n_hw), int(mode), _dp(out, "int32", n * self.n_hw),
            _stream(stream)))
        return out

    def select(self, op, target, cfg=None, flag=None, stream=None):
        import torch
        n = op.numel()
        if cfg is None:
            cfg = torch.empty(n, dtype=torch.int32, device=op.device)
        if flag is None:
            flag = torch.empty(n, dtype=torch.uint8, device=op.device)
        self._check("llama_select", self._L.llama_select(
            self._ctx, n, _dp(op, "int32"), _dp(target, "int32", n * self.n_hw),
            _dp(cfg, "int32", n), _dp(flag, "uint8", n), _stream(stream)))
        return cfg, flag

    def select_rows(self, op, target, lat, cfg=None, flag=None, stream=None):
        """Eq. 1 with a latency per (invocation, configuration): lat is [n, stride]."""
        import torch
        n = op.numel()
        stride = lat.shape[1] if lat.dim() == 2 else lat.numel() // max(n, 1)
        if cfg is None:
            cfg = torch.empty(n, dtype=torch.int32, device=op.device)
        if flag is None:
            flag = torch.empty(n, dtype=torch.uint8, device=op.device)
        self._check("llama_select_rows", self._L.llama_select_rows(
            self._ctx, n, _dp(op, "int32"), _dp(target, "int32", n * self.n_hw),
            _dp(lat, "int32", n * stride), int(stride), _dp(cfg, "int32", n), _dp(flag, "uint8", n),
            _stream(stream)))
        return cfg, flag

    def decide(self, op, elapsed, slo, queue=None, mode=SLACK_PAPER, scan=SCAN_AUTO, cfg=None,
               flag=None, stream=None, with_flag=True):
        import torch
        n = op.numel()
        if cfg is None:
            cfg = torch.empty(n, dtype=torch.int32, device=op.device)
        if flag is None and with_flag:
            flag = torch.empty(n, dtype=torch.uint8, device=op.device)
        self._check("llama_decide", self._L.llama_decide(
            self._ctx, n, _dp(op, "int32"), _dp(elapsed, "int32", n), _dp(slo, "int32", n),
            _dp(queue, "int64", self.n_hw), int(mode), int(scan), _dp(cfg, "int32", n),
            _dp(flag, "uint8", n), _stream(stream)))
        return cfg, flag

    def decide_full_noalloc(self, op, elapsed, slo, cfg, flag=None, queue=None, mode=SLACK_PAPER,
                            stream=None):
        """The full-scan decision into caller-allocated outputs, with the
        library's static per-GPU scratch (no device allocation)."""
        n = op.numel()
        self._check("llama_decide_full_noalloc", self._L.llama_decide_full_noalloc(
            self._ctx, n, _dp(op, "int32"), _dp(elapsed, "int32", n), _dp(slo, "int32", n),
            _dp(queue, "int64", self.n_hw), int(mode), _dp(cfg, "int32", n), _dp(flag, "uint8", n),
            _stream(stream)))
        return cfg, flag

    # -- Eq. 2 queueing time and the finite-alpha objective ------------------------
    def queue_time(self, q_op, q_cfg, out=None, stream=None):
        """Eq. 2 per backend from queued (op, configuration) pairs (device
        tensors); returns the int64 [n_hw] device tensor."""
        import torch
        n = q_op.numel()
        if out is None:
            out = torch.empty(self.n_hw, dtype=torch.int64, device=q_op.device)
        self._check("llama_queue_time", self._L.llama_queue_time(
            self._ctx, n, _dp(q_op, "int32"), _dp(q_cfg, "int32", n), _dp(out, "int64", self.n_hw),
            _stream(stream)))
        return out

    def feedback(self, obs_op, obs_cfg, obs_lat, beta_q16, stream=None):
        """Exponential smoothing of the profile from observations (device
        tensors), then the device rebuild of the tables and the relaxation."""
        n = obs_op.numel()
        self._check("llama_feedback", self._L.llama_feedback(
            self._ctx, n, _dp(obs_op, "int32"), _dp(obs_cfg, "int32", n), _dp(obs_lat, "int32", n),
            int(beta_q16), _stream(stream)))

    def decide_batching(self, op, elapsed, slo, available, upstream, wait_us, queue=None,
                        mode=SLACK_PAPER, cfg=None, flag=None, stream=None):
        """Safe delayed batching; per-op inputs are int32 device tensors [n_ops];
        cfg == CFG_WAIT marks a wait."""
        import torch
        n = op.numel()
        if cfg is None:
            cfg = torch.empty(n, dtype=torch.int32, device=op.device)
        if flag is None:
            flag = torch.empty(n, dtype=torch.uint8, device=op.device)
        self._check("llama_decide_batching", self._L.llama_decide_batching(
            self._ctx, n, _dp(op, "int32"), _dp(elapsed, "int32", n), _dp(slo, "int32", n),
            _dp(queue, "int64", self.n_hw), int(mode), _dp(available, "int32", self.n_ops),
            _dp(upstream, "int32", self.n_ops), _dp(wait_us, "int32", self.n_ops),
            _dp(cfg, "int32", n), _dp(flag, "uint8", n), _stream(stream)))
        return cfg, flag

    def affinity(self, op, elapsed, slo, queue=None, mode=SLACK_PAPER, aff=None, order=None,
                 with_order=True, stream=None):
        """Eq. 3 affinities [n, n_hw] (float64) and, optionally, the commit
        order [n_hw, n] (invocations by decreasing affinity per backend)."""
        import torch
        n = op.numel()
        if aff is None:
            aff = torch.empty((n, self.n_hw), dtype=torch.float64, device=op.device)
        if order is None and with_order:
            order = torch.empty((self.n_hw, n), dtype=torch.int32, device=op.device)
        self._check("llama_affinity", self._L.llama_affinity(
            self._ctx, n, _dp(op, "int32"), _dp(elapsed, "int32", n), _dp(slo, "int32", n),
            _dp(queue, "int64", self.n_hw), int(mode), _dp(aff, "float64", n * self.n_hw),
            _dp(order, "int32", n * self.n_hw), _stream(stream)))
        return aff, order

    def set_alpha(self, alpha_num, alpha_den=1):
        self._check("llama_set_alpha", self._L.llama_set_alpha(self._ctx, int(alpha_num), int(alpha_den)))

    def decide_alpha(self, op, elapsed, slo, queue=None, mode=SLACK_PAPER, cfg=None, flag=None,
                     stream=None):
        import torch
        n = op.numel()
        if cfg is None:
            cfg = torch.empty(n, dtype=torch.int32, device=op.device)
        if flag is None:
            flag = torch.empty(n, dtype=torch.uint8, device=op.device)
        self._check("llama_decide_alpha", self._L.llama_decide_alpha(
            self._ctx, n, _dp(op, "int32"), _dp(elapsed, "int32", n), _dp(slo, "int32", n),
            _dp(queue, "int64", self.n_hw), int(mode), _dp(cfg, "int32", n), _dp(flag, "uint8", n),
            _stream(stream)))
        return cfg, flag

    # -- introspection ----------------------------------------------------------
    def stats(self, reset_error=False):
        s = LlamaStats()
        self._check("llama_get_stats", self._L.llama_get_stats(self._ctx, ctypes.byref(s),
                                                               1 if reset_error else 0))
        return {k: getattr(s, k) for k, _ in LlamaStats._fields_}

    def export(self, what):
        n_ops, n_cfg = self.n_ops, self.n_cfg
        spec = {"W_paper": (0, np.int64, n_ops), "W_prob": (1, np.int64, n_ops),
                "key": (2, np.uint32, n_cfg), "ref": (3, np.int32, n_ops),
                "fastest": (4, np.int32, n_ops), "lat": (5, np.int32, n_cfg)}
        code, dt, n = spec[what]
        out = np.empty(n, dt)
        self._check("llama_debug_export", self._L.llama_debug_export(
            self._ctx, code, _hp(out), out.nbytes))
        return out

    # -- learned surrogate --------------------------------------------------------
    def surrogate_param_count(self):
        return int(self._L.llama_surrogate_param_count(self.n_cfg))

    def surrogate_init(self, seed=0, mean_log_latency=10.0):
        self._check("llama_surrogate_init",
                    self._L.llama_surrogate_init(self._ctx, int(seed), float(mean_log_latency)))

    def surrogate_set(self, params):
        p = _np(params, np.float32)
        self._check("llama_surrogate_set", self._L.llama_surrogate_set(self._ctx, _hp(p), p.size))

    def surrogate_get(self):
        out = np.empty(self.surrogate_param_count(), np.float32)
        self._check("llama_surrogate_get", self._L.llama_surrogate_get(self._ctx, _hp(out), out.size))
        return out

    def surrogate_grads(self):
        out = np.empty(self.surrogate_param_count(), np.float32)
        self._check("llama_surrogate_grads", self._L.llama_surrogate_grads(self._ctx, _hp(out), out.size))
        return out

    def surrogate_reserve(self, max_batch):
        self._check("llama_surrogate_reserve", self._L.llama_surrogate_reserve(self._ctx, int(max_batch)))

    def surrogate_forward(self, rows, feat, out=None, stream=None):
        import torch
        n = rows.numel()
        if out is None:
            out = torch.empty((n, 2), dtype=torch.float32, device=rows.device)
        self._check("llama_surrogate_forward", self._L.llama_surrogate_forward(
            self._ctx, n, _dp(rows, "int32"), _dp16(feat, 16 * n), _dp(out, "float32", 2 * n),
            _stream(stream)))
        return out

    def surrogate_train_step(self, rows, feat, y, lr, weight_decay=0.0, update=True, loss_sum=None,
                             stream=None):
        n = rows.numel()
        self._check("llama_surrogate_train_step", self._L.llama_surrogate_train_step(
            self._ctx, n, _dp(rows, "int32"), _dp16(feat, 16 * n), _dp(y, "float32", n),
            float(lr), float(weight_decay), 1 if update else 0, _dp(loss_sum, "float32", 1),
            _stream(stream)))

    def surrogate_fit(self, rows, feat, y, epochs=3, batch=4096, lr_max=5e-3, weight_decay=1e-4,
                      loss_sum=None, stream=None):
        n = rows.numel()
        self._check("llama_surrogate_fit", self._L.llama_surrogate_fit(
            self._ctx, n, _dp(rows, "int32"), _dp16(feat, 16 * n), _dp(y, "float32", n), int(epochs),
            int(batch), float(lr_max), float(weight_decay), _dp(loss_sum, "float32", 1),
            _stream(stream)))

    def surrogate_save(self, path):
        self._check("llama_surrogate_save", self._L.llama_surrogate_save(self._ctx, str(path).encode()))

    def surrogate_load(self, path):
        self._check("llama_surrogate_load", self._L.llama_surrogate_load(self._ctx, str(path).encode()))

    def set_simulator(self, a_coef, b_coef, sigma):
        """The simulator's content coefficients (numpy [n_ops, n_hw] and [n_ops]) and noise."""
        a = np.ascontiguousarray(a_coef, np.float64)
        b = np.ascontiguousarray(b_coef, np.float64)
        self._check("llama_set_simulator", self._L.llama_set_simulator(self._ctx, _hp(a), _hp(b), float(sigma)))

    def simulate(self, n, seed, first=0, stream=None):
        """n simulated executions on the GPU: (rows int32, features BF16 bits
        as int16 [n, 16], y float32) device tensors."""
        import torch
        rows = torch.empty(n, dtype=torch.int32, device="cuda")
        feat = torch.empty((n, 16), dtype=torch.int16, device="cuda")
        y = torch.empty(n, dtype=torch.float32, device="cuda")
        self._check("llama_simulate", self._L.llama_simulate(
            self._ctx, int(n), int(seed) & ((1 << 64) - 1), int(first), _dp(rows, "int32", n),
            _dp16(feat, 16 * n), _dp(y, "float32", n), _stream(stream)))
        return rows, feat, y

    def decide_learned(self, op, elapsed, slo, feat, queue=None, mode=SLACK_PAPER, spread_max=1.3862944,
                       cfg=None, flag=None, lat_out=None, lat_stride=0, stream=None):
        import torch
        n = op.numel()
        if cfg is None:
            cfg = torch.empty(n, dtype=torch.int32, device=op.device)
        if flag is None:
            flag = torch.empty(n, dtype=torch.uint8, device=op.device)
        self._check("llama_decide_learned", self._L.llama_decide_learned(
            self._ctx, n, _dp(op, "int32"), _dp(elapsed, "int32", n), _dp(slo, "int32", n),
            _dp(queue, "int64", self.n_hw), int(mode), _dp16(feat, 16 * n), float(spread_max),
            _dp(cfg, "int32", n), _dp(flag, "uint8", n),
            _dp(lat_out, "int32", n * lat_stride) if lat_out is not None else None,
            int(lat_stride), _stream(stream)))
        return cfg, flag


class Server:
    """Continuous-batching serving loop on one context (llama_serve_*)."""

    def __init__(self, llama, n_slots=65536, mem_budget_bytes=256 << 20, max_batch=65536,
                 max_inflight=4, learned=False, slack_mode=SLACK_PAPER, spread_max=1.3862944):
        self._llama = llama
        self._L = llama._L
        self.learned = bool(learned)
        cfg = ServeConfig(int(n_slots), int(mem_budget_bytes), int(max_batch), int(max_inflight),
                          1 if learned else 0, int(slack_mode), float(spread_max))
        self._srv = ctypes.c_void_p()
        llama._check("llama_serve_open", self._L.llama_serve_open(llama._ctx, ctypes.byref(cfg),
                                                                  ctypes.byref(self._srv)))
        # poll's output buffers and their pointers, reused across calls
        self._out = (np.empty(self.POLL_MAX, np.int64), np.empty(self.POLL_MAX, np.int32),
                     np.empty(self.POLL_MAX, np.uint8), np.empty(self.POLL_MAX, np.int64))
        self._out_p = tuple(_hp(a) for a in self._out)
        self._k = ctypes.c_int32()
        self._k_ref = ctypes.byref(self._k)

    POLL_MAX = 1 << 16

    def submit(self, op, elapsed, slo, feat=None, arrival_ns=None):
        """Offer requests (numpy); returns the admitted count and their tickets."""
        op, elapsed, slo = (_np(x, np.int32) for x in (op, elapsed, slo))
        n = len(op)
        f = None if feat is None else np.ascontiguousarray(feat, dtype=np.uint16)
        t = _np(arrival_ns, np.int64)
        tickets = np.empty(n, np.int64)
        k = ctypes.c_int32()
        rc = self._L.llama_serve_submit(self._srv, n, _hp(op), _hp(elapsed), _hp(slo), _hp(f), _hp(t),
                                        _hp(tickets), ctypes.byref(k))
        if rc != OK:
            raise LlamaError("llama_serve_submit", rc, "serving loop failed")
        return k.value, tickets[:k.value]

    def poll(self, max_n=1 << 16, wait_ms=0):
        """Collect up to max_n decisions (at most POLL_MAX a call): tickets,
        choices, flags, latencies in ns (numpy arrays of their own)."""
        max_n = min(int(max_n), self.POLL_MAX)
        rc = self._L.llama_serve_poll(self._srv, max_n, *self._out_p, self._k_ref, int(wait_ms))
        if rc != OK:
            raise LlamaError("llama_serve_poll", rc, "serving loop failed")
        n = self._k.value
        return tuple(a[:n].copy() for a in self._out)

    def stats(self):
        st = ServeStats()
        self._L.llama_serve_stats_get(self._srv, ctypes.byref(st))
        return {k: getattr(st, k) for k, _ in ServeStats._fields_}

    def close(self):
        if self._srv:
            rc = self._L.llama_serve_close(self._srv)
            self._srv = ctypes.c_void_p()
            if rc != OK:
                raise LlamaError("llama_serve_close", rc, "serving loop failed")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
