"""Benchmark of the per-invocation decision path on one MI355X.

One step = the whole plain decision path over one batch of pending
invocations already resident in HBM:
    relax  (remaining worst-path latency W and remaining-time thresholds)
    decide (Alg. 1 slack + Eq. 1 choice for every invocation)
captured as a HIP graph and replayed.  Default workload: 4,096 layered
pipeline DAGs of 3-200 ops (log-uniform), 16-2048 configurations per op
(log-uniform, from 4 hardware types x 64 batch sizes x 8 memory sizes),
4,000,000 invocations (seeded synthetic data); `--workload c2` runs 256 DAGs
of 10-40 ops with 64-512 configurations per op and 1,000,000 invocations.

Prints one JSON line.  `python bench.py --gpus N --steps K --warmup W`.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("invocation decisions/sec (bit-exact) + HBM GB/s frac; "
          "surrogate vs plain at ≤2% regret")
HBM_PEAK_GBS = 8000.0
# VALU integer lane-operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_GOPS = 256 * 64 * 2.4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--mode", choices=["paper", "prob"], default="paper")
    ap.add_argument("--workload", choices=["c2", "c3"], default="c3",
                    help="c3: 4,096 uneven pipelines, 4M invocations (default, the largest "
                         "single-GPU configuration); c2: 256 pipelines, 1M invocations")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the learned-surrogate section (training + fused inference)")
    ap.add_argument("--train-samples", type=int, default=10_000_000)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-loop section")
    ap.add_argument("--counter-pass", choices=["full", "learned"], default=None,
                    help="run only three launches of the full scan (C3 or C2, crossover 1/2) or of the "
                         "fused inference (C4 world, random-initialised surrogate, 1M invocations), for "
                         "rocprofv3 counter passes, and exit")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="for hardware-counter runs: a 256 MiB device copy (calibration) and a few "
                         "eager relax + decide launches on the benchmark workload, nothing timed")
    ap.add_argument("--serve-seconds", type=float, default=1.0)
    ap.add_argument("--no-pipeline", dest="pipeline", action="store_false",
                    help="run each step's relaxation and decisions back to back on one stream "
                         "(default: the relaxation of step k+1 overlaps the decisions of step k)")
    ap.add_argument("--steps-per-graph", type=int, default=20,
                    help="steps captured in one HIP graph (the timed loop replays it, then a "
                         "one-step graph for the remainder, so exactly --steps steps run)")
    ap.add_argument("--no-next1", action="store_true",
                    help="skip the queueing-time + finite-alpha section")
    ap.add_argument("--queue-entries", type=int, default=1_000_000)
    ap.add_argument("--no-next2", action="store_true", help="skip the feedback section")
    ap.add_argument("--feedback-obs", type=int, default=100_000)
    ap.add_argument("--no-next3", action="store_true", help="skip the affinity section")
    ap.add_argument("--next3-sample", type=int, default=5_000)
    ap.add_argument("--no-next4", action="store_true", help="skip the safe delayed batching section")
    ap.add_argument("--next1-sample", type=int, default=50_000)
    ap.add_argument("--kernel-reps", type=int, default=50,
                    help="launches per graph when timing single kernels")
    return ap.parse_args()


# kernel of each decision schedule (llama_autotune's numbering)
# (the LDS-staged schedule runs its 16-byte variant: the bench's arrays are aligned)
def schedule_kernel(sched):
    """Kernel name of a decision schedule (llama_autotune's numbering; the
    LDS-staged schedule runs its 16-byte variant: the bench's arrays are
    aligned)."""
    if sched == 3:
        return "decide_lds4_kernel"
    ipt, nt = ((1, "false"), (2, "false"), (4, "false"), None, (1, "true"), (2, "true"), (4, "true"))[sched]
    return f"void decide_indexed_kernel<{ipt}, {nt}>"


DECISION_PATH_END = b"// DECISION-PATH-END"


def decision_path_digest():
    """sha256 of the decision path's device source: llama_kernels.hip up to
    its DECISION-PATH-END marker (records, relaxation, decision kernels and
    their launchers)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2102_01887_amd", "csrc")
    with open(os.path.join(csrc, "llama_kernels.hip"), "rb") as f:
        text = f.read()
    cut = text.find(DECISION_PATH_END)
    if cut < 0:
        raise RuntimeError("llama_kernels.hip has no DECISION-PATH-END marker")
    return hashlib.sha256(text[:cut]).hexdigest()


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (rocprofv3 FETCH_SIZE and WRITE_SIZE, scaled by a device copy), or None
    when there is none or the decision path's source has changed since it
    was taken."""
    path = os.path.join(ROOT, "profiles", f"decide_plain_{workload}_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    digest = decision_path_digest()
    recorded, table = None, {}
    for line in open(path):
        if line.startswith("decision path sha256:"):
            recorded = line.split(":", 1)[1].strip()
        elif line.startswith("traffic_bytes_per_launch "):
            name, value = line[len("traffic_bytes_per_launch "):].rsplit(":", 1)
            table[name.strip()] = int(value)
    if recorded != digest:
        return None
    return table.get(kernel)


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def graph_of(torch, stream, fn, reps):
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        for _ in range(reps):
            fn()
    return g


def time_graph(torch, stream, g, replays):
    """Average device time of one replay (HIP events on the replay stream)."""
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        g.replay()
        a.record(stream)
        for _ in range(replays):
            g.replay()
        b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / replays


def device_copy_gbs(torch, stream, mib=512, reps=10):
    """Bytes read + written per second by a device-to-device copy of `mib`
    MiB (the runtime's copy kernel), HIP events on the copy stream: the
    bandwidth a plain streaming kernel reaches, a second denominator."""
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    with torch.cuda.stream(stream):
        dst.copy_(src)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            dst.copy_(src)
        b.record(stream)
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    return 2 * (mib << 20) / (ms * 1e-3) / 1e9


# BF16 dense MFMA peak (MI355X) in TFLOP/s; FLOPs per surrogate row (forward)
MFMA_BF16_PEAK_TFS = 2500.0
ROW_FLOPS = 2 * (32 * 256 + 256 * 256 + 256 * 2)


def bench_next1(args, torch, B, wl, log, w, op, el, slo, mode):
    """Eq. 2 queueing time over a queue snapshot, then Alg. 1 with that Q and
    the finite-alpha Eq. 1 (alpha = 1), chained on the device; parity on a
    sample against the oracle."""
    import numpy as np
    n = w.n_inv
    rng = np.random.default_rng(17)
    n_q = args.queue_entries
    q_op, q_cfg = wl.queue_snapshot(w, rng, n_q)
    # pools sized so that the backlog waits 0.2 s to 2 s depending on the backend
    waits = np.resize(np.array([200_000, 500_000, 1_000_000, 2_000_000]), w.n_hw)
    wr = wl.with_resource_totals(w, per_hw=wl.totals_for_queue(w, q_op, q_cfg, waits))
    L = B.Llama(0).load(wr)
    dq_op = torch.from_numpy(q_op).cuda()
    dq_cfg = torch.from_numpy(q_cfg).cuda()
    L.set_alpha(1, 1)
    s = torch.cuda.Stream()
    Q = torch.empty(w.n_hw, dtype=torch.int64, device="cuda")
    cfg = torch.empty(n, dtype=torch.int32, device="cuda")
    flag = torch.empty(n, dtype=torch.uint8, device="cuda")

    def qt():
        L.queue_time(dq_op, dq_cfg, out=Q, stream=s)

    def da():
        L.decide_alpha(op, el, slo, Q, mode, cfg, flag, stream=s)

    def da0():
        L.decide_alpha(op, el, slo, None, mode, cfg, flag, stream=s)

    def chain():
        qt()
        da()

    with torch.cuda.stream(s):
        for _ in range(3):
            chain()
    torch.cuda.synchronize()
    reps = args.kernel_reps
    ms_q = time_graph(torch, s, graph_of(torch, s, qt, reps), 5) / reps
    ms_a = time_graph(torch, s, graph_of(torch, s, da, reps), 5) / reps
    ms_0 = time_graph(torch, s, graph_of(torch, s, da0, reps), 5) / reps
    with torch.cuda.stream(s):
        da0()
    torch.cuda.synchronize()
    c0, f0 = cfg.cpu().numpy(), flag.cpu().numpy()
    ms_c = time_graph(torch, s, graph_of(torch, s, chain, reps), 5) / reps
    # parity: Q exactly, decisions on a sample of invocations
    import oracle
    P = oracle.Problem(wr)
    Q_or, _ = P.queue_time(q_op, q_cfg)
    sample = slice(0, min(n, args.next1_sample))
    c_or, f_or = P.decide_alpha(mode, 1, 1, Q=Q_or, sl=sample)
    cg, fg = cfg.cpu().numpy()[sample], flag.cpu().numpy()[sample]
    c0_or, f0_or = P.decide_alpha(mode, 1, 1, Q=None, sl=sample)
    exact = bool(np.array_equal(Q.cpu().numpy(), Q_or) and np.array_equal(cg, c_or)
                 and np.array_equal(fg, f_or) and np.array_equal(c0[sample], c0_or)
                 and np.array_equal(f0[sample], f0_or))
    q_bytes = n_q * (8 + 12)
    # the library merges each op's backends per call only when the call's
    # invocations pay for it (8 n_inv >= n_cfg): then per configuration the
    # merge reads its latency and two keys and writes the merged threshold
    # and two minima; otherwise the invocations are grouped by op, each op's
    # latency runs are read once and each invocation reads one pair of key
    # minima per backend.  Per invocation 17 B.
    merged = 8 * n >= wr.n_cfg
    a_bytes = n * 17 + (wr.n_cfg * 24 if merged else wr.n_cfg * 4 + n * wr.n_hw * 8)
    a_kernel = ("alpha_merge_kernel + alpha_queue_kernel" if merged else
                "grouping by op (bucket_hist/place/fine) + decide_alpha_ops_kernel (per backend: the op's "
                "latency runs in registers, counts by ballot)")
    log(f"bench: next1 queue_time {ms_q * 1e3:.2f} us, decide_alpha {ms_a * 1e3:.2f} us, exact {exact}")
    return {"alpha": [1, 1], "hw_res_total": wr.hw_res_total.tolist(), "queue_entries": n_q,
            "Q_us": Q_or.tolist(), "ms_per_chain": ms_c, "decisions_per_s": n / (ms_c * 1e-3),
            "met_slack": float(flag.float().mean().item()),
            "queue_time": {"kernel": "queue_accumulate_kernel", "ms": ms_q,
                           "roofline": {"bound": "hbm", "achieved": q_bytes / (ms_q * 1e-3) / 1e9,
                                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                        "frac": q_bytes / (ms_q * 1e-3) / 1e9 / HBM_PEAK_GBS}},
            "decide_alpha": {"kernel": a_kernel, "ms": ms_a,
                             "roofline": {"bound": "hbm", "achieved": a_bytes / (ms_a * 1e-3) / 1e9,
                                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                          "frac": a_bytes / (ms_a * 1e-3) / 1e9 / HBM_PEAK_GBS}},
            "decide_alpha_without_queue": {"kernel": "decide_alpha_merged_kernel", "ms": ms_0,
                                           "decisions_per_s": n / (ms_0 * 1e-3)},
            "bit_exact": exact,
            "parity_sample": f"Q exactly; decisions of the first {sample.stop} invocations, "
                             f"with and without the queueing times"}


def bench_next2(args, torch, B, wl, log, w, op, el, slo, mode):
    """Feedback: smoothing of the profile from a batch of observations and the
    device rebuild of the tables, then the decision of the invocation batch;
    parity of one call against the oracle (latencies exactly, decisions on a
    sample)."""
    import numpy as np
    import oracle
    n = w.n_inv
    rng = np.random.default_rng(23)
    n_obs = args.feedback_obs
    ob = [torch.from_numpy(a).cuda() for a in wl.observations(w, rng, n_obs)]
    beta = 13107  # 0.2
    L = B.Llama(0).load(w)
    s = torch.cuda.Stream()
    cfg = torch.empty(n, dtype=torch.int32, device="cuda")
    flag = torch.empty(n, dtype=torch.uint8, device="cuda")
    with torch.cuda.stream(s):
        L.feedback(*ob, beta, stream=s)
        L.decide(op, el, slo, None, mode, B.SCAN_INDEXED, cfg, flag, stream=s)
    torch.cuda.synchronize()
    lat_or, _ = oracle.feedback(*(a.cpu().numpy() for a in ob), w.cfg_off, w.lat, beta)
    w2 = w.with_invocations(w.inv_op, w.elapsed, w.slo)
    w2.lat = lat_or
    sample = slice(0, min(n, args.next1_sample))
    c_or, f_or = oracle.Problem(w2).decide(mode, sl=sample)
    exact = bool(np.array_equal(L.export("lat"), lat_or)
                 and np.array_equal(cfg.cpu().numpy()[sample], c_or)
                 and np.array_equal(flag.cpu().numpy()[sample], f_or))

    def fb():
        L.feedback(*ob, beta, stream=s)

    def step():
        fb()
        L.decide(op, el, slo, None, mode, B.SCAN_INDEXED, cfg, flag, stream=s)

    reps = max(1, args.kernel_reps // 5)
    ms_fb = time_graph(torch, s, graph_of(torch, s, fb, reps), 3) / reps
    ms_step = time_graph(torch, s, graph_of(torch, s, step, reps), 3) / reps
    # bytes of the rebuild per configuration: L, key, backend, key order read
    # (14 B), frontier, merged-frontier and full-table writes (8 + 8 + 4 B)
    rb_bytes = w.n_cfg * 34
    log(f"bench: next2 feedback {ms_fb * 1e3:.1f} us, step {ms_step * 1e3:.1f} us, exact {exact}")
    return {"observations": n_obs, "beta_q16": beta,
            "ms_feedback": ms_fb, "ms_per_step": ms_step,
            "decisions_per_s": n / (ms_step * 1e-3), "observations_per_s": n_obs / (ms_fb * 1e-3),
            "step": "feedback (smoothing + table rebuild + relaxation) + decide",
            "rebuild_roofline": {"bound": "hbm", "achieved": rb_bytes / (ms_fb * 1e-3) / 1e9,
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": rb_bytes / (ms_fb * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                 "note": "whole feedback call, 34 B per configuration"},
            "bit_exact": exact,
            "parity_sample": f"latencies exactly; decisions of the first {sample.stop} invocations"}


def bench_next3(args, torch, B, wl, log, w, op, el, slo, mode):
    """Eq. 3 affinities of every invocation to every backend and the commit
    order per backend (alpha = 1); parity on a sample against the oracle."""
    import numpy as np
    import oracle
    n = w.n_inv
    wr = wl.with_resource_totals(w)
    L = B.Llama(0).load(wr)
    L.set_alpha(1, 1)
    s = torch.cuda.Stream()
    aff = torch.empty((n, w.n_hw), dtype=torch.float64, device="cuda")
    order = torch.empty((w.n_hw, n), dtype=torch.int32, device="cuda")
    with torch.cuda.stream(s):
        L.affinity(op, el, slo, None, mode, aff, order, stream=s)
    torch.cuda.synchronize()

    def only_aff():
        L.affinity(op, el, slo, None, mode, aff, None, with_order=False, stream=s)

    def with_order():
        L.affinity(op, el, slo, None, mode, aff, order, stream=s)

    reps = max(1, args.kernel_reps // 5)
    ms_a = time_graph(torch, s, graph_of(torch, s, only_aff, reps), 3) / reps
    ms_o = time_graph(torch, s, graph_of(torch, s, with_order, reps), 3) / reps
    sample = slice(0, min(n, args.next3_sample))
    want = oracle.Problem(wr).affinity(mode, 1, 1, sl=sample)
    got = aff.cpu().numpy()[sample]
    special = ~np.isfinite(want) | (want == 0) | (want == 1)
    rel = np.abs(got[~special] - want[~special]) / np.abs(want[~special])
    ok = bool(np.array_equal(got[special], want[special]) and (rel.size == 0 or rel.max() <= 1e-15))
    o = order.cpu().numpy()
    a = aff.cpu().numpy()
    ordered = all(bool((a[o[h], h][:-1] >= a[o[h], h][1:]).all()) for h in range(w.n_hw))
    log(f"bench: next3 affinity {ms_a * 1e3:.1f} us, with commit order {ms_o * 1e3:.1f} us, within 1e-15 {ok}")
    return {"alpha": [1, 1], "ms_affinity": ms_a, "ms_affinity_and_order": ms_o,
            "invocations_per_s": n / (ms_o * 1e-3),
            "kernel": "grouping by op (bucket_hist/place/fine) + affinity_ops_kernel (per backend: the op's latency runs in registers, counts by ballot)",
            "order": "per backend, stable radix sort of the complemented affinity bits",
            "within_tolerance": ok, "max_rel_error": float(rel.max()) if rel.size else 0.0,
            "order_non_increasing": ordered,
            "parity_sample": f"affinities of the first {sample.stop} invocations, relative 1e-15"}


def bench_next4(args, torch, B, wl, log, L, w, op, el, slo, mode):
    """Safe delayed batching over the invocation batch: per op, invocations
    available U{1..64}, expected from upstream U{0..64}, estimated wait
    U[0, 0.2 s]; parity on a sample against the oracle."""
    import numpy as np
    import oracle
    n = w.n_inv
    rng = np.random.default_rng(29)
    per_op = [rng.integers(1, 65, w.n_ops), rng.integers(0, 65, w.n_ops), rng.integers(0, 200_001, w.n_ops)]
    per_op = [torch.from_numpy(a.astype(np.int32)).cuda() for a in per_op]
    s = torch.cuda.Stream()
    cfg = torch.empty(n, dtype=torch.int32, device="cuda")
    flag = torch.empty(n, dtype=torch.uint8, device="cuda")

    def run():
        L.decide_batching(op, el, slo, *per_op, None, mode, cfg, flag, stream=s)

    with torch.cuda.stream(s):
        run()
    torch.cuda.synchronize()
    reps = max(1, args.kernel_reps // 5)
    ms = time_graph(torch, s, graph_of(torch, s, run, reps), 3) / reps
    sample = slice(0, min(n, args.next1_sample))
    c_or, f_or = oracle.Problem(w).decide_batching(mode, *(a.cpu().numpy() for a in per_op), sl=sample)
    c, f = cfg.cpu().numpy(), flag.cpu().numpy()
    exact = bool(np.array_equal(c[sample], c_or) and np.array_equal(f[sample], f_or))
    log(f"bench: next4 safe delayed batching {ms * 1e3:.1f} us, exact {exact}")
    # invocations whose x* needs more than is available and that do not wait
    # are the ones the scan kernel visits; estimated from the oracle's x* on
    # the parity sample
    avail = per_op[0].cpu().numpy()
    xs_or, _ = oracle.Problem(w).decide(mode, sl=sample)
    v_s = w.inv_op[sample]
    scanned = (w.batch[w.cfg_off[v_s] + xs_or] > avail[v_s]) & (c_or != B.CFG_WAIT)
    n_cfg_op = np.diff(w.cfg_off)
    pairs = int(round(n_cfg_op[v_s][scanned].sum() * n / len(v_s)))
    ops = pairs * 3
    return {"ms": ms, "decisions_per_s": n / (ms * 1e-3),
            "kernels": "batching_commit_kernel (records) + grouping by op (bucket_hist/place/fine over the "
                       "sub-queue slots) + batching_ops_kernel (scans)",
            "wait_fraction": float(np.mean(c == B.CFG_WAIT)), "scan_fraction": float(scanned.mean()),
            "roofline": {"bound": "alu", "achieved": ops / (ms * 1e-3) / 1e9, "peak": 39321.6,
                         "unit": "Gop/s", "frac": ops / (ms * 1e-3) / 1e9 / 39321.6,
                         "note": "3 lane-ops per scanned (invocation, configuration) pair (compare, select, min); "
                                 "scanned pairs estimated from the parity sample"},
            "bit_exact": exact, "parity_sample": f"decisions of the first {sample.stop} invocations"}


def bench_surrogate(args, torch, B, wl, log):
    """Draw the training executions with the GPU simulator, train the
    surrogate with the full recipe on the GPU, time the fused inference kernel
    on 1M invocations x 64 configurations, and score its decisions against
    the simulator's truth (and the plain profile's)."""
    import numpy as np
    world = wl.make_c4_world(3)
    L = B.Llama(0).load(world.w)
    L.surrogate_init(seed=15, mean_log_latency=10.5)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    bf = lambda f: torch.from_numpy(np.ascontiguousarray(f, np.float32)).to(torch.bfloat16).cuda()
    s = torch.cuda.Stream()
    # training executions drawn on the device (llama_simulate), timed
    log(f"bench: simulating {args.train_samples} training executions on the GPU")
    L.set_simulator(world.a, world.b, world.sigma)
    L.simulate(4096, 1, stream=s)  # warm-up
    sa, sb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        sa.record(s)
        d_rows, d_feat, d_y = L.simulate(args.train_samples, 7, stream=s)
        sb.record(s)
    sb.synchronize()
    sim_ms = sa.elapsed_time(sb)
    epochs, batch = 3, 4096
    steps = epochs * (args.train_samples // batch)
    L.surrogate_reserve(batch)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    log(f"bench: training {steps} steps")
    with torch.cuda.stream(s):
        a.record(s)
        L.surrogate_fit(d_rows, d_feat, d_y, epochs=epochs, batch=batch, lr_max=5e-3,
                        weight_decay=1e-4, loss_sum=loss, stream=s)
        b.record(s)
    b.synchronize()
    train_ms = a.elapsed_time(b)
    final_loss = loss.item() / (((args.train_samples // batch + 9) // 10) * batch)
    del d_rows, d_feat, d_y
    n = 1_000_000
    w4, c4 = wl.c4_invocations(world, np.random.default_rng(8), n)
    op, el, slo, feat = dev(w4.inv_op), dev(w4.elapsed), dev(w4.slo), bf(c4.feat)
    cfg = torch.empty(n, dtype=torch.int32, device="cuda")
    flag = torch.empty(n, dtype=torch.uint8, device="cuda")
    learned = lambda: L.decide_learned(op, el, slo, feat, cfg=cfg, flag=flag, stream=s)
    plain = lambda: L.decide(op, el, slo, cfg=cfg, flag=flag, stream=s)
    with torch.cuda.stream(s):
        learned()
        plain()
    torch.cuda.synchronize()
    g_l = graph_of(torch, s, learned, 2)
    g_p = graph_of(torch, s, plain, 20)
    ms_l = time_graph(torch, s, g_l, 3) / 2
    ms_p = time_graph(torch, s, g_p, 3) / 20
    tflops = n * 64 * ROW_FLOPS / (ms_l * 1e-3) / 1e12
    # decisions on a sample, scored against the simulator's truth by the
    # oracle: targets (Alg. 1), the truth p95 latencies, the truth decision
    # (Eq. 1 on them) and the regret / miss rate all come from oracle/
    import oracle
    from oracle import mlp
    m = 20_000
    sl = slice(0, m)
    wm = w4.with_invocations(w4.inv_op[:m], w4.elapsed[:m], w4.slo[:m])
    tgt = oracle.Problem(wm).targets(0)
    ww = world.w
    rows = wm.inv_op[:, None].astype(np.int64) * 64 + np.arange(64)[None, :]
    op_m = wm.inv_op[:, None]
    mu = mlp.truth_mean_log_latency(ww.lat[rows], world.a[op_m, ww.hw[rows]], world.b[op_m],
                                    c4.n_obj[:m, None], c4.px[:m, None])
    truth = mlp.truth_p95_latency(mu, world.sigma).astype(np.int32)
    t_c, t_f = oracle.select_lat(wm.inv_op, tgt, ww.n_hw, ww.cfg_off, ww.hw, ww.batch, truth, ww.cost)
    s_c, _ = L.decide_learned(op[sl], el[sl], slo[sl], feat[sl])
    p_c, _ = L.decide(op[sl], el[sl], slo[sl])
    torch.cuda.synchronize()
    base = (wm.inv_op * 64).astype(np.int64)
    r_s = mlp.regret(s_c.cpu().numpy(), t_c, t_f, truth, tgt, ww.hw, ww.cost, ww.batch, base)
    r_p = mlp.regret(p_c.cpu().numpy(), t_c, t_f, truth, tgt, ww.hw, ww.cost, ww.batch, base)
    args._surrogate_ctx = (L, world)
    return {
        "workload": "c4: C1's 6-op DAG, 64 configs/op; train 10M simulator samples x 3 epochs "
                    "(batch 4096, AdamW, cosine lr 5e-3); infer 1M invocations x 64 configs",
        "simulator": {"kernel": "simulate_kernel (Philox4x32-10, FP64 transforms)",
                      "samples": args.train_samples, "ms": sim_ms,
                      "samples_per_s": args.train_samples / (sim_ms * 1e-3)},
        "train_ms": train_ms, "train_steps": steps,
        "train_samples_per_s": epochs * args.train_samples / (train_ms * 1e-3),
        "final_loss": final_loss,
        "inference_ms": ms_l, "decisions_per_s": n / (ms_l * 1e-3),
        "plain_decisions_per_s_same_workload": n / (ms_p * 1e-3),
        "throughput_vs_plain": ms_p / ms_l,
        "roofline": {"bound": "mfma", "achieved": tflops, "peak": MFMA_BF16_PEAK_TFS,
                     "unit": "TFLOP/s", "frac": tflops / MFMA_BF16_PEAK_TFS,
                     "kernel": "decide_learned_kernel", "flops_per_row": ROW_FLOPS},
        "regret_surrogate": r_s, "regret_plain_profile": r_p, "regret_sample": m,
        "dtype": "bf16 (fp32 accumulate)",
    }


def drive_poisson(srv, op, el, slo, rate, duration, seed, feat=None):
    """Offer a Poisson stream of the given rate for `duration` seconds (numpy
    request arrays).  Returns per-request latency (ns) from submission to the
    device time of the decision, the same from the scheduled arrival (which
    adds this Python load generator's lag), the sustained rate and the
    requests the ring did not admit at their first offer."""
    import numpy as np
    from paper_2102_01887_amd import workloads as wl
    off = wl.poisson_arrivals(np.random.default_rng(seed), rate, duration)
    n = min(len(off), len(op))
    t0 = time.monotonic_ns() + 2_000_000
    arr = t0 + off[:n]
    sub = np.zeros(n, np.int64)
    i = done = 0
    refused = 0
    lats, tick = [], []
    while done < n:
        now = time.monotonic_ns()
        j = int(np.searchsorted(arr, now, side="right"))
        if j > i:
            k, tk = srv.submit(op[i:j], el[i:j], slo[i:j], None if feat is None else feat[i:j])
            sub[i:i + k] = now
            refused += (j - i) - k
            i += k
        t, _, _, lat = srv.poll(wait_ms=0)
        done += len(t)
        lats.append(lat)
        tick.append(t)
    elapsed = (time.monotonic_ns() - t0) * 1e-9
    lat, tick = np.concatenate(lats), np.concatenate(tick)
    from_arrival = lat + (sub[tick] - arr[tick])
    return lat, from_arrival, n / elapsed, refused


def serve_runs(srv_factory, op, el, slo, rates, seconds, log, label, feat=None):
    import numpy as np
    out = []
    srv = srv_factory()
    drive_poisson(srv, op, el, slo, rates[0], 0.2, 1, feat=feat)  # warm-up, not reported
    srv.close()
    for rate in rates:
        srv = srv_factory()
        lat, lat_arr, sustained, refused = drive_poisson(srv, op, el, slo, rate, seconds, rate, feat=feat)
        st = srv.stats()
        srv.close()
        p50, p99 = (np.percentile(lat, [50, 99]) / 1e3).tolist()
        a50, a99 = (np.percentile(lat_arr, [50, 99]) / 1e3).tolist()
        log(f"bench: serve {label} {rate}/s -> p50 {p50:.1f} us p99 {p99:.1f} us "
            f"(from scheduled arrival {a50:.1f} / {a99:.1f}), {sustained:.0f}/s, "
            f"{st['batches']} claims, {st['kernel_launches']} launches, "
            f"clock {st['clock_anchors']} anchors, rate {st['clock_rate_ppb'] / 1e3:+.1f} ppm")
        out.append({"offered_per_s": rate, "decisions": int(len(lat)), "sustained_per_s": sustained,
                    "p50_us": p50, "p99_us": p99, "p50_from_arrival_us": a50, "p99_from_arrival_us": a99,
                    "claims": st["batches"], "mean_claim": len(lat) / max(1, st["batches"]),
                    "largest_claim": st["max_batch_seen"], "kernel_launches": st["kernel_launches"],
                    "capacity": st["capacity"], "peak_bytes_in_use": st["peak_bytes_in_use"],
                    "refused_at_first_offer": refused, "clock_rtt_us": st["clock_rtt_ns"] / 1e3,
                    "clock_anchors": st["clock_anchors"], "clock_rate_ppm": st["clock_rate_ppb"] / 1e3})
    return out


def bench_serving(args, torch, B, wl, log, surrogate_ctx=None):
    """Serving loop on C5 (1,024 uneven pipelines): Poisson arrivals at
    50k-500k/s, 65,536 slots, 256 MB admission budget; p50/p99 latency from
    submission to the device time of the decision, and the sustained rate.
    A last run gives the ring a 64 KiB budget (2,048 plain slots), so memory,
    not slots, limits admission."""
    import numpy as np
    log("bench: generating workload c5 (1,024 pipelines)")
    w = wl.make_c5(n_inv=600_000)
    L = B.Llama(0).load(w)
    out = {"workload": "c5: 1,024 layered pipelines of 3-200 ops, 16-2048 configs/op, "
                       "Poisson arrivals, 65,536 slots, 256 MB admission budget",
           "n_ops": w.n_ops, "n_cfg": w.n_cfg,
           "path": "persistent decision kernel (HIP graph, relaunched when it has exited) fed from a "
                   "device-mapped ring; device-clock decision times",
           "bytes_per_request": {"plain": int(L._L.llama_serve_bytes_per_request(0)),
                                 "learned": int(L._L.llama_serve_bytes_per_request(1))}}
    plain = lambda budget=256 << 20: B.Server(L, n_slots=65536, mem_budget_bytes=budget, max_batch=64,
                                             max_inflight=4)
    out["plain"] = serve_runs(plain, w.inv_op, w.elapsed, w.slo, (50_000, 100_000, 200_000, 500_000),
                              args.serve_seconds, log, "plain")
    out["plain_memory_bound"] = serve_runs(lambda: plain(64 << 10), w.inv_op, w.elapsed, w.slo, (500_000,),
                                           args.serve_seconds, log, "plain, 64 KiB budget")
    if surrogate_ctx is not None:
        Ls, world = surrogate_ctx
        wq, content = wl.c4_invocations(world, np.random.default_rng(9), 400_000)
        bits = (np.ascontiguousarray(content.feat, np.float32).view(np.uint32) >> 16).astype(np.uint16)
        learned = lambda: B.Server(Ls, n_slots=65536, mem_budget_bytes=256 << 20, max_batch=1,
                                   max_inflight=16, learned=True)
        out["learned"] = serve_runs(learned, wq.inv_op, wq.elapsed, wq.slo, (50_000, 200_000),
                                    args.serve_seconds, log, "learned", feat=bits)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the decision path "
              "is measured on one GPU's share of the pipelines; it has no multi-GPU launcher",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2102_01887_amd import binding as B
    from paper_2102_01887_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    mode = B.SLACK_PAPER if args.mode == "paper" else B.SLACK_PROB

    if args.counter_pass:
        import numpy as np
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        if args.counter_pass == "full":
            log(f"bench: full-scan counter pass on {args.workload}")
            w = wl.make_c2() if args.workload == "c2" else wl.make_c3()
            L = B.Llama(0).load(w)
            op, el, slo = dev(w.inv_op), dev(w.elapsed), dev(w.slo)
            L.relax(modes=1 << mode)
            L.reserve(w.n_inv)
            L.set_full_schedule(1, 2)
            for _ in range(3):
                L.decide(op, el, slo, None, mode, B.SCAN_FULL)
            n = w.n_inv
        else:
            log("bench: fused-inference counter pass on the C4 world")
            world = wl.make_c4_world(3)
            L = B.Llama(0).load(world.w)
            L.surrogate_init(seed=15, mean_log_latency=10.5)
            n = 1_000_000
            w4, c4 = wl.c4_invocations(world, np.random.default_rng(8), n)
            feat = torch.from_numpy(np.ascontiguousarray(c4.feat, np.float32)).to(torch.bfloat16).cuda()
            op, el, slo = dev(w4.inv_op), dev(w4.elapsed), dev(w4.slo)
            for _ in range(3):
                L.decide_learned(op, el, slo, feat)
        torch.cuda.synchronize()
        print(json.dumps({"counter_pass": args.counter_pass, "invocations": n}), flush=True)
        return

    if args.pmc_pass:
        import numpy as np
        log(f"bench: counter pass on {args.workload}")
        w = wl.make_c2() if args.workload == "c2" else wl.make_c3()
        L = B.Llama(0).load(w)
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        op, el, slo = dev(w.inv_op), dev(w.elapsed), dev(w.slo)
        L.autotune(op, el, slo)
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")  # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        for _ in range(5):
            L.relax(modes=1)
            L.decide(op, el, slo)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_pass": args.workload, "copy_bytes": src.numel() * 4,
                          "decide_algo_bytes": w.n_inv * 17}), flush=True)
        return

    log(f"bench: generating workload {args.workload}")
    w = wl.make_c2() if args.workload == "c2" else wl.make_c3()
    L = B.Llama(0).load(w)
    st = L.stats()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    op, el, slo = dev(w.inv_op), dev(w.elapsed), dev(w.slo)
    n = w.n_inv
    cfg = torch.empty(n, dtype=torch.int32, device="cuda")
    flag = torch.empty(n, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()

    def relax():
        # W for both slack modes; thresholds for the mode the step decides in
        L.relax(stream=s, modes=1 << mode)

    def decide(scan):
        return lambda: L.decide(op, el, slo, None, mode, scan, cfg, flag, stream=s)

    def step():
        relax()
        decide(B.SCAN_INDEXED)()

    tuned = L.autotune(op, el, slo, stream=s)
    log(f"bench: autotuned decision schedule: {B.SCHEDULE_NAMES[tuned[0]]} ({tuned[1]:.2f} us)")

    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        for _ in range(args.warmup):
            step()
    torch.cuda.synchronize()
    log("bench: capturing graphs")
    g_step = graph_of(torch, s, step, 1)
    spg = max(1, min(args.steps_per_graph, args.steps))
    s_dec = torch.cuda.Stream()

    def pipelined_graph(n_steps):
        """n_steps steps in one graph on two streams: the relaxation of step
        k+1 (stream s) overlaps the decisions of step k (stream s_dec); the
        relaxations alternate between the two record sets, so the one of
        step k+2 waits for the decisions of step k."""
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            fork = torch.cuda.Event()
            fork.record(s)
            s_dec.wait_event(fork)
            done = [None, None]
            last = None
            for k in range(n_steps):
                if done[k % 2] is not None:
                    s.wait_event(done[k % 2])
                relax()
                ready = torch.cuda.Event()
                ready.record(s)
                s_dec.wait_event(ready)
                L.decide(op, el, slo, None, mode, B.SCAN_INDEXED, cfg, flag, stream=s_dec)
                last = torch.cuda.Event()
                last.record(s_dec)
                done[k % 2] = last
            s.wait_event(last)
        return g

    g_steps = pipelined_graph(spg) if args.pipeline else graph_of(torch, s, step, spg)
    g_dec = graph_of(torch, s, decide(B.SCAN_INDEXED), args.kernel_reps)
    L.reserve(n)
    full_cross, full_tuned_us = L.autotune_full(op, el, slo, mode, stream=s)
    log(f"bench: full-scan schedule crossover {full_cross[0]}/{full_cross[1]} ({full_tuned_us:.1f} us)")
    g_full = graph_of(torch, s, decide(B.SCAN_FULL), max(1, args.kernel_reps // 10))
    g_wave = graph_of(torch, s, decide(B.SCAN_WAVE), 2)
    g_relax = graph_of(torch, s, relax, args.kernel_reps)
    with torch.cuda.stream(s):
        for _ in range(args.warmup):
            g_step.replay()
    torch.cuda.synchronize()

    # ---- timed region: exactly K steps ------------------------------------
    log(f"bench: timing {args.steps} steps")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(s):
        ev0.record(s)
        for _ in range(args.steps // spg):
            g_steps.replay()
        for _ in range(args.steps % spg):
            g_step.replay()
        ev1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step_dev = ev0.elapsed_time(ev1) / args.steps
    ms_step = max(wall * 1e3 / args.steps, ms_step_dev)

    # ---- single-kernel durations (HIP events over graphs of R launches) ----
    ms_dec = time_graph(torch, s, g_dec, 5) / args.kernel_reps
    ms_full = time_graph(torch, s, g_full, 3) / max(1, args.kernel_reps // 10)
    ms_wave = time_graph(torch, s, g_wave, 2) / 2
    ms_relax = time_graph(torch, s, g_relax, 5) / args.kernel_reps
    copy_gbs = device_copy_gbs(torch, s)

    # algorithmic bytes of one decide launch (indexed form):
    # 12 B invocation input + 4 B choice + 1 B flag per invocation, plus each
    # op's frontier (8 B per entry) and header once.
    hs = (w.n_hw + 2 + 3) & ~3
    algo_bytes = n * 17 + st["frontier_entries"] * 8 + w.n_ops * hs * 4
    achieved = algo_bytes / (ms_dec * 1e-3) / 1e9
    # full scan: per (invocation, config) pair one compare, one select, one min
    pairs = int(np.diff(w.cfg_off)[w.inv_op].sum())
    full_gops = pairs * 3 / (ms_full * 1e-3) / 1e9

    # parity of what was timed (the oracle also gives the CPU baseline): the
    # decisions left by one more replay of the timed multi-step graph
    torch.cuda.synchronize()
    cfg.fill_(-7)
    g_steps.replay()
    torch.cuda.synchronize()
    c_gpu, f_gpu = cfg.cpu().numpy(), flag.cpu().numpy()
    cpu = None
    bit_exact = None
    if not args.no_cpu_baseline:
        import oracle
        P = oracle.Problem(w)
        P.W(mode)
        times = []
        res = None
        while len(times) < 5 and sum(times) < 15.0:
            t = time.perf_counter()
            res = P.decide(mode)
            times.append(time.perf_counter() - t)
        bit_exact = bool(np.array_equal(res[0], c_gpu) and np.array_equal(res[1], f_gpu))
        # the same oracle on every host core this process may use (at most
        # 16 threads: one GPU's share of the host): invocations cut into one
        # contiguous part per thread, each part a single-threaded oracle call
        ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        threads = max(1, min(16, ncpu, int(os.environ.get("OMP_NUM_THREADS", ncpu) or ncpu)))
        times_mt = []
        while len(times_mt) < 5 and sum(times_mt) < 10.0:
            t = time.perf_counter()
            res_mt = P.decide_parallel(mode, threads)
            times_mt.append(time.perf_counter() - t)
        bit_exact = bit_exact and bool(np.array_equal(res_mt[0], c_gpu) and np.array_equal(res_mt[1], f_gpu))
        cpu = {"value": n / statistics.median(times), "unit": "decisions/s", "cores": 1,
               "kind": "oracle",
               "sample": f"all {n} invocations of the same workload, single-threaded oracle "
                         f"decide (Alg. 1 + Eq. 1 scan of every configuration), median of "
                         f"{len(times)} runs",
               "cpu_model": cpu_model(), "nproc": os.cpu_count(), "usable_cpus": ncpu,
               "all_cores": {"value": n / statistics.median(times_mt), "unit": "decisions/s",
                             "cores": threads, "kind": "oracle",
                             "sample": f"the same {n} invocations cut into {threads} parts, one "
                                       f"single-threaded oracle call per host thread, median of "
                                       f"{len(times_mt)} runs"}}

    next1 = None
    if not args.no_next1:
        next1 = bench_next1(args, torch, B, wl, log, w, op, el, slo, mode)
    next2 = None
    if not args.no_next2:
        next2 = bench_next2(args, torch, B, wl, log, w, op, el, slo, mode)
    next3 = None
    if not args.no_next3:
        next3 = bench_next3(args, torch, B, wl, log, w, op, el, slo, mode)
    next4 = None
    if not args.no_next4:
        next4 = bench_next4(args, torch, B, wl, log, L, w, op, el, slo, mode)
    surr = None
    args._surrogate_ctx = None
    if not args.no_surrogate:
        surr = bench_surrogate(args, torch, B, wl, log)
    serve = None
    if not args.no_serve:
        serve = bench_serving(args, torch, B, wl, log, args._surrogate_ctx)

    out = {
        "metric": METRIC,
        "value": n / (ms_step * 1e-3),
        "unit": "decisions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": ("c2 plain scaled: 256 layered DAGs of 10-40 ops, "
                                "64-512 configs/op (4 hw x batch x 4 memory sizes), "
                                "1M invocations, SLO 0.1-10 s") if args.workload == "c2" else
                               ("c3 batched uneven: 4,096 layered DAGs of 3-200 ops, "
                                "16-2048 configs/op, 4M invocations, SLO 0.1-10 s"),
                   "n_pipelines": w.n_pipelines, "n_ops": w.n_ops, "n_cfg": w.n_cfg,
                   "n_inv": n, "n_hw": w.n_hw, "slack_mode": args.mode,
                   "scan": "indexed", "step": "relax + records + decide",
                   "steps_per_graph": spg,
                   "pipelined": ("relaxation of step k+1 overlaps the decisions of step k "
                                 "(two streams, double-buffered records)") if args.pipeline else False,
                   "decide_schedule": B.SCHEDULE_NAMES[tuned[0]]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.workload, schedule_kernel(tuned[0])),
                     "kernel": schedule_kernel(tuned[0]), "kernel_ms": ms_dec,
                     "algo_bytes": algo_bytes, "copy_gbs": copy_gbs,
                     "frac_of_copy": achieved / copy_gbs},
        "cpu_baseline": cpu,
        "bit_exact": bit_exact,
        "ms_per_step_device": ms_step_dev,
        "relax_ms": ms_relax,
        "full_scan": {"kernels": "bucket by op + scan_classes_kernel (one wavefront per op: lanes = "
                                 "invocations or lanes = configurations, by the autotuned crossover)",
                      "crossover": list(full_cross), "ms": ms_full,
                      "decisions_per_s": n / (ms_full * 1e-3), "pairs": pairs,
                      "roofline": {"bound": "alu", "achieved": full_gops,
                                   "peak": VALU_PEAK_GOPS, "unit": "Gop/s",
                                   "frac": full_gops / VALU_PEAK_GOPS}},
        "wave_scan": {"kernel": "decide_wave_kernel", "ms": ms_wave,
                      "decisions_per_s": n / (ms_wave * 1e-3)},
        "frontier_entries": st["frontier_entries"],
        "next1": next1,
        "next2": next2,
        "next3": next3,
        "next4": next4,
        "surrogate": surr,
        "serving": serve,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
