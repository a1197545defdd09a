"""Brute force for Alg. 1 and Eq. 1, used to pin the oracle.

Independent of the oracle's method: it enumerates every source-to-sink path
of the DAG explicitly (the Pipeline-Decomposer's set of sequential paths,
Sec. 3.2), evaluates the remaining path latency of each suffix directly, takes
the minimum slack over the paths that contain the op (Alg. 1), and compares
configurations with exact rationals (Eq. 1).  Pure Python integers and
fractions.Fraction; only for tiny inputs.
"""
from fractions import Fraction

Q_ONE = 65536
INT32_MAX = 2**31 - 1


def successors(succ_off, succ_ids, succ_q16):
    n = len(succ_off) - 1
    succ = [[] for _ in range(n)]
    q = {}
    for v in range(n):
        for e in range(int(succ_off[v]), int(succ_off[v + 1])):
            w = int(succ_ids[e])
            succ[v].append(w)
            q[(v, w)] = Q_ONE if succ_q16 is None else int(succ_q16[e])
    return succ, q


def all_paths(succ):
    """Every sequence from an op with no predecessor to an op with no
    successor."""
    n = len(succ)
    has_pred = [False] * n
    for v in range(n):
        for w in succ[v]:
            has_pred[w] = True
    out = []

    def walk(v, prefix):
        prefix = prefix + [v]
        if not succ[v]:
            out.append(prefix)
            return
        for w in succ[v]:
            walk(w, prefix)

    for s in range(n):
        if not has_pred[s]:
            walk(s, [])
    return out


def path_latency(suffix, ref, q, prob):
    """Remaining reference latency along suffix (op first).  Plain mode:
    the sum.  Probability mode: tail first, each step adds the op's reference
    latency to the floor of the branch-discounted rest."""
    if not prob:
        return sum(int(ref[u]) for u in suffix)
    val = int(ref[suffix[-1]])
    for j in range(len(suffix) - 2, -1, -1):
        u = suffix[j]
        val = int(ref[u]) + (q[(u, suffix[j + 1])] * val) // Q_ONE
    return val


def remaining(slo, elapsed, Q):
    r = int(slo) - int(elapsed) - int(Q)
    return max(0, min(INT32_MAX, r))


def target(v, R, paths, ref, q, prob):
    """min over paths containing v of floor(ref[v] * R / pLat(v, path))."""
    if R == 0:
        return 0
    best = None
    for P in paths:
        if v not in P:
            continue
        pl = path_latency(P[P.index(v):], ref, q, prob)
        s = (int(ref[v]) * R) // pl
        best = s if best is None else min(best, s)
    return best


def select(v, tgt, cfg_off, hw, batch, lat, cost):
    """Eq. 1 with the fastest-configuration fallback.  Returns (local k, flag)."""
    a, b = int(cfg_off[v]), int(cfg_off[v + 1])
    xs = range(a, b)
    feas = [x for x in xs if int(lat[x]) < int(tgt[int(hw[x])])]
    if feas:
        x = min(feas, key=lambda x: (Fraction(int(cost[x]), int(batch[x])), x))
        return x - a, 1
    x = min(xs, key=lambda x: (int(lat[x]), x))
    return x - a, 0


def reference_cfg(v, cfg_off, hw, batch, res):
    a, b = int(cfg_off[v]), int(cfg_off[v + 1])
    cands = [x for x in range(a, b) if int(hw[x]) == 0 and int(batch[x]) == 1]
    if not cands:
        return None
    return min(cands, key=lambda x: (int(res[x]), x)) - a


def decide_all(w, prob, Q=None):
    """Full brute-force decision for every invocation of a workload."""
    succ, q = successors(w.succ_off, w.succ_ids, w.succ_q16)
    paths = all_paths(succ)
    n_ops = len(w.cfg_off) - 1
    ref = []
    for v in range(n_ops):
        k = reference_cfg(v, w.cfg_off, w.hw, w.batch, w.res)
        ref.append(int(w.lat[int(w.cfg_off[v]) + k]))
    tg, cf, fl = [], [], []
    for i in range(len(w.inv_op)):
        v = int(w.inv_op[i])
        if not (0 <= v < n_ops) or w.elapsed[i] < 0 or w.slo[i] < 0:
            tg.append([-1] * w.n_hw)
            cf.append(-1)
            fl.append(0)
            continue
        t = [target(v, remaining(w.slo[i], w.elapsed[i], 0 if Q is None else Q[h]),
                    paths, ref, q, prob) for h in range(w.n_hw)]
        k, f = select(v, t, w.cfg_off, w.hw, w.batch, w.lat, w.cost)
        tg.append(t)
        cf.append(k)
        fl.append(f)
    return tg, cf, fl
