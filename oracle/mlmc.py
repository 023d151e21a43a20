"""Multilevel Monte Carlo estimator of the oracle (Section 4.1).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* Level statistics are plain two-pass sample means and variances in double
  precision over the per-sample values the oracle returns.
* Sample numbers follow eqs. Nopt1/Noptj: with S = sum_j sqrt(V_j C_j),
  N_j = (2/tol^2) sqrt(V_j / C_j) S, rounded up.
* The iteration enforces the statistical constraint of Section 4.1,
  sum_j V_j / N_j <= tol^2 / 2 (the bias constraint is not part of it: the
  finest level L is fixed by the caller).
* Cost model: C_0 = n_0 and C_{l,l-1} = n_l + n_{l-1} (particle steps per
  sample; the paper's C_{l_j,l_{j-1}} = C_{l_j} + C_{l_{j-1}} with the cost of
  one realisation counted in time steps).
"""
import math

import numpy as np

from . import simulate
from .levels import extrapolate, heuristic, warmup_depth


def level_steps(prob, level):
    return int(round(prob["T"] / prob["dt0"])) * int(prob["M"]) ** level


def level_cost(prob, level):
    n = level_steps(prob, level)
    return n if level == 0 else n + level_steps(prob, level - 1)


QOI_X = 2   # Q = x(T), the position itself (the paper's Section 5); else Q = x(T)^2


def stats_of(xf, xc, level, qoi=0):
    """Two-pass statistics of dQ = Q_f - Q_c (dQ = Q_f at level 0), of Q_f,
    Q_c and of their co-moment; Q = x^2, or Q = x with qoi = QOI_X."""
    if qoi == QOI_X:
        qf = np.array(xf, dtype=np.float64)
        qc = np.array(xc, dtype=np.float64) if level > 0 else np.zeros_like(qf)
    else:
        qf = xf * xf
        qc = xc * xc if level > 0 else np.zeros_like(xf)
    dq = qf - qc
    n = dq.size
    out = dict(n=n)
    for name, a in (("dq", dq), ("qf", qf), ("qc", qc)):
        m = float(np.mean(a)) if n else 0.0
        out["mean_" + name] = m
        out["m2_" + name] = float(np.sum((a - m) ** 2)) if n else 0.0
    out["c_fc"] = float(np.sum((qf - out["mean_qf"]) * (qc - out["mean_qc"]))) if n else 0.0
    return out


def sample_variance(st, key="dq"):
    return st["m2_" + key] / (st["n"] - 1) if st["n"] > 1 else 0.0


def optimal_samples(V, C, tol):
    """Eqs. Nopt1/Noptj: N_j = ceil((2/tol^2) sqrt(V_j/C_j) sum_i sqrt(V_i C_i))."""
    S = 0.0
    for v, c in zip(V, C):
        S += math.sqrt(v * c)
    out = []
    for v, c in zip(V, C):
        out.append(int(math.ceil(2.0 / (tol * tol) * math.sqrt(v / c) * S)))
    return out


def estimate_fixed(prob, N, threads=None):
    """MLMC estimate (eq. mlmc-compact) with N[l] samples [0, N[l]) at level l;
    returns (estimate, per-level stats)."""
    est = 0.0
    levels = []
    for l, n in enumerate(N):
        r = simulate(prob, l, 0, int(n), threads=threads)
        st = stats_of(r["xf"], r["xc"], l, prob.get("qoi", 0))
        st["coll_f"] = int(r["cf"].astype(np.uint64).sum())
        st["coll_c"] = int(r["cc"].astype(np.uint64).sum())
        levels.append(st)
        est += st["mean_dq"]
    return est, levels


def estimate(prob, tol, L, n_warmup=1000, max_iter=8, threads=None):
    """The MLMC loop: warm-up of n_warmup samples per level, then the optimal
    sample numbers with sample variances, topped up until the statistical
    constraint holds.  Samples at level l are the indices [0, N_l)."""
    C = [level_cost(prob, l) for l in range(L + 1)]
    done = [0] * (L + 1)
    xs = [(np.zeros(0), np.zeros(0)) for _ in range(L + 1)]

    def run(l, upto):
        if upto <= done[l]:
            return
        r = simulate(prob, l, done[l], upto - done[l], threads=threads)
        xs[l] = (np.concatenate([xs[l][0], r["xf"]]), np.concatenate([xs[l][1], r["xc"]]))
        done[l] = upto

    for l in range(L + 1):
        run(l, n_warmup)
    for _ in range(max_iter):
        st = [stats_of(xs[l][0], xs[l][1], l, prob.get("qoi", 0)) for l in range(L + 1)]
        V = [sample_variance(s) for s in st]
        N = optimal_samples(V, C, tol)
        for l in range(L + 1):
            run(l, max(N[l], done[l]))
        st = [stats_of(xs[l][0], xs[l][1], l, prob.get("qoi", 0)) for l in range(L + 1)]
        V = [sample_variance(s) for s in st]
        if sum(v / d for v, d in zip(V, done)) <= 0.5 * tol * tol:
            break
    st = [stats_of(xs[l][0], xs[l][1], l, prob.get("qoi", 0)) for l in range(L + 1)]
    return dict(estimate=sum(s["mean_dq"] for s in st), N=list(done), levels=st,
                var_estimator=sum(sample_variance(s) / d for s, d in zip(st, done)))


def estimate_sequence(prob, tol0, R, L, n_warmup=1000, max_iter=10, threads=None):
    """The epsilon-adaptive on-line phase of Section 5.3: the loop of
    ``estimate`` run through the tolerances tol_r = tol0 / sqrt(2^r),
    r = 0..R.  One warm-up; each stage then computes the optimal sample
    numbers at tol_r from all samples so far, tops up, and checks the
    statistical constraint at tol_r (at most max_iter times).  Samples are
    never discarded, so stage r goes on from stage r - 1.  Returns one result
    per stage (the state when the stage ended)."""
    C = [level_cost(prob, l) for l in range(L + 1)]
    done = [0] * (L + 1)
    xs = [(np.zeros(0), np.zeros(0)) for _ in range(L + 1)]

    def run(l, upto):
        if upto <= done[l]:
            return
        r = simulate(prob, l, done[l], upto - done[l], threads=threads)
        xs[l] = (np.concatenate([xs[l][0], r["xf"]]), np.concatenate([xs[l][1], r["xc"]]))
        done[l] = upto

    def state(tol):
        st = [stats_of(xs[l][0], xs[l][1], l, prob.get("qoi", 0)) for l in range(L + 1)]
        var = sum(sample_variance(s) / d for s, d in zip(st, done))
        return dict(estimate=sum(s["mean_dq"] for s in st), N=list(done), levels=st,
                    var_estimator=var, converged=var <= 0.5 * tol * tol, tol=tol)

    for l in range(L + 1):
        run(l, n_warmup)
    out = []
    for r in range(R + 1):
        tol = tol0 / math.sqrt(2.0 ** r)
        for _ in range(max_iter):
            V = [sample_variance(s) for s in state(tol)["levels"]]
            N = optimal_samples(V, C, tol)
            for l in range(L + 1):
                run(l, max(N[l], done[l]))
            if state(tol)["converged"]:
                break
        out.append(state(tol))
    return out


def pair_cost(prob, level, coarse):
    """Cost of one sample of the pair (level, coarse) (coarse < 0: one path).
    Splitting scheme: the paths' time steps.  KD scheme: the expected KD
    steps of the paths, a KD step running from a grid point to the end of the
    grid step that holds the next collision, so a path of n steps of size dt
    at collision rate R takes n (1 - exp(-R dt)) of them on average (R = b in
    a Section 5 background, 1/eps^2 in the diffusive scaling); rounded up,
    at least 1."""
    def steps(l):
        return int(round(prob["T"] / prob["dt0"])) * int(prob["M"]) ** l

    if int(prob.get("scheme", 0)) != 1:
        return steps(level) + (steps(coarse) if coarse >= 0 else 0)

    def kd(l):
        dt = prob["dt0"] / math.pow(prob["M"], l)
        if int(prob.get("background", 0)) != 0:
            R = float(prob["bg_b"])
        else:
            R = 1.0 / (prob["eps"] * prob["eps"])
        return steps(l) * -math.expm1(-R * dt)

    c = kd(level) + (kd(coarse) if coarse >= 0 else 0.0)
    return max(1, int(math.ceil(c)))


def bias_estimate(mean_diff, M, level, coarse):
    """|E[Q_L - Q]| from the finest term of the set, E[Q_L - Q_c] with c the
    level below L: if the weak error is c1 dt_l (first order in dt), then
    E[Q_L - Q_c] = c1 dt_L (1 - M^(L-c)), so the bias c1 dt_L is
    |E[Q_L - Q_c]| / (M^(L-c) - 1)."""
    return abs(mean_diff) / (math.pow(M, level - coarse) - 1.0)


def estimate_adaptive(prob, tol, n_warmup=100, max_iter=10, L_max=None, select="tau",
                      threads=None):
    """The experiment of Section 5.3 with the level-adaptive finest level of
    Sections 4.1 and 5.2.

    Off-line part (select="tau"): n_warmup samples of the adjacent pairs of
    levels 0..tau only (``levels.warmup_depth``); V_l and V_{l,l-1} measured
    there and extrapolated beyond tau (``levels.extrapolate``); the level set
    of the heuristic (``levels.heuristic``).  select="all": every level
    0..L.  An item of the set whose pair is not a warm-up pair (a first level
    above 0 is a single path) starts with n_warmup samples of its own; a
    warm-up pair that stays in the set keeps its samples.

    On-line part: eqs. Nopt1/Noptj with the sample variances and the costs of
    ``pair_cost``, topped up until sum_j V_j/N_j <= tol^2/2 (at most max_iter
    times).  Then the bias constraint |E[Q_L - Q]| <= tol/sqrt(2): the bias is
    estimated from the finest term, E[Q_L - Q_c] / (M^(L-c) - 1) (first-order
    weak convergence in dt), and while it is above tol/sqrt(2) and L < L_max,
    L grows by one: the set is selected again for the new L (select="tau":
    from the same warm-up profile; "all": the new adjacent pair is added),
    kept items keep their samples, and the on-line loop goes on.

    Each level has one slot of samples [0, N_l) for its current pair; a
    level whose pair changes starts over.  Returns the estimate, N, the
    levels, tau, the bias estimate and the number of levels added."""
    M = int(prob["M"])
    prob = dict(prob)
    L = int(prob["L"])
    qoi = prob.get("qoi", 0)
    slots = {}   # level -> dict(coarse, xf, xc)
    active = {}  # level of the set -> coarse level (-1: single path / level 0)
    iterations = 0

    def run(l, upto):
        s = slots[l]
        n = s["xf"].size
        if upto <= n:
            return
        c = s["coarse"]
        if l == 0:
            r = simulate(prob, 0, n, upto - n, threads=threads)
        elif c < 0:
            r = simulate(prob, l, n, upto - n, single=True, threads=threads)
        else:
            r = simulate(prob, l, n, upto - n, threads=threads, coarse_level=c)
        s["xf"] = np.concatenate([s["xf"], r["xf"]])
        s["xc"] = np.concatenate([s["xc"], r["xc"]])

    def stats(l):
        s = slots[l]
        return stats_of(s["xf"], s["xc"], 0 if s["coarse"] < 0 else l, qoi)

    def use(l, c):
        s = slots.get(l)
        if s is None or s["coarse"] != c or s["xf"].size == 0:
            slots[l] = dict(coarse=c, xf=np.zeros(0), xc=np.zeros(0))
            run(l, n_warmup)
        active[l] = c

    tau = warmup_depth(prob) if select == "tau" else L
    for l in range(tau + 1):
        use(l, l - 1)
    prof_V, prof_Vd = [], []
    for l in range(tau + 1):
        st = stats(l)
        prof_V.append(sample_variance(st, "dq" if l == 0 else "qf"))
        prof_Vd.append(sample_variance(st))

    def choose():
        if select == "tau":
            V, Vd = extrapolate(prof_V, prof_Vd, tau, M, L)
            chosen = heuristic(V, Vd)
        else:
            chosen = list(range(L + 1))
        active.clear()
        prev = -1
        for l in chosen:
            use(l, prev)
            prev = l

    choose()

    def variance_sum():
        return sum(sample_variance(stats(l)) / slots[l]["xf"].size for l in active)

    def bias():
        c = active[L]
        if c < 0:
            return math.nan
        return bias_estimate(stats(L)["mean_dq"], M, L, c)

    added = 0
    stage_iter = 0
    targets_first = True
    while True:
        if not targets_first:
            met = variance_sum() <= 0.5 * tol * tol
            if met or stage_iter >= max_iter:
                if met and L_max is not None and L < L_max and bias() > tol / math.sqrt(2.0):
                    L += 1
                    prob["L"] = L
                    added += 1
                    choose()
                    stage_iter = 0
                    continue
                break
        lv = sorted(active)
        V = [sample_variance(stats(l)) for l in lv]
        C = [pair_cost(prob, l, active[l]) for l in lv]
        N = optimal_samples(V, C, tol)
        for l, n in zip(lv, N):
            run(l, max(n, slots[l]["xf"].size))
        iterations += 1
        stage_iter += 1
        targets_first = False
    lv = sorted(active)
    sts = [stats(l) for l in lv]
    return dict(estimate=sum(s["mean_dq"] for s in sts), levels=lv,
                coarse=[active[l] for l in lv], N=[slots[l]["xf"].size for l in lv],
                stats=sts, var_estimator=variance_sum(), tau=tau, L=L, bias=bias(),
                added=added, converged=variance_sum() <= 0.5 * tol * tol,
                iterations=iterations)
