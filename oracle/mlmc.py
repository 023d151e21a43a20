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
