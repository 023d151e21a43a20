"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each ``pin_*`` function raises AssertionError on failure.  They are run by
``tests/test_oracle_pins.py`` against the real oracle, and by
``tests/test_oracle_mutants.py`` against deliberately broken builds of it, to
show that a plausible slip anywhere in the oracle fails at least one pin.

Nothing here recomputes the oracle's formulas: values come from the
published Philox answers, closed-form moments of the scheme, its diffusive
and kinetic limits, exact enumeration, and distribution tests.
"""
import math
import os

import numpy as np
from scipy import stats

import oracle as O
from oracle import closed_form as CF
from oracle import mlmc as OM

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

Z_MAX = 4.5          # |z| bound for fixed-seed moment checks
P_MIN = 1e-4         # p-value floor for fixed-seed distribution tests


def maxwell_problem(eps, T=1.0, dt0=0.5, M=2, coupling=1, x0_kind=1, seed=42, stream=0):
    return dict(eps=eps, T=T, dt0=dt0, M=M, x0_kind=x0_kind, x0_a=0.0, x0_b=1.0,
                eq_kind=1, coupling=coupling, seed=seed, stream_id=stream)


def two_point_problem(eps, T, dt0, M=2, coupling=0, seed=42, stream=0):
    return dict(eps=eps, T=T, dt0=dt0, M=M, x0_kind=0, x0_a=0.0, x0_b=0.0,
                eq_kind=0, coupling=coupling, seed=seed, stream_id=stream)


AD_MAX = 6.0         # Anderson-Darling A^2 bound (fully specified law; about p = 1e-3)


def anderson_darling(x, cdf):
    """A^2 of the paper's eq. anderson for a fully specified CDF."""
    x = np.sort(np.asarray(x, dtype=np.float64))
    n = x.size
    F = np.clip(cdf(x), 1e-300, 1.0 - 1e-16)
    i = np.arange(1, n + 1)
    return float(-n - np.sum((2 * i - 1) * (np.log(F) + np.log1p(-F[::-1]))) / n)


def _z(sample, exact):
    return (float(np.mean(sample)) - exact) / (float(np.std(sample)) / math.sqrt(sample.size))


def _thr_p(prob, level):
    c = O.level_consts(prob["eps"], prob["T"], prob["dt0"], prob["M"], level)
    return c["thr"] / 2.0 ** 32


# --------------------------------------------------------------------------
def pin_philox_kat():
    """Published Philox4x32-10 known-answer vectors."""
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        out = O.philox4x32_10(v[0:4], v[4:6])
        assert [int(w) for w in out] == v[6:10], (r, [hex(int(w)) for w in out])


def pin_word_layout():
    """The documented random-number layout: the stream of Philox words of
    blocks 0, 1, 2, ... (counter (block, sample, tag, stream)); the initial
    condition takes 2 words (6 for the cosine law), then each fine step the
    decision word and a Box-Muller pair (radius, angle)."""
    for x0_kind, first in ((1, 2), (2, 6)):
        prob = dict(maxwell_problem(0.3, T=1.0, dt0=0.125, stream=77), x0_kind=x0_kind)
        rows, _ = O.trace(prob, 1, 12345)
        n = rows.shape[0]
        blocks = (first + 3 * n + 3) // 4
        w = O.words(42, 77, 1, 12345, 1, blocks).reshape(-1)
        for k in range(n):
            assert rows[k, 1] == w[first + 3 * k]
            assert rows[k, 2] == w[first + 3 * k + 1]
            assert rows[k, 3] == w[first + 3 * k + 2]
            assert rows[k, 4] == first + 3 * k + 3


def pin_uniform():
    """Odd multiples of 2^-24 strictly inside (0,1), symmetric about 1/2."""
    assert O.uniform(0) == 2.0 ** -24
    assert O.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    for w in (0, 1, 511, 512, 0x80000000, 0xDEADBEEF, 0xFFFFFFFF):
        u = O.uniform(w)
        k = u * 2.0 ** 24
        assert 0.0 < u < 1.0 and k == int(k) and int(k) % 2 == 1, (w, u)
        assert O.uniform(w) + O.uniform(0xFFFFFFFF - w) == 1.0


def pin_normals():
    """Kick and velocity normals of a trace are independent N(0,1)."""
    prob = maxwell_problem(1.0, T=1.0, dt0=1.0 / 64)
    xs, gs, u1s = [], [], []
    for smp in range(120):
        rows, _ = O.trace(prob, 0, smp, single=True)
        xs.append(rows[:, 7]); gs.append(rows[:, 8]); u1s.append(rows[:, 5])
    xi = np.concatenate(xs); g = np.concatenate(gs); u1 = np.concatenate(u1s)
    assert xi.size == 120 * 64
    for a in (xi, g):
        assert stats.kstest(a, "norm").pvalue > P_MIN
    assert abs(np.corrcoef(xi, g)[0, 1]) < 4.5 / math.sqrt(xi.size)
    assert stats.kstest(u1, "uniform").pvalue > P_MIN
    # the radius of a Box-Muller pair is a function of the first word alone
    r2 = xi * xi + g * g
    assert np.allclose(r2, -2.0 * np.log(u1), rtol=1e-12, atol=1e-12)


def pin_second_moment_cfg1():
    """Exact E[x^2] of the scheme, velocities +-1, eps=0.5, T=0.5, dt=0.01."""
    prob = two_point_problem(0.5, 0.5, 0.01)
    r = O.simulate(prob, 0, 0, 100000)
    exact = CF.second_moment(0.5, 0.01, 50, 0.0, p=_thr_p(prob, 0))
    assert abs(exact - 0.5683899408) < 1e-9
    assert abs(_z(r["xf"] ** 2, exact)) < Z_MAX


def pin_second_moment_levels():
    """Exact E[x^2] over eps from the diffusive to the free-streaming regime."""
    for eps in (1e-4, 1e-2, 0.1, 1.0, 10.0):
        for level in (0, 3, 6):
            prob = maxwell_problem(eps, stream=7)
            n = 30000 if level < 6 else 8000
            r = O.simulate(prob, level, 0, n, single=True)
            c = O.level_consts(eps, 1.0, 0.5, 2, level)
            exact = CF.second_moment(eps, c["dt"], c["n_steps"], 1.0, p=c["thr"] / 2.0 ** 32)
            z = _z(r["xf"] ** 2, exact)
            assert abs(z) < Z_MAX, (eps, level, z)


def pin_cosine_initial():
    """x0 with density 1+cos(2 pi x): CDF, mean 1/2, E[x0^2] = 1/3 + 1/(2 pi^2)."""
    for u in (1e-6, 0.1, 0.25, 0.5, 0.7, 0.999):
        x = O.cosine_icdf(u)
        assert abs(x + math.sin(2 * math.pi * x) / (2 * math.pi) - u) < 1e-12
    prob = dict(eps=1e-3, T=1.0, dt0=0.5, M=2, x0_kind=2, eq_kind=1, coupling=1, seed=42,
                stream_id=3)
    # at eps = 1e-3 the path adds N(0, ~2T) independent of x0
    r = O.simulate(prob, 0, 0, 40000, single=True)
    exact = CF.second_moment(1e-3, 0.5, 2, CF.x0_second_moment(2), p=_thr_p(prob, 0))
    assert abs(_z(r["xf"] ** 2, exact)) < Z_MAX
    assert abs(_z(r["xf"], 0.5)) < Z_MAX
    x0 = np.array([O.cosine_icdf(u) for u in (np.arange(4000) + 0.5) / 4000])
    F = lambda x: x + np.sin(2 * np.pi * x) / (2 * np.pi)
    assert np.max(np.abs(F(x0) - (np.arange(4000) + 0.5) / 4000)) < 1e-12


def pin_heat_limit():
    """eps = 0: x_T ~ N(x0, 2T) for any dt, and the coupled paths coincide."""
    for coupling in (0, 1):
        prob = maxwell_problem(0.0, T=1.0, dt0=0.5, coupling=coupling, x0_kind=0)
        r = O.simulate(prob, 4, 0, 20000)
        assert stats.kstest(r["xf"] / math.sqrt(2.0), "norm").pvalue > P_MIN
        assert stats.kstest(r["xc"] / math.sqrt(2.0), "norm").pvalue > P_MIN
        assert np.max(np.abs(r["xf"] - r["xc"])) < 1e-12
        assert np.all(r["cf"] == 32) and np.all(r["cc"] == 16)


def pin_kinetic_limit():
    """dt -> 0: E[x_T^2] tends to the kinetic displacement variance
    (square of the paper's beta weight with R = 1/eps^2)."""
    for eps in (0.3, 1.0):
        lim = CF.kinetic_limit(eps, 0.5, 0.0)
        prev = None
        for k in range(6, 16, 3):
            dt = 0.5 / 2 ** k
            v = CF.second_moment_closed(eps, dt, 2 ** k, 0.0)
            err = abs(v - lim)
            if prev is not None:
                assert err < 0.6 * prev
            prev = err
        assert prev < 1e-3 * lim
    prob = two_point_problem(1.0, 0.5, 0.5 / 512)
    r = O.simulate(prob, 0, 0, 30000)
    exact = CF.second_moment(1.0, 0.5 / 512, 512, 0.0, p=_thr_p(prob, 0))
    assert abs(exact - CF.kinetic_limit(1.0, 0.5, 0.0)) < 1e-3
    assert abs(_z(r["xf"] ** 2, exact)) < Z_MAX


def pin_two_point_bruteforce():
    """Velocities +-1: the exact law of x_n by enumeration of all velocity
    sequences, for the fine path of level 1 (20 steps) and for its coarse
    path against the exact law of level 0 (10 steps)."""
    prob = two_point_problem(0.3, 0.5, 0.05, M=2, coupling=0, stream=11)
    r = O.simulate(prob, 1, 0, 60000)          # fine: dt = 0.025, 20 steps
    c1 = O.level_consts(0.3, 0.5, 0.05, 2, 1)
    cdf_f = lambda x: CF.two_point_mixture_cdf(x, 0.0, 0.3, c1["dt"], c1["n_steps"])
    assert stats.kstest(r["xf"], cdf_f).pvalue > P_MIN
    c0 = O.level_consts(0.3, 0.5, 0.05, 2, 0)
    cdf_c = lambda x: CF.two_point_mixture_cdf(x, 0.0, 0.3, c0["dt"], c0["n_steps"])
    assert stats.kstest(r["xc"], cdf_c).pvalue > P_MIN


def pin_telescoping():
    """The coarse path of level l has the law of level l-1 (eq. telsum):
    its mean matches the exact E[Q_{l-1}], and its distribution matches an
    independent single-level run of level l-1."""
    for coupling in (0, 1):
        for eps in (1e-2, 0.3):
            prob = maxwell_problem(eps, coupling=coupling, stream=5)
            for level in (1, 3):
                r = O.simulate(prob, level, 0, 30000)
                exact_c = CF.level_second_moment(prob, level - 1)
                exact_f = CF.level_second_moment(prob, level)
                assert abs(_z(r["xc"] ** 2, exact_c)) < Z_MAX, (coupling, eps, level)
                assert abs(_z(r["xf"] ** 2, exact_f)) < Z_MAX, (coupling, eps, level)
                ind = O.simulate(prob, level - 1, 0, 30000, single=True)
                assert stats.ks_2samp(r["xc"], ind["xf"]).pvalue > P_MIN
                cind = ind["cf"].astype(np.float64)
                assert abs(r["cc"].mean() - cind.mean()) < Z_MAX * math.sqrt(
                    (r["cc"].var() + cind.var()) / 30000) + 1e-12


def _coarse_records(prob, level, nsamp):
    kicks, hits, vnew = [], [], []
    for smp in range(nsamp):
        rows, _ = O.trace(prob, level, smp)
        blk = rows[prob["M"] - 1::prob["M"]]
        kicks.append(blk[:, 12]); hits.append(blk[:, 13])
        h = blk[:, 13] > 0
        vnew.append(blk[h, 15])
    return np.concatenate(kicks), np.concatenate(hits), np.concatenate(vnew)


def pin_coupling_laws():
    """Coarse random numbers have the laws the coarse level needs (the
    Anderson-Darling methodology of the paper's consistency study): kick
    N(0,1), collision Bernoulli(p_c), new velocity from the equilibrium, and
    no lag-1 or kick/collision correlation."""
    for coupling, M, eps in ((1, 2, 0.05), (1, 4, 0.05), (0, 2, 0.05), (1, 2, 0.01)):
        prob = maxwell_problem(eps, T=1.0, dt0=0.25, M=M, coupling=coupling, stream=9)
        level = 2
        kick, hit, vnew = _coarse_records(prob, level, 400)
        assert anderson_darling(kick, stats.norm.cdf) < AD_MAX, (coupling, M, eps)
        assert stats.kstest(kick, "norm").pvalue > P_MIN, (coupling, M, eps)
        assert stats.kstest(vnew, "norm").pvalue > P_MIN, (coupling, M, eps)
        pc = _thr_p(prob, level - 1)
        nh = hit.sum()
        assert stats.binomtest(int(nh), hit.size, pc).pvalue > P_MIN, (coupling, M, eps, nh / hit.size, pc)
        k2 = kick.reshape(400, -1)
        lag = np.corrcoef(k2[:, :-1].ravel(), k2[:, 1:].ravel())[0, 1]
        assert abs(lag) < 4.5 / math.sqrt(k2[:, 1:].size)
        if 0 < nh < hit.size:
            assert abs(np.corrcoef(kick, hit)[0, 1]) < 4.5 / math.sqrt(kick.size)


def pin_coarse_threshold():
    """P(coarse collision) = 1 - (1 - thr_c2/2^32)^M (smallest of M uniform
    words below thr_c2) equals the coarse level's probability thr_c / 2^32
    to within the 2^-32 quantum, and thr_c2 <= thr_f (a coarse collision
    implies a fine one)."""
    for eps in (0.0, 1e-4, 1e-2, 0.1, 1.0, 10.0):
        for M in (2, 3, 4, 8):
            for level in (1, 2, 5, 9):
                cf = O.level_consts(eps, 1.0, 0.5, M, level)
                cc = O.level_consts(eps, 1.0, 0.5, M, level - 1)
                t2 = O.coarse_threshold(cf["thr"], cc["thr"], M)
                assert 0 <= t2 <= cf["thr"]
                got = -math.expm1(M * math.log1p(-t2 / 2.0 ** 32)) if t2 < 2 ** 32 else 1.0
                want = cc["thr"] / 2.0 ** 32
                assert abs(got - want) <= M * 2.0 ** -32 + 1e-15, (eps, M, level, got, want)


def pin_symmetry():
    """E[x_T] = E[x_0] and odd moments vanish for symmetric x0 and equilibrium."""
    prob = maxwell_problem(0.2, stream=13)
    r = O.simulate(prob, 2, 0, 40000)
    assert abs(_z(r["xf"], 0.0)) < Z_MAX and abs(_z(r["xc"], 0.0)) < Z_MAX
    assert abs(_z(r["xf"] ** 3, 0.0)) < Z_MAX


def pin_optimal_samples():
    """Eqs. Nopt1/Noptj: the continuous optimum meets the statistical
    constraint with equality, its cost equals eq. total_cost, and moving
    along the constraint surface only raises the cost."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        J = int(rng.integers(1, 10))
        V = 10.0 ** rng.uniform(-8, 1, J)
        C = rng.integers(1, 2000, J).astype(float)
        tol = 10.0 ** rng.uniform(-3.5, -1)
        N = np.array(OM.optimal_samples(V, C, tol), dtype=float)
        S = np.sum(np.sqrt(V * C))
        Ncont = 2.0 / tol ** 2 * np.sqrt(V / C) * S
        assert np.all(N >= Ncont) and np.all(N < Ncont + 1.0 + 1e-9 * Ncont)
        assert abs(np.sum(V / Ncont) - tol ** 2 / 2) < 1e-9 * tol ** 2
        assert abs(np.sum(Ncont * C) - 2.0 / tol ** 2 * S ** 2) < 1e-9 * np.sum(Ncont * C)
        if J > 1:
            for _ in range(5):
                d = rng.normal(size=J) * 0.05
                Np = Ncont * np.exp(d)
                Np *= np.sum(V / Np) / (tol ** 2 / 2)   # back onto the constraint
                assert np.sum(Np * C) >= np.sum(Ncont * C) * (1 - 1e-12)


def pin_mlmc_unbiased():
    """The MLMC estimate targets E[Q_L] (eq. unbiased)."""
    prob = maxwell_problem(0.05, coupling=1, stream=17)
    L = 4
    res = OM.estimate(prob, 2e-2, L, n_warmup=500)
    exact = CF.level_second_moment(prob, L)
    assert abs(res["estimate"] - exact) < Z_MAX * math.sqrt(res["var_estimator"])
    assert res["var_estimator"] <= 0.5 * 2e-2 ** 2 * 1.0000001


ALL_PINS = [pin_philox_kat, pin_word_layout, pin_uniform, pin_normals, pin_second_moment_cfg1,
            pin_second_moment_levels, pin_cosine_initial, pin_heat_limit, pin_kinetic_limit,
            pin_two_point_bruteforce, pin_telescoping, pin_coupling_laws, pin_coarse_threshold,
            pin_symmetry, pin_optimal_samples, pin_mlmc_unbiased]


def run_all(stop_at_first=False):
    """Runs every pin, returns the names of the failing ones."""
    failed = []
    for f in ALL_PINS:
        try:
            f()
        except Exception as e:       # a mutant may also crash or produce NaN
            failed.append("%s: %s" % (f.__name__, type(e).__name__))
            if stop_at_first:
                break
    return failed


if __name__ == "__main__":
    import json
    import sys
    print(json.dumps(run_all(stop_at_first="--first" in sys.argv)))
