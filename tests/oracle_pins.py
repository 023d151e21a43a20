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


AD_CRIT_1PCT = 3.857   # A^2 above which a fully specified law is rejected at the 1 % level


def ad_pvalue(a2):
    """p-value of an Anderson-Darling distance A^2 for a fully specified law:
    1 - ADinf(A^2), with ADinf the asymptotic distribution function in the
    approximation of G. Marsaglia and J. Marsaglia, "Evaluating the
    Anderson-Darling distribution", J. Stat. Softw. 9(2), 2004."""
    z = float(a2)
    if z <= 0.0:
        return 1.0
    if z < 2.0:
        cdf = math.exp(-1.2337141 / z) / math.sqrt(z) * (
            2.00012 + (0.247105 - (0.0649821 - (0.0347962 - (0.011672 - 0.00168691 * z) * z)
                                   * z) * z) * z)
    else:
        cdf = math.exp(-math.exp(1.0776 - (2.30695 - (0.43424 - (0.082433 - (0.008056 -
                                                                       0.0003146 * z) * z)
                                                      * z) * z) * z))
    return max(0.0, 1.0 - cdf)


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


def pin_kick_block_identity():
    """The coarse kick is the fine block's displacement that no velocity the
    coarse path keeps accounts for, normalised by its standard deviation
    (eq. chi-update with the fixed-step weights).  Deterministic identity on
    every coarse block of a trace, from the trace's positions, velocities and
    collision flags alone (no bookkeeping variable of the oracle):
      D = x_f(block end) - x_f(previous block end) = sum_m (h_f v_m + s_f xi_m),
    with v_m the velocity the fine move m is made with.
      kick sum:   kick * s_f sqrt(M) = D - h_f sum_m v_m;
      aggregated: the velocity carried into the block acts u_0 moves, the
        draw nu_j of an in-block collision at step k_j acts n_j moves (up to
        the next in-block collision or the block end); the coarse path keeps
        the carried velocity and, if it collides, the last draw, so
        kick * sqrt(M s_f^2 + h_f^2 sum_{j in A} n_j^2)
            = D - h_f u_0 v_pre - [coarse hit] h_f n_last nu_last,
        A = the draws the coarse path does not keep."""
    cases = [(1, 2, 0.05, 3), (1, 3, 0.3, 2), (1, 4, 0.1, 2), (1, 2, 1.0, 3),
             (0, 2, 0.05, 3), (0, 3, 0.3, 2)]
    checked = 0
    for k, (coupling, M, eps, level) in enumerate(cases):
        prob = maxwell_problem(eps, T=1.5 if M == 3 else 1.0, dt0=0.25 if M != 3 else 0.5,
                               M=M, coupling=coupling, stream=700 + k)
        c = O.level_consts(eps, prob["T"], prob["dt0"], M, level)
        h, sd = c["h"], c["s"]
        for smp in range(40):
            rows, _ = O.trace(prob, level, smp)
            for b in range(1, rows.shape[0] // M):
                prev = rows[b * M - 1]
                blk = rows[b * M:(b + 1) * M]
                D = blk[-1, 10] - prev[10]
                vpre_m = np.concatenate(([prev[11]], blk[:-1, 11]))   # velocity of each move
                kick, chit = blk[-1, 12], blk[-1, 13] > 0
                scale = 1e-11 * (1.0 + abs(blk[-1, 10]) + abs(prev[10]))
                if coupling == 0:
                    lhs = kick * sd * math.sqrt(M)
                    rhs = D - h * np.sum(vpre_m)
                else:
                    hits = np.nonzero(blk[:, 9] > 0)[0]
                    u0 = (hits[0] + 1) if hits.size else M
                    ends = np.append(hits[1:], M - 1)
                    n = (ends - hits).astype(np.float64)       # moves made with draw j
                    nu = blk[hits, 11]                          # draw j = velocity after its hit
                    assert np.array_equal(nu, blk[hits, 8])     # the Maxwellian draw g
                    keep_last = chit and hits.size > 0
                    A = slice(0, hits.size - 1) if keep_last else slice(0, hits.size)
                    rhs = D - h * u0 * prev[11]
                    if keep_last:
                        rhs -= h * n[-1] * nu[-1]
                    lhs = kick * math.sqrt(M * sd * sd + h * h * np.sum(n[A] ** 2))
                assert abs(lhs - rhs) <= scale, (coupling, M, eps, smp, b, lhs, rhs)
                checked += 1
    assert checked > 2000


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


# --------------------------------------------------------------------------
# Kinetic-diffusion (KD) scheme
# --------------------------------------------------------------------------
def kd_problem(eps, T=1.0, dt0=0.5, M=2, x0_kind=0, seed=42, stream=0):
    return dict(eps=eps, T=T, dt0=dt0, M=M, x0_kind=x0_kind, x0_a=0.0, x0_b=1.0,
                eq_kind=1, coupling=1, seed=seed, stream_id=stream, scheme=O.SCHEME_KD)


def pin_kd_second_moment_exact():
    """The KD step keeps the mean and variance of the kinetic motion given the
    next velocity, so in a homogeneous background E[x(T)^2] is the kinetic
    value 2 (T - eps^2 (1 - e^{-T/eps^2})) (x0 = 0) at every time step, for
    single paths and for both paths of a pair."""
    cases = [(1.0, 0.5, 0, False), (0.3, 0.5, 0, False), (0.3, 0.25, 2, False),
             (0.1, 0.5, 1, False), (0.3, 0.5, 2, True), (2.0, 0.5, 1, False)]
    for k, (eps, dt0, level, single) in enumerate(cases):
        prob = kd_problem(eps, dt0=dt0, stream=300 + k)
        r = O.simulate(prob, level, 0, 100000, single=single)
        exact = CF.kinetic_limit(eps, prob["T"], 0.0)
        assert abs(_z(r["xf"] ** 2, exact)) < Z_MAX, (eps, dt0, level, "fine")
        if level >= 1 and not single:
            assert abs(_z(r["xc"] ** 2, exact)) < Z_MAX, (eps, dt0, level, "coarse")
            assert abs(_z(r["xf"] ** 2 - r["xc"] ** 2, 0.0)) < Z_MAX


def _velocity_jump(theta, R, mu, sigma, n, rng):
    """Exact velocity-jump motion over [0, theta] right after a collision:
    velocities N(mu, sigma^2), redrawn at rate R.  Returns (dx, v_end)."""
    v = mu + sigma * rng.standard_normal(n)
    t = np.zeros(n)
    dx = np.zeros(n)
    live = np.ones(n, dtype=bool)
    while live.any():
        idx = np.nonzero(live)[0]
        tau = rng.exponential(1.0 / R, size=idx.size)
        end = t[idx] + tau >= theta
        stop = idx[end]
        dx[stop] += v[stop] * (theta - t[stop])
        live[stop] = False
        go = idx[~end]
        dx[go] += v[go] * tau[~end]
        t[go] += tau[~end]
        v[go] = mu + sigma * rng.standard_normal(go.size)
    return dx, v


def pin_kd_diffusive_phase_bruteforce():
    """eqs. advection and diffusion are the conditional mean and variance of
    the kinetic displacement over theta given the final velocity: checked
    against a brute-force velocity-jump simulation (moments weighted by 1
    and by the velocity)."""
    rng = np.random.default_rng(7)
    R, mu, sigma = 2.0, 0.3, 1.5
    for theta in (0.02, 0.2, 1.0, 2.5):   # y = R theta on both sides of the series switch
        # a(v) is affine and d(v)^2 quadratic in v - mu: read them off the
        # oracle at a few velocities and check that structure
        vs = mu + sigma * np.array([-2.0, 0.0, 1.0, 3.0])
        ad = np.array([O.kd_coeffs(theta, R, mu, sigma, v) for v in vs])
        a0, a1 = ad[1, 0], ad[2, 0] - ad[1, 0]
        D0, D1 = ad[1, 1] ** 2, (ad[2, 1] ** 2 - ad[1, 1] ** 2) / sigma ** 2
        assert np.allclose(ad[:, 0], a0 + a1 * (vs - mu) / sigma, rtol=1e-12, atol=1e-14)
        assert np.allclose(ad[:, 1] ** 2, D0 + D1 * (vs - mu) ** 2, rtol=1e-10, atol=1e-14)
        dx, v = _velocity_jump(theta, R, mu, sigma, 400000, rng)
        w = v - mu
        r = dx - (a0 + a1 * w / sigma)
        s2 = r * r - (D0 + D1 * w * w)
        for sample in (r, r * w, s2, s2 * w * w / sigma ** 2):
            assert abs(_z(sample, 0.0)) < Z_MAX, theta


def _kd_coarse_rows(prob, level, nsamp):
    rows = [O.kd_coarse_numbers(prob, level, s)[0] for s in range(nsamp)]
    return np.concatenate(rows)


def pin_kd_coarse_number_laws():
    """The aggregated coarse numbers have the laws of the coarse path's own
    numbers (Section 3.2): chi~ ~ N(0,1) (eq. chi-update), nu~ ~ N(0,1) (eq.
    nu-update), E~ ~ Exp(1) by memorylessness (eq. epsilon-update), and
    chi~ is uncorrelated with nu~."""
    for k, (eps, level, nsamp) in enumerate(((0.3, 3, 3000), (1.0, 2, 6000), (0.05, 2, 1500))):
        rows = _kd_coarse_rows(kd_problem(eps, stream=320 + k), level, nsamp)
        assert rows.shape[0] > 5000
        assert anderson_darling(rows[:, 0], stats.norm.cdf) < AD_MAX, (eps, "chi")
        assert anderson_darling(rows[:, 1], stats.norm.cdf) < AD_MAX, (eps, "nu")
        assert anderson_darling(rows[:, 2], stats.expon.cdf) < AD_MAX, (eps, "E")
        assert abs(_z(rows[:, 0] * rows[:, 1], 0.0)) < Z_MAX
        assert np.all(rows[:, 3] >= 1)


def pin_kd_coarse_matches_level_below():
    """The coarse path of a level-l pair has the law of the KD path of level
    l-1 (the telescoping requirement): two-sample tests of x and of x^4."""
    for k, (eps, level) in enumerate(((0.3, 2), (1.0, 1), (0.1, 3))):
        pair = O.simulate(kd_problem(eps, x0_kind=1, stream=340 + k), level, 0, 100000)
        below = O.simulate(kd_problem(eps, x0_kind=1, stream=360 + k), level - 1, 0, 100000)
        a, b = pair["xc"], below["xf"]
        assert stats.ks_2samp(a, b).pvalue > P_MIN, (eps, level)
        d = np.mean(a ** 4) - np.mean(b ** 4)
        se = math.sqrt((np.var(a ** 4) + np.var(b ** 4)) / a.size)
        assert abs(d / se) < Z_MAX, (eps, level)


def pin_kd_invariants():
    """Paths without a collision before T stream freely with the shared
    initial velocity, so both paths of such a pair end at the same point;
    coarse collisions are fine collisions; in the diffusive regime every
    time step holds a collision and the two paths stay close (the
    aggregated diffusive number follows the fine diffusive motion)."""
    r = O.simulate(kd_problem(5.0, stream=380), 2, 0, 20000)
    free = r["cf"] == 0
    assert free.sum() > 10000
    assert np.array_equal(r["xf"][free], r["xc"][free])
    assert np.all(r["cc"] <= r["cf"])
    assert not np.array_equal(r["xf"][~free], r["xc"][~free])
    r0 = O.simulate(kd_problem(0.3, stream=381), 0, 0, 1000)
    assert np.all(r0["cc"] == 0) and np.all(r0["xc"] == 0.0)
    prob = kd_problem(1e-3, stream=382)
    r = O.simulate(prob, 3, 0, 20000)
    assert np.all(r["cf"] == 16) and np.all(r["cc"] == 8)
    dq = r["xf"] ** 2 - r["xc"] ** 2
    assert np.var(dq) < 1e-6 * np.var(r["xf"] ** 2)


def pin_kd_nonadjacent_pairs():
    """The coarse path of a KD pair (l, l') with l' < l - 1 has the law of the
    KD path of level l' (two-sample KS and x^4 tests) and the exact second
    moment."""
    for k, (eps, l, lc, M) in enumerate(((0.3, 4, 1, 2), (1.0, 3, 0, 2), (0.1, 2, 0, 3))):
        prob = kd_problem(eps, x0_kind=1, M=M, T=1.5 if M == 3 else 1.0, stream=420 + k)
        pair = O.simulate(prob, l, 0, 100000, coarse_level=lc)
        below = O.simulate(dict(prob, stream_id=440 + k), lc, 0, 100000)
        a, b = pair["xc"], below["xf"]
        assert stats.ks_2samp(a, b).pvalue > P_MIN, (eps, l, lc)
        assert abs(_z(a ** 2, CF.kinetic_limit(eps, prob["T"], 1.0))) < Z_MAX


def _velocity_jump_last_duration(theta, R, n, rng):
    """Time during which the last velocity of a velocity-jump motion over
    [0, theta] (collisions at rate R) acts, for n independent paths."""
    t = np.zeros(n)
    last = np.zeros(n)
    live = np.ones(n, dtype=bool)
    while live.any():
        idx = np.nonzero(live)[0]
        tau = rng.exponential(1.0 / R, size=idx.size)
        end = t[idx] + tau >= theta
        live[idx[end]] = False
        go = idx[~end]
        t[go] += tau[~end]
        last[go] = t[go]
    return theta - last


def pin_kd_aggregation_weights():
    """The weights of eq. chi-update (Section 3.2), phase by phase:
      - zeta_m is the expected time the next velocity acts in diffusive phase
        m: eq. advection (mu = 0) is a_m = sigma nu_{m+1} zeta_m, checked
        against the phase's own a_m, and zeta against a brute-force
        velocity-jump simulation over theta_m;
      - theta'_m = theta_m - zeta_m and tau'_m = tau_m + zeta_{m-1}, so
        alpha_m nu_m = sigma tau_m nu_m + a_{m-1}: the whole displacement
        that nu_m causes (its flight and the previous phase's advection);
      - beta_m^2 is the variance of the unconditioned diffusive displacement
        over theta'_m: brute-force velocity-jump simulation;
      - the coarse number is the normalised weighted sum over its window, the
        window's first phase (the coarse path's own flight) without an alpha
        term, and the next window opens with the flight whose velocity
        number the coarse path takes (eq. nu-update)."""
    rng = np.random.default_rng(11)
    picks = []
    for k, (eps, level, M) in enumerate(((0.3, 3, 2), (0.1, 2, 2), (0.5, 2, 4), (0.3, 2, 3),
                                         (0.3, 1, 2))):
        prob = kd_problem(eps, M=M, T=1.5 if M == 3 else 1.0, stream=720 + k)
        R, sigma = 1.0 / eps ** 2, 1.0 / eps
        dtf = prob["dt0"] / M ** level
        for smp in range(60):
            ph, co, _ = O.kd_phases(prob, level, smp)
            assert ph.shape[0] >= co.shape[0] >= 1
            for m in range(ph.shape[0]):
                r = ph[m]
                sc = 1e-12 * (1.0 + abs(r[12]) + sigma * abs(r[14]) * dtf)
                assert abs(sigma * r[14] * r[5] - r[12]) <= sc, (eps, smp, m)
                assert abs(r[6] - (r[4] - r[5])) <= 1e-15 * (1.0 + r[4])
                c = r[2] + r[3]
                assert abs(r[4] - ((math.floor(c / dtf) + 1.0) * dtf - c)) <= 1e-12 * dtf
                if r[1] == 0:
                    assert ph[m - 1, 0] == r[0]
                    assert abs(r[7] - (r[3] + ph[m - 1, 5])) <= 1e-14 * (1.0 + r[7])
                    lhs = r[8] * r[10]
                    rhs = sigma * r[3] * r[10] + ph[m - 1, 12]
                    assert abs(lhs - rhs) <= 1e-12 * (1.0 + abs(lhs)), (eps, smp, m, lhs, rhs)
                else:
                    assert r[7] == 0.0 and r[8] == 0.0
                    assert m == 0 or ph[m - 1, 0] == r[0] - 1
            for w in range(co.shape[0]):
                sel = ph[ph[:, 0] == w]
                assert sel[0, 1] == 1 and np.all(sel[1:, 1] == 0) and sel.shape[0] == co[w, 3]
                num = np.sum(sel[:, 9] * sel[:, 11]) + np.sum(sel[1:, 8] * sel[1:, 10])
                den = np.sum(sel[:, 9] ** 2) + np.sum(sel[1:, 8] ** 2)
                assert abs(co[w, 0] - num / math.sqrt(den)) <= 1e-12 * (1.0 + abs(co[w, 0]))
                nxt = ph[ph[:, 0] == w + 1]
                if nxt.shape[0]:
                    assert co[w, 1] == nxt[0, 10]
            picks.extend((R, sigma, r[4], r[5], r[6], r[9]) for r in ph)
    picks = np.array(picks)
    # brute force at phases spread over y = R theta (both sides of the series switch)
    y = picks[:, 0] * picks[:, 2]
    for lo, hi in ((0.005, 0.05), (0.1, 0.8), (1.0, 4.0), (5.0, 20.0)):
        cand = np.nonzero((y > lo) & (y < hi))[0]
        assert cand.size > 0, (lo, hi)
        R, sigma, theta, zeta, theta_p, beta = picks[cand[cand.size // 2]]
        last = _velocity_jump_last_duration(theta, R, 200000, rng)
        assert abs(_z(last, zeta)) < Z_MAX, (lo, hi, "zeta")
        dx, _ = _velocity_jump(theta_p, R, 0.0, sigma, 200000, rng)
        assert abs(_z(dx * dx, beta * beta)) < Z_MAX, (lo, hi, "beta")


KD_PINS = [pin_kd_aggregation_weights, pin_kd_second_moment_exact, pin_kd_diffusive_phase_bruteforce,
           pin_kd_coarse_number_laws, pin_kd_coarse_matches_level_below, pin_kd_invariants,
           pin_kd_nonadjacent_pairs]

def pin_nonadjacent_pairs():
    """A pair of levels (l, l') with l' < l - 1 (a non-contiguous hierarchy,
    Section 4.2): its coarse path is the scheme at level l' (exact second
    moment of the discrete scheme, P1), for both couplings and M = 2, 3."""
    for k, (M, coupling, l, lc) in enumerate(((2, 1, 4, 1), (2, 0, 5, 2), (3, 1, 3, 1))):
        prob = maxwell_problem(0.2, T=1.5 if M == 3 else 1.0, M=M, coupling=coupling,
                               stream=400 + k)
        r = O.simulate(prob, l, 0, 100000, coarse_level=lc)
        assert abs(_z(r["xc"] ** 2, CF.level_second_moment(prob, lc))) < Z_MAX, (M, l, lc)
        assert abs(_z(r["xf"] ** 2, CF.level_second_moment(prob, l))) < Z_MAX, (M, l, lc)
        n_c = int(round(prob["T"] / prob["dt0"])) * M ** lc
        assert np.all(r["cc"] <= n_c)


ALL_PINS = [pin_philox_kat, pin_word_layout, pin_uniform, pin_normals, pin_second_moment_cfg1,
            pin_second_moment_levels, pin_cosine_initial, pin_heat_limit, pin_kinetic_limit,
            pin_two_point_bruteforce, pin_telescoping, pin_coupling_laws, pin_kick_block_identity,
            pin_coarse_threshold,
            pin_symmetry, pin_optimal_samples, pin_mlmc_unbiased, pin_nonadjacent_pairs]


def run_all(stop_at_first=False, pins=None):
    """Runs every pin (or those given), returns the names of the failing ones."""
    failed = []
    for f in (ALL_PINS + KD_PINS + BG_PINS if pins is None else pins):
        try:
            f()
        except Exception as e:       # a mutant may also crash or produce NaN
            failed.append("%s: %s" % (f.__name__, type(e).__name__))
            if stop_at_first:
                break
    return failed


# --------------------------------------------------------------------------
# KD scheme in the backgrounds of Section 5 (piecewise-linear collision rate)
# --------------------------------------------------------------------------
def bg_problem(kind, a, b, T=1.0, dt0=1.0, M=2, seed=42, stream=0, x0_kind=0):
    """x(0) = 1, Maxwellian mu = 0, sigma = 1, dt_l = dt0 / M^l (Section 5)."""
    return dict(eps=1.0, T=T, dt0=dt0, M=M, x0_kind=x0_kind, x0_a=1.0, x0_b=0.0, eq_kind=1,
                coupling=1, seed=seed, stream_id=stream, scheme=O.SCHEME_KD,
                background=kind, bg_a=a, bg_b=b)


def paper_rate(kind, a, b, x):
    """The collision rates R_1 and R_2 as Section 5 defines them."""
    x = np.asarray(x, dtype=np.float64)
    if kind == O.BG_B1:
        return np.where(x <= 1.0, -b * (a * (x - 1.0) - 1.0), b * (a * (x - 1.0) + 1.0))
    return np.where(x <= 1.0, b, b * (a * (x - 1.0) + 1.0))


def _thinning_flights(kind, a, b, x, v, n, rng, horizon):
    """First event times of the Poisson process of rate R(x + v t), by
    thinning with the bound of R over the flight's reach in [0, horizon]."""
    ends = x + v * np.array([0.0, horizon])
    rmax = float(np.max(paper_rate(kind, a, b, np.append(ends, 1.0))))
    t = np.zeros(n)
    out = np.full(n, np.inf)
    live = np.ones(n, dtype=bool)
    while live.any():
        idx = np.nonzero(live)[0]
        t[idx] += rng.exponential(1.0 / rmax, size=idx.size)
        over = t[idx] > horizon
        live[idx[over]] = False
        idx = idx[~over]
        acc = rng.uniform(size=idx.size) * rmax < paper_rate(kind, a, b, x + v * t[idx])
        out[idx[acc]] = t[idx[acc]]
        live[idx[acc]] = False
    return out


def pin_bg_flight_law():
    """eq. intinv: flight times from exponential numbers have the law of the
    first collision of the inhomogeneous Poisson process of rate R(x + v t),
    checked against a brute-force thinning simulation (flights that cross the
    kink at x = 1 in both directions, toward and away from higher rates)."""
    rng = np.random.default_rng(21)
    cases = [(O.BG_B1, 10.0, 1.0, 0.5, 1.3), (O.BG_B1, 10.0, 1.0, 1.4, -2.0),
             (O.BG_B2, 20.0, 2.0, 0.8, 0.9), (O.BG_B2, 5.0, 1.0, 1.5, -1.1),
             (O.BG_B1, 0.0, 3.0, 1.0, 0.7), (O.BG_B1, 50.0, 0.5, 1.0, 0.05)]
    for kind, a, b, x, v in cases:
        n = 20000
        E = rng.exponential(size=n)
        tau = np.array([O.bg_flight(kind, a, b, x, v, e) for e in E])
        for e, t in zip(E[:200], tau[:200]):     # the root solves eq. intinv
            assert abs(O.bg_rate_integral(kind, a, b, x, v, t) - e) <= 1e-12 * (1.0 + e)
        ref = _thinning_flights(kind, a, b, x, v, n, rng, 40.0 / b)
        assert np.all(np.isfinite(ref))
        assert stats.ks_2samp(tau, ref).pvalue > P_MIN, (kind, a, b, x, v)
        crossed = np.mean((x - 1.0) * (x + v * tau - 1.0) < 0.0)
        assert crossed > 0.05 or a == 0.0 or v == 0.05, (kind, a, b, x, v, crossed)


def pin_bg_rate_integral_exact():
    """The rate integral along a flight against adaptive quadrature of the
    paper's R (both sides of the kink, backward integration for t < 0)."""
    from scipy import integrate
    rng = np.random.default_rng(22)
    for _ in range(60):
        kind = int(rng.choice([O.BG_B1, O.BG_B2]))
        a, b = float(rng.uniform(0, 30)), float(rng.uniform(0.5, 5))
        x, v, t = float(rng.uniform(-1, 3)), float(rng.normal() * 2), float(rng.uniform(-1, 1))
        f = lambda s: float(paper_rate(kind, a, b, x + v * s))
        lo, hi = (0.0, t) if t >= 0 else (t, 0.0)
        pts = [(1.0 - x) / v] if v != 0 and lo < (1.0 - x) / v < hi else None
        q = integrate.quad(f, lo, hi, points=pts, epsabs=1e-13, epsrel=1e-13)[0]
        q = q if t >= 0 else -q
        assert abs(O.bg_rate_integral(kind, a, b, x, v, t) - q) <= 1e-10 * (1.0 + abs(q))


def pin_bg_homogeneous_limit():
    """a = 0 is the homogeneous background R = b: the background path agrees
    with the homogeneous KD path (exact flight E/b, coarse collision = fine
    collision) to rounding, with equal KD step counts, for paths and pairs."""
    for k, (b, level, single) in enumerate(((1.0, 3, False), (100.0, 4, False), (10.0, 2, True),
                                            (1000.0, 6, False))):
        prob = bg_problem(O.BG_B1, 0.0, b, stream=500 + k)
        h = O.simulate(prob, level, 0, 3000, single=single)
        g = O.simulate_kd_bg(prob, level, 0, 3000, single=single, general=True)
        assert np.array_equal(h["cf"], g["cf"]) and np.array_equal(h["cc"], g["cc"]), (b, level)
        scale = max(1.0, float(np.max(np.abs(h["xf"]))))
        assert np.max(np.abs(h["xf"] - g["xf"])) <= 1e-12 * scale, (b, level)
        assert np.max(np.abs(h["xc"] - g["xc"])) <= 1e-12 * scale, (b, level)


def pin_bg_symmetric_mean():
    """In the symmetric background B1 (x0 = 1, mu = 0) the law of x(T) - 1 is
    symmetric, so E[x(T)] = 1 and E[(x(T) - 1)^3] = 0, for single paths and
    both paths of a pair, in the kinetic and the diffusive regime."""
    for k, (a, b, level) in enumerate(((10.0, 1.0, 3), (10.0, 100.0, 2), (2.0, 1000.0, 6),
                                       (100.0, 10.0, 4))):
        prob = bg_problem(O.BG_B1, a, b, stream=520 + k)
        r = O.simulate(prob, level, 0, 40000)
        for x in (r["xf"], r["xc"]):
            assert abs(_z(x, 1.0)) < Z_MAX, (a, b, level)
            assert abs(_z((x - 1.0) ** 3, 0.0)) < Z_MAX, (a, b, level)


def pin_bg_pair_paths_have_level_laws():
    """In a background, the fine path of a level-l pair has the law of the
    single path of level l (the pair loop's extra fine steps beyond T are
    removed), in B1 and B2; with a = 0 the coarse path also has the law of
    the single path of level l - 1 (telescoping).  With a > 0 the coarse law
    is only close to it: the flight time then depends on the velocity, so the
    weight alpha_m = sigma tau'_m of eq. chi-update is no longer independent
    of nu_m and chi~ is not exactly N(0,1) (measured in the consistency
    harness)."""
    for k, (kind, a, b, level) in enumerate(((O.BG_B1, 10.0, 100.0, 3), (O.BG_B2, 10.0, 10.0, 2),
                                             (O.BG_B2, 50.0, 1000.0, 5), (O.BG_B1, 5.0, 1.0, 1),
                                             (O.BG_B1, 0.0, 100.0, 3), (O.BG_B2, 0.0, 3.0, 2))):
        prob = bg_problem(kind, a, b, stream=540 + k)
        pair = O.simulate_kd_bg(prob, level, 0, 40000, general=True)
        checks = [(level, pair["xf"])] + ([(level - 1, pair["xc"])] if a == 0.0 else [])
        for lev, x in checks:
            ind = O.simulate(dict(prob, stream_id=560 + k), lev, 0, 40000, single=True)
            assert stats.ks_2samp(x, ind["xf"]).pvalue > P_MIN, (kind, a, b, level, lev)
            d = np.mean(x ** 2) - np.mean(ind["xf"] ** 2)
            se = math.sqrt((np.var(x ** 2) + np.var(ind["xf"] ** 2)) / x.size)
            assert abs(d / se) < Z_MAX, (kind, a, b, level, lev)


def _kinetic_background_paths(kind, a, b, T, n, rng):
    """Brute-force velocity-jump process in a background: x(0) = 1, velocities
    N(0, 1) redrawn at the collisions of the Poisson process of rate R(x)."""
    x = np.ones(n)
    v = rng.standard_normal(n)
    t = np.zeros(n)
    live = np.ones(n, dtype=bool)
    while live.any():
        idx = np.nonzero(live)[0]
        # bound of R over the rest of each flight (|x| moves by at most |v| T)
        reach = np.abs(v[idx]) * (T - t[idx])
        rmax = paper_rate(kind, a, b, np.array([1.0]))[0] + b * a * (np.abs(x[idx] - 1.0) + reach)
        dt = rng.exponential(1.0 / rmax)
        end = t[idx] + dt >= T
        stop = idx[end]
        x[stop] += v[stop] * (T - t[stop])
        live[stop] = False
        go = idx[~end]
        dtg = dt[~end]
        x[go] += v[go] * dtg
        t[go] += dtg
        acc = rng.uniform(size=go.size) * rmax[~end] < paper_rate(kind, a, b, x[go])
        hit = go[acc]
        v[hit] = rng.standard_normal(hit.size)
    return x


def pin_bg_kinetic_limit():
    """dt << 1/R: every KD step is a kinetic flight plus a short diffusive
    remainder, so the scheme tends to the kinetic process; x(T) against a
    brute-force velocity-jump simulation in the same background (KS test and
    the second moment)."""
    rng = np.random.default_rng(23)
    for k, (kind, a, b) in enumerate(((O.BG_B1, 10.0, 1.0), (O.BG_B2, 20.0, 2.0))):
        prob = bg_problem(kind, a, b, stream=580 + k)
        kd = O.simulate(prob, 10, 0, 30000, single=True)["xf"]
        ref = _kinetic_background_paths(kind, a, b, 1.0, 30000, rng)
        assert stats.ks_2samp(kd, ref).pvalue > P_MIN, (kind, a, b)
        d = np.mean(kd ** 2) - np.mean(ref ** 2)
        se = math.sqrt((np.var(kd ** 2) + np.var(ref ** 2)) / kd.size)
        assert abs(d / se) < Z_MAX, (kind, a, b)


def pin_bg_coarse_number_laws():
    """Section 5.1's check in the paper's background B1 (a = 10, b = 100 and
    1000): the aggregated coarse numbers have the laws of the coarse path's
    own numbers -- chi~, nu~ ~ N(0,1), E~ ~ Exp(1) (eq. epsilon-update with
    the rate integral along the fine flight) -- by Anderson-Darling, and the
    phase weights satisfy the identities of the homogeneous case with the
    phase's own rate R_m (a_m = sigma nu_{m+1} zeta_m, and alpha_m nu_m =
    sigma tau_m nu_m + a_{m-1})."""
    for k, (a, b, level) in enumerate(((10.0, 100.0, 5), (10.0, 1000.0, 5), (10.0, 100.0, 9))):
        prob = bg_problem(O.BG_B1, a, b, stream=600 + k)
        rows, checked = [], 0
        for smp in range(2000 if level < 9 else 300):
            ph, co, _ = O.kd_bg_phases(prob, level, smp)
            rows.append(co)
            for m in range(ph.shape[0]):
                r = ph[m]
                assert abs(r[14] * r[5] - r[12]) <= 1e-12 * (1.0 + abs(r[12]))
                if r[1] == 0:
                    lhs, rhs = r[8] * r[10], r[3] * r[10] + ph[m - 1, 12]
                    assert abs(lhs - rhs) <= 1e-12 * (1.0 + abs(lhs))
                    checked += 1
        rows = np.concatenate(rows)
        assert rows.shape[0] > 1000 and checked > 0
        assert anderson_darling(rows[:, 0], stats.norm.cdf) < AD_MAX, (a, b, level, "chi")
        assert anderson_darling(rows[:, 1], stats.norm.cdf) < AD_MAX, (a, b, level, "nu")
        assert anderson_darling(rows[:, 2], stats.expon.cdf) < AD_MAX, (a, b, level, "E")


def pin_bg_pair_fine_path_is_its_own_path():
    """A pair's fine path consumes exactly the random numbers of a single KD
    path under the same counter tag, and the pair loop's fine steps beyond T
    only feed the coarse aggregation (the fine path ends at the first state
    whose pending collision is at or after T): positions equal to rounding,
    KD step counts equal, including the samples where the coarse path still
    collides before T after the fine path has ended."""
    for k, (kind, a, b, level) in enumerate(((O.BG_B1, 10.0, 100.0, 3), (O.BG_B2, 50.0, 10.0, 2),
                                             (O.BG_B1, 100.0, 1.0, 4), (O.BG_B2, 10.0, 1000.0, 6))):
        prob = bg_problem(kind, a, b, stream=620 + k)
        pair = O.simulate(prob, level, 0, 20000)
        own = O.simulate_kd_bg(prob, level, 0, 20000, single=True, pair_tag=True)
        assert np.array_equal(pair["cf"], own["cf"]), (kind, a, b, level)
        assert np.max(np.abs(pair["xf"] - own["xf"])) <= 1e-13 * (1.0 + np.max(np.abs(own["xf"])))


BG_PINS = [pin_bg_pair_fine_path_is_its_own_path, pin_bg_flight_law, pin_bg_rate_integral_exact, pin_bg_homogeneous_limit,
           pin_bg_symmetric_mean, pin_bg_pair_paths_have_level_laws, pin_bg_kinetic_limit,
           pin_bg_coarse_number_laws]


if __name__ == "__main__":
    import json
    import sys
    sel = KD_PINS if "--kd" in sys.argv else (BG_PINS if "--bg" in sys.argv else None)
    print(json.dumps(run_all(stop_at_first="--first" in sys.argv, pins=sel)))
