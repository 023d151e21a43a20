"""Synthetic workloads shared by the tests, the smoke check and the benchmark.

Holds only problem parameters and seeded input generators (no arithmetic of
the particle method), so both the FP64 oracle and the HIP library can be fed
from it.  Each workload restates one configuration of the multilevel
asymptotic-preserving Monte Carlo study in plain numbers:

* ``cfg1``  single-level scheme, FP64 state: x0 = 0, velocities +-1,
            eps = 0.5, T = 0.5, dt = 0.01 (50 steps), N = 1e5, seed 42.
* ``cfg2``  MLMC: x0 ~ N(0,1), Maxwellian equilibrium, eps = 0.01, T = 1,
            dt0 = 0.5, M = 2, levels 0..8, RMSE 1e-3, FP32 state.
* ``cfg3``  eps sweep {1e-4, 1e-3, 1e-2, 1e-1, 1} x RMSE {1e-2, 3e-3, 1e-3}
            with the cfg2 setup, all requests in one batched launch.
* ``cfg4``  precision study: x0 with density 1 + cos(2 pi x) on [0,1],
            eps = 1e-3, T = 1, dt0 = 0.5, M = 2, L = 10; x^2 and a 64-bin
            histogram on [-4, 5).
* ``cfg_kd`` the cfg2 estimate with the kinetic-diffusion scheme (homogeneous
            background: collision rate 1/eps^2, Maxwellian velocities of
            standard deviation 1/eps), FP64 state.
* ``cfg_bg`` the test case of Section 5: KD scheme, x(0) = 1, T = 1, dt_l =
            2^-l, Maxwellian N(0, 1), collision rate of background B1
            (b (a |x-1| + 1)) or B2 (b left of 1, b (a (x-1) + 1) right of it),
            QoI the position x(T).
* ``cfg5``  serving stream: Poisson arrivals at 200/s, eps log-uniform in
            [1e-4, 1], T uniform in [0.1, 1] (dt0 = T/2, L = 8), RMSE
            log-uniform in [1e-3, 1e-2], Maxwellian, x0 ~ N(0,1).
"""
import numpy as np

X0_DELTA, X0_NORMAL, X0_COSINE = 0, 1, 2
BG_DIFFUSIVE, BG_B1, BG_B2 = 0, 1, 2
QOI_X2, QOI_X2_HIST, QOI_X = 0, 1, 2
EQ_TWO_POINT, EQ_MAXWELLIAN = 0, 1
COUPLING_KICK_SUM, COUPLING_AGGREGATE = 0, 1
SCHEME_SPLITTING, SCHEME_KD = 0, 1


def cfg1():
    return dict(eps=0.5, T=0.5, dt0=0.01, M=2, L=0, x0_kind=X0_DELTA, x0_a=0.0, x0_b=0.0,
                eq_kind=EQ_TWO_POINT, coupling=COUPLING_KICK_SUM, fp64_state=1, seed=42,
                stream_id=1)


CFG1_N = 100000


def cfg2(eps=0.01, coupling=COUPLING_AGGREGATE, stream_id=2):
    return dict(eps=eps, T=1.0, dt0=0.5, M=2, L=8, x0_kind=X0_NORMAL, x0_a=0.0, x0_b=1.0,
                eq_kind=EQ_MAXWELLIAN, coupling=coupling, fp64_state=0, seed=42,
                stream_id=stream_id)


CFG2_TOL = 1e-3

CFG3_EPS = (1e-4, 1e-3, 1e-2, 1e-1, 1.0)
CFG3_TOL = (1e-2, 3e-3, 1e-3)


def cfg_kd(eps=0.01, stream_id=6):
    """The cfg2 estimate with the kinetic-diffusion scheme instead of the
    splitting scheme (homogeneous background, FP64 state)."""
    return dict(cfg2(eps=eps, stream_id=stream_id), fp64_state=1, scheme=SCHEME_KD)


def cfg_bg(background=BG_B1, a=10.0, b=1000.0, M=2, L=8, stream_id=7):
    """The test case of Section 5 with the KD scheme: x(0) = 1, T = 1, time
    steps dt_l = 2^-l (dt0 = 1, M = 2), Maxwellian N(0, 1), collision rate of
    background B1 or B2 with parameters a, b; QoI the position x(T)."""
    return dict(eps=0.0, T=1.0, dt0=1.0, M=M, L=L, x0_kind=X0_DELTA, x0_a=1.0, x0_b=0.0,
                eq_kind=EQ_MAXWELLIAN, coupling=COUPLING_AGGREGATE, fp64_state=1, seed=42,
                stream_id=stream_id, scheme=SCHEME_KD, background=background, bg_a=a, bg_b=b,
                qoi=QOI_X)


def cfg3():
    """(problems, tolerances) of the eps sweep; stream_id = request index."""
    probs, tols = [], []
    k = 0
    for eps in CFG3_EPS:
        for tol in CFG3_TOL:
            probs.append(cfg2(eps=eps, stream_id=100 + k))
            tols.append(tol)
            k += 1
    return probs, tols


def cfg4(fp64_state=0):
    return dict(eps=1e-3, T=1.0, dt0=0.5, M=2, L=10, x0_kind=X0_COSINE, x0_a=0.0, x0_b=0.0,
                eq_kind=EQ_MAXWELLIAN, coupling=COUPLING_AGGREGATE, fp64_state=fp64_state,
                seed=42, stream_id=4, qoi=1, nbins=64, hist_lo=-4.0, hist_hi=5.0)


def cfg5_trace(n, rate=200.0, seed=1234):
    """Poisson arrival times and per-request problems/tolerances."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n))
    eps = 10.0 ** rng.uniform(-4.0, 0.0, size=n)
    T = rng.uniform(0.1, 1.0, size=n)
    tol = 10.0 ** rng.uniform(-3.0, -2.0, size=n)
    probs = []
    for i in range(n):
        probs.append(dict(eps=float(eps[i]), T=float(T[i]), dt0=float(T[i]) / 2.0, M=2, L=8,
                          x0_kind=X0_NORMAL, x0_a=0.0, x0_b=1.0, eq_kind=EQ_MAXWELLIAN,
                          coupling=COUPLING_AGGREGATE, fp64_state=0, seed=42,
                          stream_id=1000 + i))
    return arrivals.tolist(), probs, tol.tolist()
