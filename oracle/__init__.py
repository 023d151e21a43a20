"""FP64 CPU oracle of the multilevel asymptotic-preserving Monte Carlo method.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark.  The product package never imports it, and
it imports nothing from the product package.

Contents
--------
``oracle.c``           particle schemes (asymptotic-preserving splitting and the
                       kinetic-diffusion scheme), fine/coarse correlation,
                       Philox4x32-10 (plain C, double precision, one
                       trajectory at a time)
``closed_form.py``     exact second moment of the discrete scheme and its
                       kinetic and diffusive limits
``mlmc.py``            two-pass level statistics, optimal sample numbers
                       (Section 4.1, eqs. Nopt1/Noptj) and the MLMC loop
``build.py``           compiles ``oracle.c`` with gcc into ``liboracle.so``
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB_PATH lets the mutation tests load a deliberately broken build.
_LIB_PATH = os.environ.get("ORACLE_LIB_PATH", os.path.join(_HERE, "liboracle.so"))
_lib = None

X0_DELTA, X0_NORMAL, X0_COSINE = 0, 1, 2
BG_DIFFUSIVE, BG_B1, BG_B2 = 0, 1, 2
QOI_X2, QOI_X2_HIST, QOI_X = 0, 1, 2
EQ_TWO_POINT, EQ_MAXWELLIAN = 0, 1
COUPLING_KICK_SUM, COUPLING_AGGREGATE = 0, 1
SCHEME_SPLITTING, SCHEME_KD = 0, 1


def lib():
    """Loads ``liboracle.so``, building it with gcc first if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _build
            _build.build()
        L = ctypes.CDLL(_LIB_PATH)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.oracle_philox4x32_10.restype = None
        L.oracle_uniform.argtypes = [ctypes.c_uint32]
        L.oracle_uniform.restype = ctypes.c_double
        L.oracle_cosine_icdf.argtypes = [ctypes.c_double]
        L.oracle_cosine_icdf.restype = ctypes.c_double
        L.oracle_coarse_threshold.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int]
        L.oracle_coarse_threshold.restype = ctypes.c_uint64
        L.oracle_level_consts.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_int, ctypes.c_int, dp, u64p]
        L.oracle_level_consts.restype = None
        common = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                  ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                  ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                  ctypes.c_uint32]
        L.oracle_simulate.argtypes = common + [ctypes.c_uint64, u64p, ctypes.c_uint64,
                                               dp, dp, u32p, u32p, ctypes.c_int]
        L.oracle_simulate.restype = ctypes.c_int
        L.oracle_trace.argtypes = common + [ctypes.c_uint64, dp, ctypes.c_uint64, dp]
        L.oracle_trace.restype = ctypes.c_uint64
        L.oracle_words.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, u32p]
        L.oracle_words.restype = None
        L.oracle_simulate_kd.argtypes = L.oracle_simulate.argtypes
        L.oracle_simulate_kd.restype = ctypes.c_int
        L.oracle_simulate_pair.argtypes = [
            ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
            ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, u64p,
            ctypes.c_uint64, dp, dp, u32p, u32p, ctypes.c_int]
        L.oracle_simulate_pair.restype = ctypes.c_int
        L.oracle_kd_coeffs.argtypes = [ctypes.c_double] * 5 + [dp]
        L.oracle_kd_coeffs.restype = None
        L.oracle_kd_coarse_numbers.argtypes = [
            ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
            ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
            ctypes.c_uint32, ctypes.c_uint64, dp, ctypes.c_uint64, dp]
        L.oracle_kd_coarse_numbers.restype = ctypes.c_uint64
        L.oracle_kd_phases.argtypes = [
            ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
            ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
            ctypes.c_uint32, ctypes.c_uint64, dp, ctypes.c_uint64, dp, ctypes.c_uint64, u64p, dp]
        L.oracle_kd_phases.restype = ctypes.c_uint64
        L.oracle_simulate_kd_bg.argtypes = [
            ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
            ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
            ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32,
            ctypes.c_uint64, u64p, ctypes.c_uint64, dp, dp, u32p, u32p, ctypes.c_int]
        L.oracle_simulate_kd_bg.restype = ctypes.c_int
        L.oracle_kd_bg_phases.argtypes = [
            ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
            ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double,
            ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, dp,
            ctypes.c_uint64, dp, ctypes.c_uint64, u64p, dp]
        L.oracle_kd_bg_phases.restype = ctypes.c_uint64
        for name in ("oracle_bg_rate", "oracle_bg_rate_integral", "oracle_bg_flight"):
            getattr(L, name).restype = ctypes.c_double
        L.oracle_bg_rate.argtypes = [ctypes.c_int] + [ctypes.c_double] * 3
        L.oracle_bg_rate_integral.argtypes = [ctypes.c_int] + [ctypes.c_double] * 5
        L.oracle_bg_flight.argtypes = [ctypes.c_int] + [ctypes.c_double] * 5
        _lib = L
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def default_threads():
    return max(1, len(os.sched_getaffinity(0)))


def philox4x32_10(ctr, key):
    """One Philox4x32-10 block: four counter words, two key words -> four words."""
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                               _ptr(out, ctypes.c_uint32))
    return out


def uniform(w):
    return lib().oracle_uniform(int(w))


def cosine_icdf(u):
    return lib().oracle_cosine_icdf(float(u))


def coarse_threshold(thr_f, thr_c, M):
    return int(lib().oracle_coarse_threshold(int(thr_f), int(thr_c), int(M)))


def level_consts(eps, T, dt0, M, level):
    """(dt, h, s, p, n_steps, threshold) of one level."""
    d = np.zeros(4)
    n = np.zeros(2, dtype=np.uint64)
    lib().oracle_level_consts(eps, T, dt0, M, level, _ptr(d, ctypes.c_double),
                              _ptr(n, ctypes.c_uint64))
    return dict(dt=d[0], h=d[1], s=d[2], p=d[3], n_steps=int(n[0]), thr=int(n[1]))


def _common_args(prob, level, single):
    return (float(prob["eps"]), float(prob["T"]), float(prob["dt0"]), int(prob["M"]),
            int(level), int(bool(single)), int(prob["x0_kind"]), float(prob.get("x0_a", 0.0)),
            float(prob.get("x0_b", 0.0)), int(prob["eq_kind"]), int(prob.get("coupling", 0)),
            int(prob.get("seed", 42)), int(prob.get("stream_id", 0)))


def simulate(prob, level, sample_begin=0, n=None, samples=None, single=False, threads=None,
             coarse_level=None):
    """Final positions and collision counts of fine/coarse pairs.

    ``prob`` is a dict with keys eps, T, dt0, M, x0_kind, x0_a, x0_b, eq_kind,
    coupling, seed, stream_id and optionally scheme (SCHEME_SPLITTING, the
    default, or SCHEME_KD: the kinetic-diffusion scheme, Maxwellian only;
    its counts are KD steps, i.e. collisions before T).  Either a contiguous
    range [sample_begin, sample_begin+n) or an explicit index array
    ``samples``.  ``coarse_level`` (pairs only; default level - 1) puts the
    coarse path of the pair at that level (one coarse step per
    M^(level - coarse_level) fine steps).  Returns dict(xf, xc, cf, cc) of
    numpy arrays.
    """
    kd = int(prob.get("scheme", SCHEME_SPLITTING)) == SCHEME_KD
    if kd and int(prob["eq_kind"]) != EQ_MAXWELLIAN:
        raise ValueError("the KD scheme needs the Maxwellian equilibrium")
    if kd and int(prob.get("background", BG_DIFFUSIVE)) != BG_DIFFUSIVE:
        return simulate_kd_bg(prob, level, sample_begin, n, samples, single, threads,
                              coarse_level)
    if samples is not None:
        idx = np.ascontiguousarray(samples, dtype=np.uint64)
        count = idx.size
        idx_p = _ptr(idx, ctypes.c_uint64)
    else:
        count = int(n)
        idx = None
        idx_p = None
    xf = np.zeros(count)
    xc = np.zeros(count)
    cf = np.zeros(count, dtype=np.uint32)
    cc = np.zeros(count, dtype=np.uint32)
    if count:
        if coarse_level is not None and not single and int(coarse_level) != int(level) - 1:
            a = _common_args(prob, level, single)
            st = lib().oracle_simulate_pair(
                int(kd), *a[:5], int(coarse_level), *a[6:], int(sample_begin), idx_p, count,
                _ptr(xf, ctypes.c_double), _ptr(xc, ctypes.c_double),
                _ptr(cf, ctypes.c_uint32), _ptr(cc, ctypes.c_uint32),
                int(threads or default_threads()))
            if st != 0:
                raise ValueError("coarse_level must be in [0, level)")
            return dict(xf=xf, xc=xc, cf=cf, cc=cc)
        fn = lib().oracle_simulate_kd if kd else lib().oracle_simulate
        fn(*_common_args(prob, level, single), int(sample_begin), idx_p,
                              count, _ptr(xf, ctypes.c_double), _ptr(xc, ctypes.c_double),
                              _ptr(cf, ctypes.c_uint32), _ptr(cc, ctypes.c_uint32),
                              int(threads or default_threads()))
    return dict(xf=xf, xc=xc, cf=cf, cc=cc)


TRACE_COLUMNS = ("n", "w_decision", "w_radius", "w_angle", "words_used", "u1", "u2", "xi", "g",
                 "hit", "xf", "vf", "kick", "coarse_hit", "xc", "vc")


def trace(prob, level, sample, single=False):
    """Per-fine-step record of one sample (columns ``TRACE_COLUMNS``) and
    the final (x_f, x_c)."""
    nsteps = level_consts(prob["eps"], prob["T"], prob["dt0"], prob["M"], level)["n_steps"]
    rows = np.zeros((nsteps, 16))
    fin = np.zeros(2)
    used = lib().oracle_trace(*_common_args(prob, level, single), int(sample),
                              _ptr(rows, ctypes.c_double), nsteps, _ptr(fin, ctypes.c_double))
    return rows[:used], fin


def words(seed, stream_id, tag, sample_begin, n_samples, n_steps):
    """Philox words, array [n_samples, n_steps, 4] for counters
    (step, sample, tag, stream_id)."""
    out = np.zeros((n_samples, n_steps, 4), dtype=np.uint32)
    lib().oracle_words(int(seed), int(stream_id), int(tag), int(sample_begin), int(n_samples),
                       int(n_steps), _ptr(out, ctypes.c_uint32))
    return out


def kd_coeffs(theta, R, mu, sigma, v_next):
    """(a, d): advection and diffusion coefficient of a KD diffusive phase of
    length theta ending with velocity v_next (eqs. advection and diffusion,
    homogeneous background with collision rate R and Maxwellian N(mu,
    sigma^2))."""
    out = np.zeros(2)
    lib().oracle_kd_coeffs(float(theta), float(R), float(mu), float(sigma), float(v_next),
                           _ptr(out, ctypes.c_double))
    return float(out[0]), float(out[1])


def kd_coarse_numbers(prob, level, sample, cap=None, coarse_level=None):
    """Coarse numbers of one KD pair (coarse path at coarse_level, default
    level - 1), one row per coarse KD step: (chi~, nu~, E~, fine KD steps
    aggregated), and the final (x_f, x_c)."""
    if cap is None:   # coarse steps of a pair, up to the end of the last one (past T)
        cap = 2 * int(math.ceil(prob["T"] / prob["dt0"] - 1e-9)) * int(prob["M"]) ** level + 8
    rows = np.zeros((cap, 4))
    fin = np.zeros(2)
    used = lib().oracle_kd_coarse_numbers(
        float(prob["eps"]), float(prob["T"]), float(prob["dt0"]), int(prob["M"]), int(level),
        int(level - 1 if coarse_level is None else coarse_level), int(prob["x0_kind"]), float(prob.get("x0_a", 0.0)), float(prob.get("x0_b", 0.0)),
        int(prob.get("seed", 42)), int(prob.get("stream_id", 0)), int(sample),
        _ptr(rows, ctypes.c_double), cap, _ptr(fin, ctypes.c_double))
    return rows[:used], fin


KD_PHASE_COLUMNS = ("window", "first", "t", "tau", "theta", "zeta", "theta_p", "tau_p", "alpha",
                    "beta", "nu", "chi", "a", "d", "nu_next", "xf")


def kd_phases(prob, level, sample, coarse_level=None):
    """Fine KD phases of one pair, one row per fine KD step (columns
    ``KD_PHASE_COLUMNS``: the coarse step it is aggregated into, whether it
    opens that window, flight start time and length, theta, zeta, theta',
    tau', the weights alpha and beta, its numbers nu, chi, its a and d, the
    next velocity number and x_f after it), the coarse rows of
    ``kd_coarse_numbers`` and the final (x_f, x_c)."""
    cap = 2 * int(math.ceil(prob["T"] / prob["dt0"] - 1e-9)) * int(prob["M"]) ** level + 8
    phases = np.zeros((cap, 16))
    rows = np.zeros((cap, 4))
    fin = np.zeros(2)
    nc = np.zeros(1, dtype=np.uint64)
    used = lib().oracle_kd_phases(
        float(prob["eps"]), float(prob["T"]), float(prob["dt0"]), int(prob["M"]), int(level),
        int(level - 1 if coarse_level is None else coarse_level), int(prob["x0_kind"]),
        float(prob.get("x0_a", 0.0)), float(prob.get("x0_b", 0.0)),
        int(prob.get("seed", 42)), int(prob.get("stream_id", 0)), int(sample),
        _ptr(phases, ctypes.c_double), cap, _ptr(rows, ctypes.c_double), cap,
        _ptr(nc, ctypes.c_uint64), _ptr(fin, ctypes.c_double))
    return phases[:used], rows[:int(nc[0])], fin


def simulate_kd_bg(prob, level, sample_begin=0, n=None, samples=None, single=False, threads=None,
                   coarse_level=None, general=False, pair_tag=False):
    """KD paths or pairs in a background of Section 5 (prob["background"] =
    BG_B1 or BG_B2, parameters prob["bg_a"], prob["bg_b"]; Maxwellian with mu
    = 0, sigma = 1; eps is not used).  general=True takes the background path
    also at a = 0 (which otherwise runs the homogeneous path with R = b);
    pair_tag=True runs single paths under the counter tag of the level's
    pairs (the random numbers of the pairs' fine paths)."""
    if samples is not None:
        idx = np.ascontiguousarray(samples, dtype=np.uint64)
        count = idx.size
        idx_p = _ptr(idx, ctypes.c_uint64)
    else:
        count = int(n)
        idx_p = None
    xf = np.zeros(count)
    xc = np.zeros(count)
    cf = np.zeros(count, dtype=np.uint32)
    cc = np.zeros(count, dtype=np.uint32)
    if count:
        st = lib().oracle_simulate_kd_bg(
            float(prob["T"]), float(prob["dt0"]), int(prob["M"]), int(level),
            -1 if coarse_level is None else int(coarse_level),
            2 if (single and pair_tag) else int(bool(single)),
            int(prob["x0_kind"]), float(prob.get("x0_a", 0.0)), float(prob.get("x0_b", 0.0)),
            int(prob["background"]), float(prob["bg_a"]), float(prob["bg_b"]), int(bool(general)),
            int(prob.get("seed", 42)), int(prob.get("stream_id", 0)), int(sample_begin), idx_p,
            count, _ptr(xf, ctypes.c_double), _ptr(xc, ctypes.c_double),
            _ptr(cf, ctypes.c_uint32), _ptr(cc, ctypes.c_uint32), int(threads or default_threads()))
        if st != 0:
            raise ValueError("bad background or coarse level")
    return dict(xf=xf, xc=xc, cf=cf, cc=cc)


def kd_bg_phases(prob, level, sample, coarse_level=None):
    """As kd_phases for a pair in a background (phase column 15 = the phase's
    collision rate R_m)."""
    cap = 2 * int(math.ceil(prob["T"] / prob["dt0"] - 1e-9)) * int(prob["M"]) ** level + 8
    phases = np.zeros((cap, 16))
    rows = np.zeros((cap, 4))
    fin = np.zeros(2)
    nc = np.zeros(1, dtype=np.uint64)
    used = lib().oracle_kd_bg_phases(
        float(prob["T"]), float(prob["dt0"]), int(prob["M"]), int(level),
        int(level - 1 if coarse_level is None else coarse_level), int(prob["x0_kind"]),
        float(prob.get("x0_a", 0.0)), float(prob.get("x0_b", 0.0)), int(prob["background"]),
        float(prob["bg_a"]), float(prob["bg_b"]), int(prob.get("seed", 42)),
        int(prob.get("stream_id", 0)), int(sample), _ptr(phases, ctypes.c_double), cap,
        _ptr(rows, ctypes.c_double), cap, _ptr(nc, ctypes.c_uint64), _ptr(fin, ctypes.c_double))
    return phases[:used], rows[:int(nc[0])], fin


def bg_rate(kind, a, b, x):
    return lib().oracle_bg_rate(int(kind), float(a), float(b), float(x))


def bg_rate_integral(kind, a, b, x, v, t):
    """int_0^t R(x + v s) ds of a background."""
    return lib().oracle_bg_rate_integral(int(kind), float(a), float(b), float(x), float(v),
                                         float(t))


def bg_flight(kind, a, b, x, v, E):
    """Flight time of eq. intinv in a background."""
    return lib().oracle_bg_flight(int(kind), float(a), float(b), float(x), float(v), float(E))
