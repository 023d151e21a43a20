"""Python binding of ``libmlmc_ap.so`` (multilevel asymptotic-preserving Monte
Carlo on MI355X).

Argument marshalling only: every step of the particle method runs in the HIP
kernels behind the C ABI declared in ``include/mlmc_ap.h``; the functions
here carry the same names.  PyTorch is used only to hand over device memory
(tensors for the optional dumps) and the current HIP stream.

If the library has not been built this module raises on import of any entry
point -- there is no fallback.
"""
import ctypes
import struct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlmc_ap.so")

MAX_LEVELS = 31

X0_DELTA, X0_NORMAL, X0_COSINE = 0, 1, 2
EQ_TWO_POINT, EQ_MAXWELLIAN = 0, 1
COUPLING_KICK_SUM, COUPLING_AGGREGATE = 0, 1
QOI_X2, QOI_X2_HIST, QOI_X = 0, 1, 2
BG_DIFFUSIVE, BG_B1, BG_B2 = 0, 1, 2
SCHEME_SPLITTING, SCHEME_KD = 0, 1

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EBUSY",
          -5: "ECANCELLED", -6: "ENOTFOUND", -7: "EAGAIN"}


class MlmcApError(RuntimeError):
    def __init__(self, status, where, detail):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__("%s failed: %s (%s)" % (where, self.name, detail))


class Problem(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("T", ctypes.c_double), ("dt0", ctypes.c_double),
                ("M", ctypes.c_int32), ("L", ctypes.c_int32), ("x0_kind", ctypes.c_int32),
                ("eq_kind", ctypes.c_int32), ("x0_a", ctypes.c_double), ("x0_b", ctypes.c_double),
                ("coupling", ctypes.c_int32), ("qoi", ctypes.c_int32), ("nbins", ctypes.c_int32),
                ("fp64_state", ctypes.c_int32), ("hist_lo", ctypes.c_double),
                ("hist_hi", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("stream_id", ctypes.c_uint32), ("scheme", ctypes.c_uint32),
                ("background", ctypes.c_uint32), ("bg_a", ctypes.c_double),
                ("bg_b", ctypes.c_double)]


class LevelStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("mean_dq", ctypes.c_double), ("m2_dq", ctypes.c_double),
                ("mean_qf", ctypes.c_double), ("m2_qf", ctypes.c_double),
                ("mean_qc", ctypes.c_double), ("m2_qc", ctypes.c_double),
                ("c_fc", ctypes.c_double), ("coll_f", ctypes.c_uint64), ("coll_c", ctypes.c_uint64)]


class LevelInfo(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("dt", "h", "s", "p", "dt_c", "h_c", "s_c", "p_c")] + \
               [(k, ctypes.c_uint64) for k in ("n_steps", "thr_f", "thr_c", "thr_c2")]


class Tuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("ppt", ctypes.c_int32),
                ("waves_per_simd", ctypes.c_int32), ("tp_max_samples", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("batched", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("n_warmup", ctypes.c_uint64), ("tuning", Tuning),
                ("level_select", ctypes.c_int32), ("L_max", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("estimate", ctypes.c_double), ("var_estimator", ctypes.c_double),
                ("L", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("status", ctypes.c_int32),
                ("N", ctypes.c_uint64 * MAX_LEVELS), ("lv", LevelStats * MAX_LEVELS),
                ("particle_steps", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("seconds", ctypes.c_double), ("gpu_seconds", ctypes.c_double),
                ("kernel_seconds", ctypes.c_double), ("level_mask", ctypes.c_uint64),
                ("bias_estimate", ctypes.c_double), ("bias_se", ctypes.c_double),
                ("tau", ctypes.c_int32), ("levels_added", ctypes.c_int32),
                ("device_planned", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_samples_per_tick", ctypes.c_uint64),
                ("max_active", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("options", Options)]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in
                ("submitted", "admitted", "completed", "cancelled", "rejected", "ticks",
                 "particle_steps", "bytes_reserved", "bytes_peak")] + \
               [("active", ctypes.c_int32), ("queued", ctypes.c_int32),
                ("busy_seconds", ctypes.c_double)]


_P = ctypes.POINTER
_vp = ctypes.c_void_p
# name -> argtypes (restype is the int status unless listed in _RESTYPE)
_SIGNATURES = {
    "mlmc_ap_init": [],
    "mlmc_ap_release": [],
    "mlmc_ap_status_str": [ctypes.c_int],
    "mlmc_ap_last_error": [],
    "mlmc_ap_version": [],
    "mlmc_ap_validate": [_P(Problem)],
    "mlmc_ap_level_constants": [_P(Problem), ctypes.c_int32, _P(LevelInfo)],
    "mlmc_ap_optimal_samples": [_P(ctypes.c_double), _P(ctypes.c_double), ctypes.c_int32,
                                ctypes.c_double, _P(ctypes.c_uint64)],
    "mlmc_ap_merge_stats": [_P(LevelStats), _P(LevelStats), _P(LevelStats)],
    "mlmc_ap_simulate_level": [_P(Problem), ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                               ctypes.c_uint64, _P(LevelStats), _vp, _vp, _P(ctypes.c_uint64), _vp],
    "mlmc_ap_simulate_pair": [_P(Problem), ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                              ctypes.c_uint64, _P(LevelStats), _vp, _vp, _P(ctypes.c_uint64), _vp],
    "mlmc_ap_kd_coarse_numbers": [_P(Problem), ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                  ctypes.c_uint64, ctypes.c_uint32, _vp, _vp, _vp],
    "mlmc_ap_simulate_level_noalloc": [_P(Problem), ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_uint64, ctypes.c_uint64, _P(LevelStats), _vp, _vp,
                                       _P(ctypes.c_uint64), _vp],
    "mlmc_ap_select_levels_heuristic": [_P(ctypes.c_double), _P(ctypes.c_double), ctypes.c_int32,
                                        _P(ctypes.c_uint64)],
    "mlmc_ap_warmup_depth": [_P(Problem), _P(ctypes.c_int32)],
    "mlmc_ap_extrapolate_variances": [_P(ctypes.c_double), _P(ctypes.c_double), ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_int32, _P(ctypes.c_double),
                                      _P(ctypes.c_double)],
    "mlmc_ap_select_levels_optimal": [_P(ctypes.c_double), _P(ctypes.c_double),
                                      _P(ctypes.c_double), _P(ctypes.c_double), ctypes.c_int32,
                                      _P(ctypes.c_uint64), _P(ctypes.c_double)],
    "mlmc_ap_estimate": [_P(Problem), ctypes.c_double, _P(Options), _P(Result),
                         _P(ctypes.c_uint64), _vp],
    "mlmc_ap_estimate_sequence": [_P(Problem), ctypes.c_double, ctypes.c_int32, _P(Options),
                                  _P(Result), _vp],
    "mlmc_ap_plain_mc": [_P(Problem), ctypes.c_double, _P(Options), _P(Result), _vp],
    "mlmc_ap_estimate_batch": [_P(Problem), _P(ctypes.c_double), ctypes.c_int32, _P(Options),
                               _P(Result), _vp],
    "mlmc_ap_autotune": [_P(Problem), ctypes.c_double, ctypes.c_char_p, _P(Tuning), _vp],
    "mlmc_ap_set_tuning": [_P(Tuning)],
    "mlmc_ap_server_create": [_P(ServerConfig), _P(_vp)],
    "mlmc_ap_server_destroy": [_vp],
    "mlmc_ap_server_submit": [_vp, _P(Problem), ctypes.c_double, _P(ctypes.c_uint64)],
    "mlmc_ap_server_step": [_vp, _P(ctypes.c_int32)],
    "mlmc_ap_server_poll": [_vp, ctypes.c_uint64, _P(Result)],
    "mlmc_ap_server_cancel": [_vp, ctypes.c_uint64],
    "mlmc_ap_server_get_stats": [_vp, _P(ServerStats)],
    "mlmc_ap_server_run_trace": [_vp, ctypes.c_int32, _P(ctypes.c_double), _P(Problem),
                                 _P(ctypes.c_double), _P(Result), _P(ctypes.c_double)],
    "mlmc_ap_philox_words": [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                             ctypes.c_uint64, ctypes.c_uint32, _vp, _vp],
    "mlmc_ap_rng_normals": [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                            ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32, _vp, _vp],
}
_RESTYPE = {"mlmc_ap_status_str": ctypes.c_char_p, "mlmc_ap_last_error": ctypes.c_char_p,
            "mlmc_ap_version": ctypes.c_char_p}

_lib = None


def lib():
    """The loaded ``libmlmc_ap.so``; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmlmc_ap.so is not built (%s); run "
                               "python -m paper_2004_04071_amd.build" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = _RESTYPE.get(name, ctypes.c_int)
        _lib = L
    return _lib


def _check(status, where):
    if status != 0:
        raise MlmcApError(status, where, lib().mlmc_ap_last_error().decode())
    return status


def _stream(stream):
    """A hipStream_t handle: explicit int/None, a torch stream, or torch's
    current stream when torch's GPU runtime is already initialised."""
    if stream is None:
        try:
            import torch
            if torch.cuda.is_initialized():
                return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        except ImportError:
            pass
        return None
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _dev_ptr(t, min_elems, dtypes, what):
    """Device address of an optional output tensor after checking, before any
    launch, everything the kernels will assume of it: a contiguous GPU tensor
    of one of ``dtypes`` (names of torch dtypes) with at least ``min_elems``
    elements.  The kernels write that many elements without bounds checks."""
    if t is None:
        return None
    if not hasattr(t, "data_ptr") or not hasattr(t, "dtype"):
        raise TypeError("%s must be a torch GPU tensor" % what)
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("%s must be a contiguous GPU tensor" % what)
    name = str(t.dtype).replace("torch.", "")
    if name not in dtypes:
        raise ValueError("%s must have dtype %s, not %s" % (what, " or ".join(dtypes), name))
    if t.numel() < min_elems:
        raise ValueError("%s holds %d elements; %d are written" % (what, t.numel(), min_elems))
    return ctypes.c_void_p(t.data_ptr())


def _traj_dtype(P):
    """Element type of the trajectory dump: double for FP64 state and the KD
    scheme (which runs in FP64), float otherwise."""
    return "float64" if (P.fp64_state or P.scheme == SCHEME_KD) else "float32"


def _dump_ptrs(P, n_samples, traj, coll):
    n2 = 2 * int(n_samples)
    return (_dev_ptr(traj, n2, (_traj_dtype(P),), "traj"),
            _dev_ptr(coll, n2, ("int32", "uint32"), "coll"))


def problem(eps, T, dt0, M=2, L=0, x0_kind=X0_NORMAL, x0_a=0.0, x0_b=1.0, eq_kind=EQ_MAXWELLIAN,
            coupling=None, qoi=QOI_X2, nbins=64, hist_lo=-4.0, hist_hi=5.0, fp64_state=0,
            seed=42, stream_id=0, scheme=SCHEME_SPLITTING, background=BG_DIFFUSIVE, bg_a=0.0,
            bg_b=0.0):
    """Builds an ``mlmc_ap_problem``; the coupling defaults to the aggregated
    kick for the Maxwellian equilibrium and the kick sum otherwise.
    ``scheme``: SCHEME_SPLITTING (default) or SCHEME_KD (kinetic-diffusion;
    Maxwellian, fp64_state = 1, and eps > 0 or a background).  ``background``
    (KD only): BG_DIFFUSIVE (rate 1/eps^2) or BG_B1 / BG_B2 of Section 5 with
    parameters ``bg_a`` >= 0, ``bg_b`` > 0."""
    if coupling is None:
        coupling = COUPLING_AGGREGATE if eq_kind == EQ_MAXWELLIAN else COUPLING_KICK_SUM
    return Problem(eps=eps, T=T, dt0=dt0, M=M, L=L, x0_kind=x0_kind, eq_kind=eq_kind, x0_a=x0_a,
                   x0_b=x0_b, coupling=coupling, qoi=qoi, nbins=nbins, fp64_state=fp64_state,
                   hist_lo=hist_lo, hist_hi=hist_hi, seed=seed, stream_id=stream_id,
                   scheme=scheme, background=background, bg_a=bg_a, bg_b=bg_b)


def as_problem(p):
    if isinstance(p, Problem):
        return p
    return problem(**p)


def stats_dict(s):
    return {k: getattr(s, k) for k, _ in LevelStats._fields_}


_STATS_NAMES = tuple(k for k, _ in LevelStats._fields_)
_STATS_FORMAT = "<Q7dQQ"  # the LevelStats layout (80 bytes)
assert struct.calcsize(_STATS_FORMAT) == ctypes.sizeof(LevelStats)


def result_dict(r):
    L = r.L
    raw = ctypes.string_at(ctypes.addressof(r.lv), (L + 1) * ctypes.sizeof(LevelStats))
    return dict(estimate=r.estimate, var_estimator=r.var_estimator, L=L,
                iterations=r.iterations, converged=bool(r.converged), status=r.status,
                N=list(r.N[:L + 1]),
                levels=[dict(zip(_STATS_NAMES, t)) for t in struct.iter_unpack(_STATS_FORMAT, raw)],
                particle_steps=int(r.particle_steps), launches=int(r.launches),
                seconds=r.seconds, gpu_seconds=r.gpu_seconds, kernel_seconds=r.kernel_seconds,
                level_mask=int(r.level_mask),
                level_set=[l for l in range(L + 1) if (int(r.level_mask) >> l) & 1],
                bias_estimate=r.bias_estimate, bias_se=r.bias_se, tau=r.tau,
                levels_added=r.levels_added, device_planned=r.device_planned)


BATCHED_DIRECT, BATCHED_GRAPH, BATCHED_TIMED, BATCHED_PER_LEVEL = 0, 1, 2, -1


LEVELS_ALL, LEVELS_HEURISTIC, LEVELS_OPTIMAL, LEVELS_HEURISTIC_TAU = 0, 1, 2, 3


def options(batched=BATCHED_DIRECT, max_iter=0, n_warmup=0, block=0, ppt=0, waves_per_simd=0,
            tp_max_samples=0, level_select=LEVELS_ALL, L_max=0):
    """mlmc_ap_options: batched = 0 (direct persistent launch, default), 1 (hipGraph
    replay), 2 (direct, particle kernel timed), -1 (one launch per level);
    level_select = LEVELS_ALL (levels 0..L), LEVELS_HEURISTIC, LEVELS_OPTIMAL or
    LEVELS_HEURISTIC_TAU (warm-up of levels 0..tau, KD only); L_max > L: the
    finest level grows while the bias estimate exceeds tol/sqrt(2)."""
    return Options(batched=batched, max_iter=max_iter, n_warmup=n_warmup,
                   tuning=Tuning(block=block, ppt=ppt, waves_per_simd=waves_per_simd,
                                 tp_max_samples=tp_max_samples),
                   level_select=level_select, L_max=L_max)


# ---------------------------------------------------------------------------
# Entry points (same names as the C ABI).
# ---------------------------------------------------------------------------
def mlmc_ap_init():
    _check(lib().mlmc_ap_init(), "mlmc_ap_init")


def mlmc_ap_release():
    _check(lib().mlmc_ap_release(), "mlmc_ap_release")


def mlmc_ap_version():
    return lib().mlmc_ap_version().decode()


def mlmc_ap_status_str(status):
    return lib().mlmc_ap_status_str(int(status)).decode()


def mlmc_ap_last_error():
    return lib().mlmc_ap_last_error().decode()


def mlmc_ap_validate(p):
    """Returns the status code (0 = valid) without raising."""
    return lib().mlmc_ap_validate(ctypes.byref(as_problem(p)))


def mlmc_ap_level_constants(p, level):
    out = LevelInfo()
    _check(lib().mlmc_ap_level_constants(ctypes.byref(as_problem(p)), int(level),
                                         ctypes.byref(out)), "mlmc_ap_level_constants")
    return {k: getattr(out, k) for k, _ in LevelInfo._fields_}


def mlmc_ap_optimal_samples(V, C, tol):
    n = len(V)
    Va = (ctypes.c_double * n)(*V)
    Ca = (ctypes.c_double * n)(*C)
    Na = (ctypes.c_uint64 * n)()
    _check(lib().mlmc_ap_optimal_samples(Va, Ca, n, float(tol), Na), "mlmc_ap_optimal_samples")
    return [int(x) for x in Na]


def mlmc_ap_merge_stats(a, b):
    A = LevelStats(**a) if isinstance(a, dict) else a
    B = LevelStats(**b) if isinstance(b, dict) else b
    out = LevelStats()
    _check(lib().mlmc_ap_merge_stats(ctypes.byref(A), ctypes.byref(B), ctypes.byref(out)),
           "mlmc_ap_merge_stats")
    return stats_dict(out)


def mlmc_ap_simulate_level(p, level, sample_begin, n_samples, single=False, traj=None,
                           coll=None, hist=False, stream=None):
    """Statistics of samples [sample_begin, sample_begin + n_samples) of one
    level.  ``traj``/``coll``: optional device tensors (2 n_samples floats or
    doubles / int32) receiving final positions and collision counts.
    With ``hist=True`` returns (stats, histogram list) instead of stats."""
    P = as_problem(p)
    out = LevelStats()
    hbuf = None
    if hist:
        hbuf = (ctypes.c_uint64 * (3 * P.nbins + 4))()
    tp, cp = _dump_ptrs(P, n_samples, traj, coll)
    _check(lib().mlmc_ap_simulate_level(ctypes.byref(P), int(level), int(bool(single)),
                                        int(sample_begin), int(n_samples), ctypes.byref(out),
                                        tp, cp, hbuf, _stream(stream)),
           "mlmc_ap_simulate_level")
    if hist:
        return stats_dict(out), [int(x) for x in hbuf]
    return stats_dict(out)


NOALLOC_MAX_SAMPLES = 1 << 22


def mlmc_ap_simulate_level_noalloc(p, level, sample_begin, n_samples, single=False, traj=None,
                                   coll=None, hist=False, stream=None):
    """As mlmc_ap_simulate_level, through the allocation-free entry point (the
    library allocates nothing; at most NOALLOC_MAX_SAMPLES samples per call)."""
    P = as_problem(p)
    out = LevelStats()
    hbuf = None
    if hist:
        hbuf = (ctypes.c_uint64 * (3 * P.nbins + 4))()
    tp, cp = _dump_ptrs(P, n_samples, traj, coll)
    _check(lib().mlmc_ap_simulate_level_noalloc(ctypes.byref(P), int(level), int(bool(single)),
                                                int(sample_begin), int(n_samples),
                                                ctypes.byref(out), tp, cp, hbuf, _stream(stream)),
           "mlmc_ap_simulate_level_noalloc")
    if hist:
        return stats_dict(out), [int(x) for x in hbuf]
    return stats_dict(out)


def mlmc_ap_simulate_pair(p, level, coarse_level, sample_begin, n_samples, traj=None, coll=None,
                          hist=False, stream=None):
    """As mlmc_ap_simulate_level for the pair (level, coarse_level)."""
    P = as_problem(p)
    out = LevelStats()
    hbuf = None
    if hist:
        hbuf = (ctypes.c_uint64 * (3 * P.nbins + 4))()
    tp, cp = _dump_ptrs(P, n_samples, traj, coll)
    _check(lib().mlmc_ap_simulate_pair(ctypes.byref(P), int(level), int(coarse_level),
                                       int(sample_begin), int(n_samples), ctypes.byref(out),
                                       tp, cp, hbuf, _stream(stream)),
           "mlmc_ap_simulate_pair")
    if hist:
        return stats_dict(out), [int(x) for x in hbuf]
    return stats_dict(out)


def _doubles(v):
    v = [float(x) for x in v]
    return (ctypes.c_double * max(1, len(v)))(*v)


def mlmc_ap_select_levels_heuristic(V, Vdiff):
    """Selected levels (sorted list) from V_l and V_{l,l-1} (Vdiff[0] ignored)."""
    L = len(V) - 1
    m = ctypes.c_uint64()
    _check(lib().mlmc_ap_select_levels_heuristic(_doubles(V), _doubles(Vdiff), L, ctypes.byref(m)),
           "mlmc_ap_select_levels_heuristic")
    return [l for l in range(L + 1) if (m.value >> l) & 1]


def mlmc_ap_warmup_depth(p):
    """Warm-up depth tau of Section 5.3 for a problem."""
    t = ctypes.c_int32()
    _check(lib().mlmc_ap_warmup_depth(ctypes.byref(as_problem(p)), ctypes.byref(t)),
           "mlmc_ap_warmup_depth")
    return t.value


def mlmc_ap_extrapolate_variances(V, Vdiff, tau, M, L):
    """(V, Vdiff) of levels 0..L from the measured values of levels 0..tau."""
    vo = (ctypes.c_double * (L + 1))()
    vdo = (ctypes.c_double * (L + 1))()
    _check(lib().mlmc_ap_extrapolate_variances(_doubles(V), _doubles(Vdiff), int(tau), int(M),
                                               int(L), vo, vdo),
           "mlmc_ap_extrapolate_variances")
    return list(vo), list(vdo)


def mlmc_ap_select_levels_optimal(V, C, Vpair, Cpair):
    """(levels, cost) minimising eq. level_selection; Vpair/Cpair are
    (L+1) x (L+1) nested lists or arrays, entry [i][j] for i > j."""
    L = len(V) - 1
    flat = lambda a: [float(a[i][j]) for i in range(L + 1) for j in range(L + 1)]
    m = ctypes.c_uint64()
    c = ctypes.c_double()
    _check(lib().mlmc_ap_select_levels_optimal(_doubles(V), _doubles(C), _doubles(flat(Vpair)),
                                               _doubles(flat(Cpair)), L, ctypes.byref(m),
                                               ctypes.byref(c)),
           "mlmc_ap_select_levels_optimal")
    return [l for l in range(L + 1) if (m.value >> l) & 1], c.value


def mlmc_ap_estimate(p, rmse_tol, opt=None, hist=False, stream=None):
    """MLMC estimate of E[x_L(T)^2] to RMSE ``rmse_tol`` (dict).  With
    ``hist=True`` the dict also holds per-level histograms."""
    P = as_problem(p)
    res = Result()
    hbuf = None
    if hist:
        hbuf = (ctypes.c_uint64 * ((3 * P.nbins + 4) * (P.L + 1)))()
    _check(lib().mlmc_ap_estimate(ctypes.byref(P), float(rmse_tol),
                                  ctypes.byref(opt) if opt is not None else None,
                                  ctypes.byref(res), hbuf, _stream(stream)), "mlmc_ap_estimate")
    d = result_dict(res)
    if hist:
        w = 3 * P.nbins + 4
        d["hist"] = [[int(x) for x in hbuf[l * w:(l + 1) * w]] for l in range(P.L + 1)]
    return d


def mlmc_ap_estimate_into(P, rmse_tol, opt, res, stream=None):
    """mlmc_ap_estimate of a marshalled Problem into a caller-owned Result,
    without conversion (for loops that convert only what they keep, with
    result_dict); returns res."""
    _check(lib().mlmc_ap_estimate(ctypes.byref(P), float(rmse_tol),
                                  ctypes.byref(opt) if opt is not None else None,
                                  ctypes.byref(res), None, _stream(stream)), "mlmc_ap_estimate")
    return res


def mlmc_ap_estimate_sequence(p, rmse_tol0, R, opt=None, stream=None):
    """The estimate through the tolerances rmse_tol0 / sqrt(2^r), r = 0..R,
    continuing from the same samples: a list of R + 1 result dicts."""
    P = as_problem(p)
    res = (Result * max(int(R) + 1, 1))()
    _check(lib().mlmc_ap_estimate_sequence(ctypes.byref(P), float(rmse_tol0), int(R),
                                           ctypes.byref(opt) if opt is not None else None,
                                           res, _stream(stream)), "mlmc_ap_estimate_sequence")
    return [result_dict(r) for r in res]


def mlmc_ap_plain_mc(p, rmse_tol, opt=None, stream=None):
    P = as_problem(p)
    res = Result()
    _check(lib().mlmc_ap_plain_mc(ctypes.byref(P), float(rmse_tol),
                                  ctypes.byref(opt) if opt is not None else None,
                                  ctypes.byref(res), _stream(stream)), "mlmc_ap_plain_mc")
    return result_dict(res)


def mlmc_ap_estimate_batch(problems, rmse_tols, opt=None, stream=None):
    n = len(problems)
    Ps = (Problem * n)(*[as_problem(p) for p in problems])
    tols = (ctypes.c_double * n)(*[float(t) for t in rmse_tols])
    res = (Result * n)()
    _check(lib().mlmc_ap_estimate_batch(Ps, tols, n, ctypes.byref(opt) if opt is not None else None,
                                        res, _stream(stream)), "mlmc_ap_estimate_batch")
    return [result_dict(r) for r in res]


def mlmc_ap_autotune(p, rmse_tol, cache_path=None, stream=None):
    out = Tuning()
    _check(lib().mlmc_ap_autotune(ctypes.byref(as_problem(p)), float(rmse_tol),
                                  cache_path.encode() if cache_path else None, ctypes.byref(out),
                                  _stream(stream)), "mlmc_ap_autotune")
    return dict(block=out.block, ppt=out.ppt, waves_per_simd=out.waves_per_simd)


def mlmc_ap_set_tuning(block=0, ppt=0, waves_per_simd=0, tp_max_samples=0):
    """Default tuning of the current device; zero arguments keep the current
    value (tp_max_samples < 0 switches the time-parallel path off)."""
    t = Tuning(block=block, ppt=ppt, waves_per_simd=waves_per_simd, tp_max_samples=tp_max_samples)
    _check(lib().mlmc_ap_set_tuning(ctypes.byref(t)), "mlmc_ap_set_tuning")


def mlmc_ap_server_create(hbm_budget_bytes=0, max_samples_per_tick=0, max_active=0, opt=None):
    cfg = ServerConfig(hbm_budget_bytes=hbm_budget_bytes,
                       max_samples_per_tick=max_samples_per_tick, max_active=max_active,
                       reserved=0, options=opt if opt is not None else options())
    h = ctypes.c_void_p()
    _check(lib().mlmc_ap_server_create(ctypes.byref(cfg), ctypes.byref(h)), "mlmc_ap_server_create")
    return h


def mlmc_ap_server_destroy(srv):
    _check(lib().mlmc_ap_server_destroy(srv), "mlmc_ap_server_destroy")


def mlmc_ap_server_submit(srv, p, rmse_tol):
    t = ctypes.c_uint64()
    _check(lib().mlmc_ap_server_submit(srv, ctypes.byref(as_problem(p)), float(rmse_tol),
                                       ctypes.byref(t)), "mlmc_ap_server_submit")
    return int(t.value)


def mlmc_ap_server_step(srv):
    n = ctypes.c_int32()
    _check(lib().mlmc_ap_server_step(srv, ctypes.byref(n)), "mlmc_ap_server_step")
    return int(n.value)


def mlmc_ap_server_poll(srv, ticket):
    """The result dict, or None while the request is pending; raises for a
    cancelled or unknown ticket."""
    res = Result()
    st = lib().mlmc_ap_server_poll(srv, int(ticket), ctypes.byref(res))
    if st == -7:
        return None
    _check(st, "mlmc_ap_server_poll")
    return result_dict(res)


def mlmc_ap_server_cancel(srv, ticket):
    _check(lib().mlmc_ap_server_cancel(srv, int(ticket)), "mlmc_ap_server_cancel")


def mlmc_ap_server_get_stats(srv):
    out = ServerStats()
    _check(lib().mlmc_ap_server_get_stats(srv, ctypes.byref(out)), "mlmc_ap_server_get_stats")
    return {k: getattr(out, k) for k, _ in ServerStats._fields_}


def mlmc_ap_server_run_trace(srv, arrival_s, problems, rmse_tols):
    """Replays an arrival trace in real time; returns (latencies, results)."""
    n = len(arrival_s)
    arr = (ctypes.c_double * n)(*[float(a) for a in arrival_s])
    Ps = (Problem * n)(*[as_problem(p) for p in problems])
    tols = (ctypes.c_double * n)(*[float(t) for t in rmse_tols])
    res = (Result * n)()
    lat = (ctypes.c_double * n)()
    _check(lib().mlmc_ap_server_run_trace(srv, n, arr, Ps, tols, res, lat),
           "mlmc_ap_server_run_trace")
    return [float(x) for x in lat], [result_dict(r) for r in res]


def mlmc_ap_kd_coarse_numbers(p, level, coarse_level, sample_begin, n_samples, max_rows, rows,
                              counts, stream=None):
    """Coarse numbers of KD pairs into the device tensors ``rows`` (float64,
    n_samples * max_rows * 4: chi~, nu~, E~, fine steps aggregated per coarse
    KD step) and ``counts`` (int32/uint32, n_samples: coarse KD steps per
    pair)."""
    n, m = int(n_samples), int(max_rows)
    _check(lib().mlmc_ap_kd_coarse_numbers(
        ctypes.byref(as_problem(p)), int(level), int(coarse_level), int(sample_begin), n, m,
        _dev_ptr(rows, n * m * 4, ("float64",), "rows"),
        _dev_ptr(counts, n, ("int32", "uint32"), "counts"), _stream(stream)),
        "mlmc_ap_kd_coarse_numbers")


def mlmc_ap_philox_words(seed, stream_id, tag, sample_begin, n_samples, n_steps, out, stream=None):
    """Fills the device tensor ``out`` (n_samples * n_steps * 4 int32) with
    Philox4x32-10 words."""
    _check(lib().mlmc_ap_philox_words(int(seed), int(stream_id), int(tag), int(sample_begin),
                                      int(n_samples), int(n_steps),
                                      _dev_ptr(out, 4 * int(n_samples) * int(n_steps),
                                               ("int32", "uint32"), "out"), _stream(stream)),
           "mlmc_ap_philox_words")


def mlmc_ap_rng_normals(seed, stream_id, tag, sample_begin, n_samples, n_steps, fp64, out,
                        stream=None):
    _check(lib().mlmc_ap_rng_normals(int(seed), int(stream_id), int(tag), int(sample_begin),
                                     int(n_samples), int(n_steps), int(fp64),
                                     _dev_ptr(out, 4 * int(n_samples) * int(n_steps),
                                              ("float64",) if fp64 else ("float32",), "out"),
                                     _stream(stream)), "mlmc_ap_rng_normals")
