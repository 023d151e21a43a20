"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bars:
  * Philox words, uniforms, collision decisions and counts: bit-exact;
  * FP32 positions: |x_gpu - x_oracle| <= 1e-5 max(|x_oracle|, rms(x_oracle));
    FP64 positions: 1e-12 relative to the same scale;
  * statistics: the device reduction against two-pass FP64 statistics of the
    oracle's trajectories;
  * estimates: equal to the oracle's estimate on the same samples within the
    FP32 rounding bound, and within 4 standard errors of the exact E[Q_L].
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import closed_form as CF
from oracle import mlmc as OM

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2004_04071_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    pkg.mlmc_ap_init()
    yield


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def two_pass(xf, xc, level, single=False):
    return OM.stats_of(xf, xc, 0 if single else level)


def run_level(prob, level, n, begin=0, single=False):
    """GPU dump and statistics of one level, with the oracle's values."""
    P = pkg.as_problem(prob)
    dt = torch.float64 if P.fp64_state else torch.float32
    traj = torch.full((2 * n,), float("nan"), dtype=dt, device="cuda")
    coll = torch.full((2 * n,), -1, dtype=torch.int32, device="cuda")
    st = pkg.mlmc_ap_simulate_level(P, level, begin, n, single=single, traj=traj, coll=coll)
    torch.cuda.synchronize()
    ref = O.simulate(prob, level, begin, n, single=single)
    x = traj.cpu().double().numpy()
    c = coll.cpu().numpy().astype(np.int64)
    return st, x[:n], x[n:], c[:n], c[n:], ref


def check_trajectories(prob, level, n, begin=0, single=False, rel=None):
    st, xf, xc, cf, cc, ref = run_level(prob, level, n, begin, single)
    fp64 = bool(prob.get("fp64_state", 0))
    if rel is None:
        rel = 1e-12 if fp64 else 1e-5
    coarse = level >= 1 and not single
    assert np.array_equal(cf, ref["cf"].astype(np.int64)), "fine collision counts differ"
    assert np.array_equal(cc, ref["cc"].astype(np.int64)), "coarse collision counts differ"
    scale_f = np.maximum(np.abs(ref["xf"]), math.sqrt(np.mean(ref["xf"] ** 2)))
    err_f = np.max(np.abs(xf - ref["xf"]) / scale_f)
    err_c = 0.0
    if coarse:
        scale_c = np.maximum(np.abs(ref["xc"]), math.sqrt(np.mean(ref["xc"] ** 2)))
        err_c = np.max(np.abs(xc - ref["xc"]) / scale_c)
    else:
        assert np.all(xc == 0.0)
    say("level %d n %d: max scaled error fine %.3e coarse %.3e" % (level, n, err_f, err_c))
    assert err_f <= rel and err_c <= rel
    # device statistics against two-pass statistics of the device's own dump
    dev = two_pass(xf, xc, level, single)
    assert st["n"] == n
    assert st["coll_f"] == int(cf.sum()) and st["coll_c"] == int(cc.sum())
    sd = math.sqrt(dev["m2_dq"] / max(n - 1, 1)) + 1e-300
    assert abs(st["mean_dq"] - dev["mean_dq"]) <= 1e-12 * (abs(dev["mean_dq"]) + sd)
    assert st["m2_dq"] == pytest.approx(dev["m2_dq"], rel=1e-9, abs=1e-18)
    if coarse:
        for k in ("mean_qf", "mean_qc"):
            assert st[k] == pytest.approx(dev[k], rel=1e-12, abs=1e-14)
        for k in ("m2_qf", "m2_qc", "c_fc"):
            assert st[k] == pytest.approx(dev[k], rel=1e-9, abs=1e-12)
    return st, ref


# ---------------------------------------------------------------------------
# Random number path
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed,stream_id,tag,begin", [
    (42, 0, 0, 0), (42, 7, 8, 1000), (2 ** 63 + 5, 1234, 72, 2 ** 32 - 300),
    (0xDEADBEEFCAFEF00D, 2 ** 32 - 1, 30, 12345)])
def test_philox_words_bit_exact(seed, stream_id, tag, begin):
    ns, nt = 300, 7
    out = torch.zeros(ns * nt * 4, dtype=torch.int32, device="cuda")
    pkg.mlmc_ap_philox_words(seed, stream_id, tag, begin, ns, nt, out)
    got = out.cpu().numpy().view(np.uint32).reshape(ns, nt, 4)
    ref = O.words(seed, stream_id, tag, begin, ns, nt)
    assert np.array_equal(got, ref)


def test_uniforms_and_normals():
    ns, nt = 2000, 16
    out32 = torch.zeros(ns * nt * 4, dtype=torch.float32, device="cuda")
    out64 = torch.zeros(ns * nt * 4, dtype=torch.float64, device="cuda")
    pkg.mlmc_ap_rng_normals(42, 3, 5, 0, ns, nt, 0, out32)
    pkg.mlmc_ap_rng_normals(42, 3, 5, 0, ns, nt, 1, out64)
    g32 = out32.cpu().double().numpy().reshape(-1, 4)
    g64 = out64.cpu().numpy().reshape(-1, 4)
    w = O.words(42, 3, 5, 0, ns, nt).reshape(-1, 4)
    u1 = (2.0 * (w[:, 1] >> 9).astype(np.float64) + 1.0) * 2.0 ** -24
    u2 = (2.0 * (w[:, 2] >> 9).astype(np.float64) + 1.0) * 2.0 ** -24
    for u, col in ((u1, 0), (u2, 1)):
        assert np.array_equal(g32[:, col], u) and np.array_equal(g64[:, col], u)
    r = np.sqrt(-2.0 * np.log(u1))
    xi = r * np.cos(2 * np.pi * u2)
    g = r * np.sin(2 * np.pi * u2)
    e32 = max(np.max(np.abs(g32[:, 2] - xi)), np.max(np.abs(g32[:, 3] - g)))
    e64 = max(np.max(np.abs(g64[:, 2] - xi)), np.max(np.abs(g64[:, 3] - g)))
    say("normals: max abs error FP32 %.3e, FP64 %.3e" % (e32, e64))
    assert e64 <= 1e-13
    assert e32 <= 1e-5


# ---------------------------------------------------------------------------
# Trajectories, collision counts and tile statistics
# ---------------------------------------------------------------------------
CASES = {
    "cfg1_fp64": (W.cfg1(), 0, 1000, 0, False),
    "cfg1_fp32": (dict(W.cfg1(), fp64_state=0), 0, 1000, 0, False),
    "cfg2_l0": (W.cfg2(), 0, 777, 0, False),
    "cfg2_l1": (W.cfg2(), 1, 1000, 0, False),
    "cfg2_l4": (W.cfg2(), 4, 600, 0, False),
    "cfg2_l8": (W.cfg2(), 8, 300, 0, False),
    "cfg2_l3_kick_sum": (W.cfg2(coupling=0), 3, 513, 0, False),
    "cfg2_l5_offset": (W.cfg2(), 5, 400, 123456789, False),
    "cfg2_single_l3": (W.cfg2(), 3, 500, 0, True),
    "eps0_l4": (W.cfg2(eps=0.0), 4, 500, 0, False),
    "eps1e-4_l6": (W.cfg2(eps=1e-4), 6, 300, 0, False),
    "eps1_l6": (W.cfg2(eps=1.0), 6, 300, 0, False),
    "free_streaming_wide": (W.cfg2(eps=1e6), 3, 300, 0, False),
    "twopoint_M4_l2": (dict(W.cfg1(), fp64_state=0, M=4, L=3, T=0.5, dt0=0.05), 2, 700, 0, False),
    "maxwell_M4_agg_l2": (dict(W.cfg2(eps=0.05), M=4, L=3), 2, 700, 0, False),
    "cfg4_cos_l2_fp32": (dict(W.cfg4(0), qoi=0), 2, 900, 0, False),
    "cfg4_cos_l2_fp64": (dict(W.cfg4(1), qoi=0), 2, 900, 0, False),
    "cfg2_fp64_l3": (dict(W.cfg2(), fp64_state=1), 3, 500, 0, False),
    # M = 3: coarse blocks at run-time positions, groups of four steps with a tail
    "maxwell_M3_agg_l2": (dict(W.cfg2(eps=0.05), M=3, L=3, T=1.5, dt0=0.5), 2, 600, 7, False),
    "twopoint_M3_l2": (dict(W.cfg1(), fp64_state=0, M=3, L=3, T=0.3, dt0=0.1), 2, 600, 0, False),
    "maxwell_M3_single_l3": (dict(W.cfg2(eps=0.3), M=3, L=3, T=1.5, dt0=0.5), 3, 300, 0, True),
    # an odd step count at level 0 (tail of three steps, then 6 and 12 at levels 1, 2)
    "maxwell_n0_3_l1": (dict(W.cfg2(eps=0.2), T=1.5, dt0=0.5), 1, 600, 0, False),
}


@pytest.mark.parametrize("case", list(CASES), ids=list(CASES))
def test_trajectory_parity(case):
    prob, level, n, begin, single = CASES[case]
    say("case", case)
    check_trajectories(prob, level, n, begin, single)


def test_wide_thresholds_used():
    c = pkg.mlmc_ap_level_constants(pkg.as_problem(W.cfg2(eps=1e6)), 3)
    assert c["thr_f"] == 0


@pytest.mark.parametrize("level,n", [(0, 1), (0, 63), (0, 65), (0, 1024 * 1024 - 1),
                                     (0, 1024 * 1024 + 1), (0, 1025 * 1024 + 3),
                                     (0, 2048 * 1024 + 7), (1, 1024 * 1024 + 5),
                                     (4, 1024 * 256 + 255), (5, 63), (5, 65), (5, 256 * 64),
                                     (5, 256 * 64 + 1), (5, 1025 * 64 + 3)])
def test_tile_and_group_boundaries(level, n):
    """Ragged tiles of every width (2048 samples below 4 fine steps, 1024 below
    16, 256 below 64, 64 from there on; an item of fewer than 1024 such tiles
    takes a quarter of the width, repeatedly: 512-sample tiles for level 0
    near 2^20 samples), one full 256-tile reduction group, and more than one
    group."""
    prob = W.cfg2(eps=0.3)
    st = pkg.mlmc_ap_simulate_level(prob, level, 5, n)
    ref = O.simulate(prob, level, 5, n)
    r = two_pass(ref["xf"], ref["xc"], level)
    assert st["n"] == n and st["coll_f"] == int(ref["cf"].astype(np.int64).sum())
    assert st["coll_c"] == int(ref["cc"].astype(np.int64).sum())
    sd = math.sqrt(r["m2_dq"] / max(n - 1, 1))
    assert abs(st["mean_dq"] - r["mean_dq"]) <= 2e-6 * (abs(r["mean_dq"]) + sd + abs(r["mean_qf"]))
    if n > 1:
        assert st["m2_dq"] == pytest.approx(r["m2_dq"], rel=1e-5)


def test_zero_samples():
    st = pkg.mlmc_ap_simulate_level(W.cfg2(), 2, 0, 0)
    assert st["n"] == 0


def test_split_ranges_merge():
    """Statistics of [0,a) merged with [a,n) equal those of [0,n) to rounding."""
    prob = W.cfg2(eps=0.1)
    a, n = 3000, 10000
    s1 = pkg.mlmc_ap_simulate_level(prob, 3, 0, a)
    s2 = pkg.mlmc_ap_simulate_level(prob, 3, a, n - a)
    s = pkg.mlmc_ap_simulate_level(prob, 3, 0, n)
    m = pkg.mlmc_ap_merge_stats(s1, s2)
    assert m["n"] == s["n"] and m["coll_f"] == s["coll_f"] and m["coll_c"] == s["coll_c"]
    for k in ("mean_dq", "mean_qf", "mean_qc"):
        assert m[k] == pytest.approx(s[k], rel=1e-12, abs=1e-15)
    for k in ("m2_dq", "m2_qf", "m2_qc", "c_fc"):
        assert m[k] == pytest.approx(s[k], rel=1e-10)


# ---------------------------------------------------------------------------
# Histogram (precision study)
# ---------------------------------------------------------------------------
def oracle_hist(x, lo, hi, nb):
    t = (x - lo) * (nb / (hi - lo))
    b = np.floor(t).astype(np.int64)
    return b


@pytest.mark.parametrize("fp64", [0, 1])
def test_histogram_counts(fp64):
    prob = W.cfg4(fp64)
    level, n = 3, 20000
    st, h = pkg.mlmc_ap_simulate_level(prob, level, 0, n, hist=True)
    ref = O.simulate(prob, level, 0, n)
    nb = 64
    bf = oracle_hist(ref["xf"], -4.0, 5.0, nb)
    bc = oracle_hist(ref["xc"], -4.0, 5.0, nb)
    h = np.array(h, dtype=np.int64)
    assert h[:3 * nb:3].sum() + h[3 * nb] + h[3 * nb + 1] == n
    assert h[1:3 * nb:3].sum() + h[3 * nb + 2] + h[3 * nb + 3] == n
    for b in range(nb):
        assert abs(h[3 * b] - np.sum(bf == b)) <= 2
        assert abs(h[3 * b + 1] - np.sum(bc == b)) <= 2
        assert abs(h[3 * b + 2] - np.sum((bf == b) & (bc == b))) <= 2


# ---------------------------------------------------------------------------
# Estimates: launch modes, tunings, graph replays, batching
# ---------------------------------------------------------------------------
def _key(r):
    return (r["estimate"], r["var_estimator"], tuple(r["N"]),
            tuple(tuple(sorted(l.items())) for l in r["levels"]))


def test_estimate_bitwise_across_modes_and_tunings():
    prob = W.cfg2(eps=0.05)
    base = pkg.mlmc_ap_estimate(prob, 1e-2, pkg.options(batched=1))
    say("estimate", base["estimate"], "N", base["N"])
    for opt in (pkg.options(batched=-1), pkg.options(batched=2), pkg.options(batched=0),
                pkg.options(batched=3),
                pkg.options(batched=1, block=64, ppt=1, waves_per_simd=2),
                pkg.options(batched=2, block=128, ppt=2, waves_per_simd=8),
                pkg.options(batched=-1, block=256, ppt=1)):
        r = pkg.mlmc_ap_estimate(prob, 1e-2, opt)
        assert _key(r) == _key(base)


# Level 0 in tiles of 1, 2, 8 and 32 samples per lane and level 1 in tiles
# of 4 and 16 (the item's size picks the width): every particles-per-thread
# shape runs each sample once, with the statistics of one trajectory per lane.
@pytest.mark.parametrize("level,n", [(0, 100_000), (0, 300_000), (0, 1_000_000),
                                     (0, 3_000_000), (1, 500_000), (1, 2_000_000)])
def test_particles_per_thread_on_every_tile_width(level, n):
    prob = W.cfg2(eps=0.05, stream_id=62)
    ref = None
    try:
        for ppt in (1, 2, 4):
            pkg.mlmc_ap_set_tuning(ppt=ppt)
            st = pkg.mlmc_ap_simulate_level(prob, level, 0, n)
            torch.cuda.synchronize()
            say("level", level, "n", n, "ppt", ppt, "mean dQ", st["mean_dq"])
            assert st["n"] == n
            if ref is None:
                ref = st
            else:
                assert st == ref, (ppt, st, ref)
    finally:
        pkg.mlmc_ap_set_tuning(ppt=1)


# Every launch shape the tuning accepts, on the three particle kernels (FP32
# and FP64 splitting, KD with its time-parallel warm-up): the same estimate,
# bit for bit, as the default shape.
SHAPES = [(64, 1, 1), (64, 4, 2), (128, 2, 4), (128, 4, 8), (256, 2, 1), (256, 4, 8)]


@pytest.mark.parametrize("name,prob,tol,extra", [
    ("fp32", W.cfg2(eps=0.05, stream_id=63), 5e-3, {}),
    ("fp64", dict(W.cfg2(eps=0.05, stream_id=64), fp64_state=1), 5e-3, {}),
    ("kd", W.cfg_kd(eps=0.01, stream_id=65), 5e-3, {}),
    ("fp32_heuristic_levels", W.cfg2(eps=0.01, stream_id=66), 3e-3,
     dict(level_select=pkg.LEVELS_HEURISTIC)),
    ("kd_b1", W.cfg_bg(W.BG_B1, 10.0, 1000.0, L=8, stream_id=67), 1e-3, {}),
], ids=["fp32", "fp64", "kd", "fp32_heuristic_levels", "kd_b1"])
def test_estimate_bitwise_across_launch_shapes(name, prob, tol, extra):
    base = pkg.mlmc_ap_estimate(prob, tol, pkg.options(batched=0, block=256, ppt=1,
                                                       waves_per_simd=8, **extra))
    say(name, "estimate", base["estimate"], "N", base["N"])
    for b, p, w in SHAPES:
        for batched in (0, -1):
            r = pkg.mlmc_ap_estimate(prob, tol, pkg.options(batched=batched, block=b, ppt=p,
                                                            waves_per_simd=w, **extra))
            assert _key(r) == _key(base), (name, b, p, w, batched)


def test_graph_replays_match_eager():
    prob = W.cfg2(eps=0.2, stream_id=9)
    eager = pkg.mlmc_ap_estimate(prob, 5e-3, pkg.options(batched=2))
    for _ in range(3):
        _ = torch.randn(1000, device="cuda").sum().item()  # unrelated eager work in between
        r = pkg.mlmc_ap_estimate(prob, 5e-3, pkg.options(batched=1))
        assert _key(r) == _key(eager)


def test_estimate_batch_equals_alone():
    probs = [W.cfg2(eps=e, stream_id=20 + i) for i, e in enumerate((1e-3, 0.05, 1.0))]
    tols = [1e-2, 5e-3, 1e-2]
    batch = pkg.mlmc_ap_estimate_batch(probs, tols)
    for p, t, b in zip(probs, tols, batch):
        alone = pkg.mlmc_ap_estimate(p, t)
        assert _key(alone) == _key(b)


def test_estimate_matches_oracle_and_closed_form():
    prob = W.cfg2(eps=0.05, stream_id=31)
    L = prob["L"]
    res = pkg.mlmc_ap_estimate(prob, 5e-3)
    assert res["converged"] and res["var_estimator"] <= 0.5 * 5e-3 ** 2
    exact = CF.level_second_moment(prob, L)
    assert abs(res["estimate"] - exact) <= 4.0 * math.sqrt(res["var_estimator"])
    est, levels = OM.estimate_fixed(prob, res["N"])
    say("gpu %.9f oracle %.9f exact %.9f sd %.2e" % (res["estimate"], est, exact,
                                                      math.sqrt(res["var_estimator"])))
    assert abs(res["estimate"] - est) <= 2e-5 * abs(exact)
    for l in range(L + 1):
        g, o = res["levels"][l], levels[l]
        assert g["n"] == o["n"]
        assert g["coll_f"] == o["coll_f"] and g["coll_c"] == o["coll_c"]
        assert g["m2_dq"] == pytest.approx(o["m2_dq"], rel=1e-3)


def test_single_level_hierarchy_estimate():
    """L = 0: the hierarchy is level 0 alone, the sum of eqs. Nopt1/Noptj has
    one term, and N_0 = ceil(2/tol^2 V_0) from the warm-up's variance; the
    device-planned and host-planned forms agree bit for bit, and the estimate
    is within 4 standard errors of the exact E[Q_0]."""
    prob = dict(W.cfg2(eps=0.05, stream_id=68), L=0)
    tol = 5e-3
    dev = pkg.mlmc_ap_estimate(prob, tol, pkg.options(batched=0))
    host = pkg.mlmc_ap_estimate(prob, tol, pkg.options(batched=3))
    assert _key(dev) == _key(host)
    assert dev["device_planned"] >= 1 and len(dev["N"]) == 1 and dev["converged"]
    exact = CF.level_second_moment(prob, 0)
    say("L=0: N %s estimate %.8f exact %.8f sd %.2e" % (dev["N"], dev["estimate"], exact,
                                                        math.sqrt(dev["var_estimator"])))
    assert abs(dev["estimate"] - exact) <= 4.0 * math.sqrt(dev["var_estimator"])
    assert dev["var_estimator"] <= 0.5 * tol ** 2 * (1.0 + 1e-12)


def test_estimate_with_warm_up_enough():
    """A tolerance the warm-up already meets: the device-planned top-up has no
    work (an empty table through the particle and reduction kernels), and the
    result is the warm-up's, as when the host plans."""
    prob = W.cfg2(eps=0.05, stream_id=69)
    dev = pkg.mlmc_ap_estimate(prob, 1.0, pkg.options(batched=0))
    host = pkg.mlmc_ap_estimate(prob, 1.0, pkg.options(batched=3))
    assert _key(dev) == _key(host)
    assert all(n == 1000 for n in dev["N"]) and dev["converged"]


def test_plain_mc_estimate():
    prob = W.cfg2(eps=0.1, stream_id=41)
    res = pkg.mlmc_ap_plain_mc(prob, 1e-2)
    L = prob["L"]
    assert res["N"][:L] == [0] * L and res["N"][L] > 0
    exact = CF.level_second_moment(prob, L)
    assert abs(res["estimate"] - exact) <= 4.0 * math.sqrt(res["var_estimator"])


def test_concurrent_calls_on_distinct_streams():
    """Host threads calling the library at once, each on its own stream
    (ctypes releases the interpreter lock during a call): every result equals
    the same call made alone, bitwise."""
    import threading
    probs = [W.cfg2(eps=e, stream_id=70 + i) for i, e in enumerate((0.01, 0.05, 0.2, 1.0))]
    alone = [pkg.mlmc_ap_estimate(p, 5e-3) for p in probs]
    streams = [torch.cuda.Stream() for _ in probs]
    out = [None] * len(probs)
    errors = []

    def work(i):
        try:
            with torch.cuda.stream(streams[i]):
                out[i] = pkg.mlmc_ap_estimate(probs[i], 5e-3,
                                              stream=streams[i].cuda_stream)
        except Exception as e:  # reported below
            errors.append(e)

    threads = [threading.Thread(target=work, args=(i,)) for i in range(len(probs))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    torch.cuda.synchronize()
    assert not errors, errors
    for a, b in zip(alone, out):
        assert _key(a) == _key(b)


# ---------------------------------------------------------------------------
# Device-planned top-up: after the warm-up of a lone request in a direct
# launch, the device computes eqs. Nopt1/Noptj and the top-up's table and
# launches it behind the warm-up; the host checks the numbers (an error if
# they differ).  Results are those of the host-planned forms, bit for bit.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,prob,tol,plain", [
    ("cfg2_eps0.05", W.cfg2(eps=0.05, stream_id=41), 5e-3, False),
    ("cfg2_eps1e-4", W.cfg2(eps=1e-4, stream_id=42), 1e-2, False),
    ("plain_mc_eps0.3", W.cfg2(eps=0.3, stream_id=43), 2e-2, True),
    ("kd_eps0.05", W.cfg_kd(eps=0.05, stream_id=44), 1e-2, False),
    ("bg_b2_L5", dict(W.cfg_bg(W.BG_B2, 10.0, 100.0, stream_id=45), L=5), 5e-3, False),
], ids=lambda v: v if isinstance(v, str) else "")
def test_device_planned_top_up_equals_host_planned(name, prob, tol, plain):
    say("case", name)
    fn = pkg.mlmc_ap_plain_mc if plain else pkg.mlmc_ap_estimate
    host = fn(prob, tol, pkg.options(batched=-1))
    for batched in (0, 2):
        dev = fn(prob, tol, pkg.options(batched=batched))
        assert dev["device_planned"] == 1, (batched, dev["launches"])
        assert _key(dev) == _key(host)
        assert dev["launches"] == host["launches"]
        assert dev["particle_steps"] == host["particle_steps"]
    assert host["device_planned"] == 0
    for batched in (1, 3):  # graph replays; direct launches planned by the host
        r = fn(prob, tol, pkg.options(batched=batched))
        assert r["device_planned"] == 0 and _key(r) == _key(host)


def test_device_planned_top_up_declined_when_too_large():
    """A first top-up of more tile records than the buffers hold (about 3.5e6
    tiles at level 0 here) is not launched by the device: the host plans it,
    with the same results as the per-level form."""
    prob = dict(W.cfg2(eps=0.01, stream_id=46), L=2)
    dev = pkg.mlmc_ap_estimate(prob, 1e-4, pkg.options(batched=0))
    host = pkg.mlmc_ap_estimate(prob, 1e-4, pkg.options(batched=-1))
    say("N", dev["N"], "device_planned", dev["device_planned"])
    assert dev["N"][0] > 2 ** 31
    assert dev["device_planned"] == 0
    assert _key(dev) == _key(host)
