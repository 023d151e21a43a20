"""GPU parity of the kinetic-diffusion (KD) scheme against the FP64 oracle,
through the C ABI.

Bars (derivation in the design notes):
  * KD step counts (collisions before T), fine and coarse: bit-exact;
  * positions (FP64 state): |x_gpu - x_oracle| <= 1e-12 max(|x_oracle|,
    rms(x_oracle)) -- both sides take the same FP64 operations, and differ only
    by the last-bit differences of exp, log, sin/cos and sqrt between the two
    math libraries, a few units of 1e-16 per KD step over at most a few
    hundred steps (measured: at most 2.5e-14);
  * statistics: the device reduction against two-pass FP64 statistics of the
    device's own dump;
  * estimates: within 4.5 standard errors of the exact E[x(T)^2], which the
    KD construction keeps at every time step in a homogeneous background.
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

REL = 1e-12


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


def kd(eps, T=1.0, dt0=0.5, M=2, L=8, x0_kind=W.X0_NORMAL, stream_id=500, **kw):
    p = dict(eps=eps, T=T, dt0=dt0, M=M, L=L, x0_kind=x0_kind, x0_a=0.0, x0_b=1.0,
             eq_kind=W.EQ_MAXWELLIAN, coupling=W.COUPLING_AGGREGATE, fp64_state=1, seed=42,
             stream_id=stream_id, scheme=W.SCHEME_KD)
    p.update(kw)
    return p


def run_level(prob, level, n, begin=0, single=False, samples=None):
    P = pkg.as_problem(prob)
    traj = torch.full((2 * n,), float("nan"), dtype=torch.float64, device="cuda")
    coll = torch.full((2 * n,), -1, dtype=torch.int32, device="cuda")
    hist = prob.get("qoi", 0) == pkg.QOI_X2_HIST
    out = pkg.mlmc_ap_simulate_level(P, level, begin, n, single=single, traj=traj, coll=coll,
                                     hist=hist)
    torch.cuda.synchronize()
    st = out[0] if hist else out
    x = traj.cpu().numpy()
    c = coll.cpu().numpy().astype(np.int64)
    return st, x[:n], x[n:], c[:n], c[n:]


def scaled_error(got, want):
    scale = np.maximum(np.abs(want), math.sqrt(np.mean(want ** 2)))
    return float(np.max(np.abs(got - want) / scale))


CASES = [
    # name, problem, level, begin, n, single
    ("l0_ragged", kd(0.3, stream_id=501), 0, 5, 1000, False),
    ("pair_l3_ragged", kd(0.3, stream_id=502), 3, 17, 3001, False),
    ("pair_kinetic_eps1_l2", kd(1.0, stream_id=503), 2, 0, 2000, False),
    ("pair_diffusive_eps0.01_l4", kd(0.01, stream_id=504), 4, 0, 1500, False),
    ("single_l5", kd(0.1, stream_id=505), 5, 3, 700, True),
    ("pair_M3", kd(0.2, T=1.5, M=3, stream_id=506), 2, 0, 1200, False),
    ("pair_M4", kd(0.1, M=4, stream_id=507), 2, 9, 1000, False),
    ("pair_free_streaming_eps5", kd(5.0, x0_kind=W.X0_DELTA, stream_id=508), 2, 0, 1000, False),
    ("pair_cosine_x0_hist", kd(0.05, x0_kind=W.X0_COSINE, stream_id=509, qoi=1, nbins=64,
                               hist_lo=-4.0, hist_hi=5.0), 3, 0, 1000, False),
    ("pair_last_samples", kd(0.2, stream_id=510), 2, 2 ** 32 - 777, 777, False),
    ("one_sample", kd(0.2, stream_id=511), 1, 0, 1, False),
    ("pair_wide_tiles_l1", kd(0.3, stream_id=512), 1, 0, 70001, False),
]


@pytest.mark.parametrize("name,prob,level,begin,n,single", CASES, ids=[c[0] for c in CASES])
def test_kd_trajectories_match_oracle(name, prob, level, begin, n, single):
    say("case", name)
    st, xf, xc, cf, cc = run_level(prob, level, n, begin, single)
    ref = O.simulate(prob, level, begin, n, single=single)
    assert np.array_equal(cf, ref["cf"].astype(np.int64)), "fine KD step counts differ"
    assert np.array_equal(cc, ref["cc"].astype(np.int64)), "coarse KD step counts differ"
    coarse = level >= 1 and not single
    ef = scaled_error(xf, ref["xf"])
    ec = scaled_error(xc, ref["xc"]) if coarse else 0.0
    say("  max scaled error fine %.3e coarse %.3e" % (ef, ec))
    assert ef <= REL and ec <= REL
    if not coarse:
        assert np.all(xc == 0.0)
    dev = OM.stats_of(xf, xc, 0 if single else level)
    assert st["n"] == n
    assert st["coll_f"] == int(cf.sum()) and st["coll_c"] == int(cc.sum())
    sd = math.sqrt(dev["m2_dq"] / max(n - 1, 1)) + 1e-300
    assert abs(st["mean_dq"] - dev["mean_dq"]) <= 1e-12 * (abs(dev["mean_dq"]) + sd)
    assert st["m2_dq"] == pytest.approx(dev["m2_dq"], rel=1e-9, abs=1e-18)
    if coarse:
        for k in ("m2_qf", "m2_qc", "c_fc"):
            assert st[k] == pytest.approx(dev[k], rel=1e-9, abs=1e-12)


def test_kd_histogram_counts_exact():
    prob = kd(0.05, x0_kind=W.X0_COSINE, stream_id=520, qoi=1, nbins=64, hist_lo=-4.0,
              hist_hi=5.0)
    P = pkg.as_problem(prob)
    st, hist = pkg.mlmc_ap_simulate_level(P, 2, 0, 5000, hist=True)
    ref = O.simulate(prob, 2, 0, 5000)
    edges = -4.0 + 9.0 / 64.0 * np.arange(65)
    for col, x in ((0, ref["xf"]), (1, ref["xc"])):
        counts, _ = np.histogram(x, bins=edges)
        got = np.asarray(hist[: 3 * 64]).reshape(64, 3)[:, col]
        # a position within rounding of a bin edge may fall either way
        assert np.abs(got.astype(np.int64) - counts).sum() <= 2


def test_kd_full_size_sampled():
    """Level 8 of the KD workload at a launch of 2e5 samples: 300 sampled
    trajectories against the oracle, one by one."""
    prob = W.cfg_kd()
    n = 200000
    st, xf, xc, cf, cc = run_level(prob, 8, n)
    idx = np.random.default_rng(3).choice(n, 300, replace=False)
    ref = O.simulate(prob, 8, samples=idx)
    assert np.array_equal(cf[idx], ref["cf"].astype(np.int64))
    assert np.array_equal(cc[idx], ref["cc"].astype(np.int64))
    assert scaled_error(xf[idx], ref["xf"]) <= REL
    assert scaled_error(xc[idx], ref["xc"]) <= REL
    assert st["n"] == n and not np.isnan(xf).any()


def key(r):
    return (r["estimate"], r["var_estimator"], tuple(r["N"]),
            tuple(tuple(sorted(l.items())) for l in r["levels"]))


@pytest.mark.parametrize("batched", [-1, 0, 1, 2])
def test_kd_estimate_exact_and_mode_independent(batched):
    """A KD MLMC estimate hits the exact E[x(T)^2] and is bitwise the same in
    every launch mode."""
    prob = kd(0.1, L=5, stream_id=530)
    r = pkg.mlmc_ap_estimate(prob, 5e-3, pkg.options(batched=batched))
    exact = CF.kinetic_limit(0.1, 1.0, 1.0)
    say("batched %d estimate %.6f exact %.6f sd %.2e N %s" % (
        batched, r["estimate"], exact, math.sqrt(r["var_estimator"]), r["N"]))
    assert r["converged"]
    assert abs(r["estimate"] - exact) <= 4.5 * math.sqrt(r["var_estimator"])
    ref = pkg.mlmc_ap_estimate(prob, 5e-3, pkg.options(batched=0))
    assert key(r) == key(ref)


def test_kd_estimate_matches_oracle_on_same_samples():
    """The per-level means of a GPU estimate against the oracle's on the same
    sample ranges."""
    prob = kd(0.3, L=3, stream_id=531)
    r = pkg.mlmc_ap_estimate(prob, 2e-2)
    est, levels = OM.estimate_fixed(prob, r["N"])
    for got, want in zip(r["levels"], levels):
        sd = math.sqrt(want["m2_dq"] / max(want["n"] - 1, 1))
        assert got["n"] == want["n"]
        assert abs(got["mean_dq"] - want["mean_dq"]) <= 1e-10 * (abs(want["mean_dq"]) + sd)
        assert got["coll_f"] == want["coll_f"] and got["coll_c"] == want["coll_c"]
    assert abs(r["estimate"] - est) <= 1e-10 * (abs(est) + 1.0)


def test_kd_batch_equals_single_requests():
    probs = [kd(e, L=4, stream_id=540 + i) for i, e in enumerate((0.05, 0.3, 1.0))]
    tols = [1e-2, 2e-2, 3e-2]
    batch = pkg.mlmc_ap_estimate_batch(probs, tols)
    for p, t, b in zip(probs, tols, batch):
        assert key(b) == key(pkg.mlmc_ap_estimate(p, t))


def test_kd_rejects_mixed_batches():
    with pytest.raises(pkg.MlmcApError):
        pkg.mlmc_ap_estimate_batch([kd(0.1, L=2), dict(kd(0.1, L=2), scheme=0)], [1e-2, 1e-2])


def test_kd_bench_workload_full_size_against_oracle():
    """The KD estimate the benchmark times (eps = 0.01, L = 8, RMSE 1e-3, FP64
    state; direct persistent launches timed by HIP events, block 256, 8 waves
    per SIMD), at its full sample numbers: every level's fine and coarse KD
    step totals equal the oracle's exactly, and the level means and the
    estimate agree to FP64 rounding."""
    prob = W.cfg_kd()
    r = pkg.mlmc_ap_estimate(prob, 1e-3, pkg.options(batched=2, block=256, ppt=1,
                                                     waves_per_simd=8))
    say("KD bench workload: N %s estimate %.9f" % (r["N"], r["estimate"]))
    assert r["converged"]
    est, levels = OM.estimate_fixed(prob, r["N"])
    for l, (g, o) in enumerate(zip(r["levels"], levels)):
        say("  level %d n %d steps %d/%d mean dq %.12e oracle %.12e" % (
            l, g["n"], g["coll_f"], g["coll_c"], g["mean_dq"], o["mean_dq"]))
        assert g["n"] == o["n"]
        assert g["coll_f"] == o["coll_f"] and g["coll_c"] == o["coll_c"]
        assert abs(g["mean_dq"] - o["mean_dq"]) <= 1e-10 * o["mean_qf"]
        assert g["m2_dq"] == pytest.approx(o["m2_dq"], rel=1e-6)
    assert abs(r["estimate"] - est) <= 1e-10 * abs(est)
