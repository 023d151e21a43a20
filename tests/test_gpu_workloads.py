"""The full-size workloads on the GPU, through the C ABI.

* eps sweep at RMSE 1e-3 (eps in {1e-4, 1e-3, 1e-2, 1e-1, 1}, the batched
  launch): each estimate within 4 standard errors of the exact E[Q_8] and
  with the statistical constraint met; at the full sample numbers, sampled
  trajectories (runs of 256 samples at random offsets of every level) equal
  the oracle's one by one.
* precision study (density 1 + cos 2 pi x, eps = 1e-3, L = 10): FP32 and
  FP64 particle state against the oracle per level, and both MLMC estimates
  against the exact E[Q_10].
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


def dump(prob, level, begin, n):
    P = pkg.as_problem(prob)
    dt = torch.float64 if P.fp64_state else torch.float32
    traj = torch.empty(2 * n, dtype=dt, device="cuda")
    coll = torch.empty(2 * n, dtype=torch.int32, device="cuda")
    st = pkg.mlmc_ap_simulate_level(P, level, begin, n, traj=traj, coll=coll)
    torch.cuda.synchronize()
    x = traj.cpu().double().numpy()
    c = coll.cpu().numpy().astype(np.int64)
    return st, x[:n], x[n:], c[:n], c[n:]


@pytest.fixture(scope="module")
def sweep():
    probs, tols = W.cfg3()
    sel = [(p, t) for p, t in zip(probs, tols) if t == 1e-3]
    res = pkg.mlmc_ap_estimate_batch([p for p, _ in sel], [t for _, t in sel])
    return sel, res


def test_eps_sweep_rmse_1e3(sweep):
    sel, res = sweep
    for (p, t), r in zip(sel, res):
        exact = CF.level_second_moment(p, p["L"])
        sd = math.sqrt(r["var_estimator"])
        say("eps %.0e: estimate %.7f exact %.7f sd %.2e N %s" % (p["eps"], r["estimate"], exact,
                                                                 sd, r["N"]))
        assert r["converged"] and r["var_estimator"] <= 0.5 * t * t * (1 + 1e-12)
        assert abs(r["estimate"] - exact) <= 4.0 * sd
        # the coarse path of every level has the law of the level below
        for l in range(1, p["L"] + 1):
            lv = r["levels"][l]
            e_c = CF.level_second_moment(p, l - 1)
            sd_c = math.sqrt(lv["m2_qc"] / (lv["n"] - 1) / lv["n"])
            assert abs(lv["mean_qc"] - e_c) <= 4.5 * sd_c + 1e-12


def test_eps_sweep_sampled_trajectories(sweep):
    """At the sample numbers of the full runs: runs of 256 samples at random
    offsets of every level against the oracle, one by one."""
    sel, res = sweep
    rng = np.random.default_rng(11)
    for (p, t), r in zip(sel, res):
        for l in range(p["L"] + 1):
            N = r["N"][l]
            for begin in rng.integers(0, max(N - 256, 1), size=2):
                n = int(min(256, N - begin))
                st, xf, xc, cf, cc = dump(p, l, int(begin), n)
                ref = O.simulate(p, l, int(begin), n)
                assert np.array_equal(cf, ref["cf"].astype(np.int64))
                assert np.array_equal(cc, ref["cc"].astype(np.int64))
                # per-trajectory bar: 1e-5 max(|x_oracle|, rms(x_oracle))
                sf = np.maximum(np.abs(ref["xf"]), math.sqrt(np.mean(ref["xf"] ** 2)))
                assert np.max(np.abs(xf - ref["xf"]) / sf) <= 1e-5
                if l >= 1:
                    sc = np.maximum(np.abs(ref["xc"]), math.sqrt(np.mean(ref["xc"] ** 2)))
                    assert np.max(np.abs(xc - ref["xc"]) / sc) <= 1e-5


@pytest.mark.parametrize("level,n", [(0, 20000), (2, 20000), (5, 8000), (8, 2000), (10, 1000)])
def test_precision_study_levels(level, n):
    """FP32 and FP64 particle state against the FP64 oracle on the same
    samples: per-trajectory error and the error of the level mean."""
    p32 = dict(W.cfg4(0), qoi=0)
    p64 = dict(W.cfg4(1), qoi=0)
    ref = O.simulate(p32, level, 0, n)
    dq_ref = ref["xf"] ** 2 - (ref["xc"] ** 2 if level else 0.0)
    sd = math.sqrt(np.var(dq_ref) / n) + 1e-300
    out = {}
    worst = {}
    for name, p, tol in (("fp32", p32, 1e-5), ("fp64", p64, 1e-12)):
        st, xf, xc, cf, cc = dump(p, level, 0, n)
        dq = xf ** 2 - (xc ** 2 if level else 0.0)
        worst[name] = np.max(np.abs(dq - dq_ref))
        assert np.array_equal(cf, ref["cf"].astype(np.int64))
        assert np.array_equal(cc, ref["cc"].astype(np.int64))
        scale = np.maximum(np.abs(ref["xf"]), math.sqrt(np.mean(ref["xf"] ** 2)))
        err = np.max(np.abs(xf - ref["xf"]) / scale)
        assert err <= tol, (name, err)
        out[name] = (st["mean_dq"] - dq_ref.mean(), err)
    say("level %d: mean dQ error fp32 %.3e fp64 %.3e (standard error %.3e); "
        "max trajectory error fp32 %.2e fp64 %.2e" % (level, out["fp32"][0], out["fp64"][0], sd,
                                                     out["fp32"][1], out["fp64"][1]))
    # FP64 state: rounding only; FP32 state: far below the 1e-3 RMSE target
    assert abs(out["fp64"][0]) <= worst["fp64"] + 1e-15 <= 1e-10
    assert abs(out["fp32"][0]) <= worst["fp32"] + 1e-15
    assert abs(out["fp32"][0]) <= 1e-5


def test_precision_study_estimates():
    """cfg4 MLMC estimates with FP32 and FP64 state: both within 4 standard
    errors of the exact E[Q_10] = 2.3819542840; histograms sum to N."""
    tol = 3e-3
    exact = CF.level_second_moment(W.cfg4(0), 10)
    assert abs(exact - 2.3819542840) < 1e-9
    r32 = pkg.mlmc_ap_estimate(W.cfg4(0), tol, hist=True)
    r64 = pkg.mlmc_ap_estimate(W.cfg4(1), tol, hist=True)
    for r in (r32, r64):
        sd = math.sqrt(r["var_estimator"])
        assert r["converged"] and abs(r["estimate"] - exact) <= 4.0 * sd
        for l, h in enumerate(r["hist"]):
            nb = 64
            assert sum(h[:3 * nb:3]) + h[3 * nb] + h[3 * nb + 1] == r["N"][l]
    say("cfg4: fp32 %.7f fp64 %.7f exact %.7f sd %.2e" % (r32["estimate"], r64["estimate"], exact,
                                                           math.sqrt(r32["var_estimator"])))


def test_bench_workload_full_size_against_oracle():
    """The estimate the benchmark times (eps = 0.01, L = 8, RMSE 1e-3; direct
    persistent launches with the particle kernel timed by HIP events; block
    256, one trajectory per lane, 8 waves per SIMD), at its full sample
    numbers: every level's fine and coarse collision totals over its N_l
    samples equal the oracle's exactly (integer decisions), and the level
    means and the estimate agree within the FP32 per-trajectory bar."""
    prob = W.cfg2()
    r = pkg.mlmc_ap_estimate(prob, 1e-3, pkg.options(batched=2, block=256, ppt=1,
                                                     waves_per_simd=8))
    say("bench workload: N %s estimate %.7f" % (r["N"], r["estimate"]))
    assert r["converged"]
    est, levels = OM.estimate_fixed(prob, r["N"])
    for l, (g, o) in enumerate(zip(r["levels"], levels)):
        say("  level %d n %d coll %d/%d mean dq %.9e oracle %.9e" % (
            l, g["n"], g["coll_f"], g["coll_c"], g["mean_dq"], o["mean_dq"]))
        assert g["n"] == o["n"]
        assert g["coll_f"] == o["coll_f"] and g["coll_c"] == o["coll_c"]
        assert abs(g["mean_dq"] - o["mean_dq"]) <= 2e-5 * o["mean_qf"]
        # FP32 rounding of the positions (~1e-7 relative) against level
        # differences dQ of standard deviation down to ~1e-3
        assert g["m2_dq"] == pytest.approx(o["m2_dq"], rel=1e-2)
    assert abs(r["estimate"] - est) <= 2e-5 * abs(est)


def test_plain_mc_full_size():
    """Plain Monte Carlo at level 8 to RMSE 1e-3 (the benchmark's comparison
    run, single trajectories): its persistent launches against one per-level
    run over the same samples [0, N) -- collision totals exactly equal, mean
    and variance to FP64 summation order -- and sampled runs of 256
    trajectories at random offsets against the oracle, one by one."""
    prob = W.cfg2()
    L = prob["L"]
    r = pkg.mlmc_ap_plain_mc(prob, 1e-3)
    N = r["N"][L]
    g = r["levels"][L]
    say("plain MC: N %d estimate %.7f" % (N, r["estimate"]))
    assert r["converged"] and N > 10 ** 7
    st = pkg.mlmc_ap_simulate_level(prob, L, 0, N, single=True)
    assert st["n"] == N and st["coll_f"] == g["coll_f"] and st["coll_c"] == 0
    assert abs(st["mean_dq"] - g["mean_dq"]) <= 1e-12 * g["mean_dq"]
    assert st["m2_dq"] == pytest.approx(g["m2_dq"], rel=1e-10)
    rng = np.random.default_rng(12)
    for begin in rng.integers(0, N - 256, size=4):
        P = pkg.as_problem(prob)
        traj = torch.empty(512, dtype=torch.float32, device="cuda")
        coll = torch.empty(512, dtype=torch.int32, device="cuda")
        pkg.mlmc_ap_simulate_level(P, L, int(begin), 256, single=True, traj=traj, coll=coll)
        torch.cuda.synchronize()
        x = traj.cpu().double().numpy()[:256]
        c = coll.cpu().numpy().astype(np.int64)[:256]
        ref = O.simulate(prob, L, int(begin), 256, single=True)
        assert np.array_equal(c, ref["cf"].astype(np.int64))
        scale = np.maximum(np.abs(ref["xf"]), math.sqrt(np.mean(ref["xf"] ** 2)))
        assert np.max(np.abs(x - ref["xf"]) / scale) <= 1e-5


def test_eps_sweep_all_requests_as_benchmarked():
    """The benchmark's eps sweep: all 15 requests (5 eps x 3 tolerances) in
    one batched launch per iteration; every estimate meets its own
    statistical constraint and lies within 4.5 standard errors of its exact
    E[Q_8]; each equals the same request run alone (bitwise)."""
    probs, tols = W.cfg3()
    batch = pkg.mlmc_ap_estimate_batch(probs, tols)
    worst = 0.0
    for p, t, r in zip(probs, tols, batch):
        assert r["converged"] and r["var_estimator"] <= 0.5 * t * t * (1 + 1e-12)
        z = abs(r["estimate"] - CF.level_second_moment(p, p["L"])) / math.sqrt(r["var_estimator"])
        worst = max(worst, z)
        assert z <= 4.5, (p["eps"], t, r["estimate"])
    say("eps sweep, 15 requests: worst |z| %.2f" % worst)
    for i in (0, 7, 14):
        alone = pkg.mlmc_ap_estimate(probs[i], tols[i])
        assert alone["estimate"] == batch[i]["estimate"] and alone["N"] == batch[i]["N"]


def test_bench_estimate_launch_forms_bitwise_equal():
    """The benchmarked estimate in each launch form it reports (direct, timed,
    hipGraph replay, one launch per level) at full size: bitwise the same
    estimate, sample numbers and per-level statistics."""
    prob = W.cfg2()
    tk = dict(block=256, ppt=1, waves_per_simd=8)
    runs = [pkg.mlmc_ap_estimate(prob, 1e-3, pkg.options(batched=b, **tk)) for b in (0, 2, 1, -1)]
    ref = runs[0]
    for r in runs[1:]:
        assert r["estimate"] == ref["estimate"] and r["N"] == ref["N"]
        assert r["levels"] == ref["levels"]


def test_cfg1_full_size_fp64():
    """The plain single-level scheme at its stated size (velocities +-1,
    eps = 0.5, T = 0.5, dt = 0.01, N = 1e5, FP64 state): every trajectory
    against the oracle (collision counts exact, positions within 1e-12 on
    the R12 scale), and E[x^2] within 4 standard errors of the scheme's exact
    second moment 0.5683899408."""
    prob = W.cfg1()
    n = W.CFG1_N
    st, xf, xc, cf, cc = dump(prob, 0, 0, n)
    ref = O.simulate(prob, 0, 0, n)
    assert np.array_equal(cf, ref["cf"].astype(np.int64))
    assert np.all(cc == 0) and np.all(xc == 0.0)
    scale = np.maximum(np.abs(ref["xf"]), math.sqrt(np.mean(ref["xf"] ** 2)))
    err = float(np.max(np.abs(xf - ref["xf"]) / scale))
    q = ref["xf"] ** 2
    sd = float(np.std(q)) / math.sqrt(n)
    say("cfg1: N %d, E[x^2] gpu %.10f oracle %.10f exact 0.5683899408 sd %.2e, max traj err %.1e"
        % (n, st["mean_dq"], q.mean(), sd, err))
    assert err <= 1e-12
    assert st["n"] == n and st["coll_f"] == int(ref["cf"].astype(np.uint64).sum())
    assert abs(st["mean_dq"] - q.mean()) <= 1e-12
    assert abs(st["mean_dq"] - 0.5683899408) <= 4.0 * sd


def test_fp32_estimate_loop_against_oracle_loop():
    """The FP32-state estimator's own sample-number loop against the oracle's
    independent loop (``oracle.mlmc.estimate``, FP64) on the same problem.
    Their level variances differ by the FP32 rounding of the positions (about
    1e-6 relative), so eqs. Nopt1/Noptj give sample numbers that agree to
    about that relative size, not exactly: every N_l within 1e-4 relative
    (+2), the same number of top-up iterations, and estimates within 2e-5 of
    E[Q_L] of each other."""
    prob = W.cfg2(eps=0.05, stream_id=33)
    L, tol = prob["L"], 5e-3
    res = pkg.mlmc_ap_estimate(prob, tol, pkg.options(max_iter=8))
    ref = OM.estimate(prob, tol, L, n_warmup=1000, max_iter=8)
    exact = CF.level_second_moment(prob, L)
    say("fp32 loop: gpu N %s it %d est %.8f; oracle N %s est %.8f; exact %.8f"
        % (res["N"], res["iterations"], res["estimate"], ref["N"], ref["estimate"], exact))
    for a, b in zip(res["N"], ref["N"]):
        assert abs(a - b) <= 1e-4 * b + 2, (res["N"], ref["N"])
    assert res["converged"]
    assert abs(res["estimate"] - ref["estimate"]) <= 2e-5 * abs(exact)
    assert abs(res["estimate"] - exact) <= 4.0 * math.sqrt(res["var_estimator"])
