"""The experiment protocol of Section 5.3 and the level-adaptive finest level
(Sections 4.1 and 5.2).

CPU: the warm-up depth tau and the extrapolated profile on hand-derived
cases (oracle and library); the O(dt^3) rate that the extrapolation assumes,
measured on the oracle's KD scheme; the bias estimate against exact level
means (the splitting scheme's closed form); the oracle's protocol loop
against what fixes it from outside: E[x(T)] = 1 in the symmetric background
B1, the statistical constraint, the level set recomputed from a fresh warm-up,
every item's statistics recomputed from scratch, and, with a growing L, the
RMSE against the exact limit.
GPU: the library's LEVELS_HEURISTIC_TAU estimate and its adaptive L against
the oracle's loop (same tau, level set, sample numbers; FP64 state), and the
validation rules."""
import math

import pytest

import oracle as O
import workloads as W
from oracle import closed_form as CF
from oracle import levels as OL
from oracle import mlmc as OM

pkg = pytest.importorskip("paper_2004_04071_amd")


@pytest.fixture(scope="module")
def lib():
    try:
        return pkg.lib()
    except Exception as e:  # pragma: no cover
        pytest.skip("library not built: %s" % e)


# (problem, tau) derived by hand: tau = round(log_M(dt0 R)) within [1, L]
DEPTH = [
    (W.cfg_bg(a=10.0, b=1000.0, L=14), 10),   # log2(1000) = 9.97
    (W.cfg_bg(a=10.0, b=1000.0, L=8), 8),     # clamped to L
    (W.cfg_bg(a=1.0, b=100.0, L=14), 7),      # log2(100) = 6.64
    (W.cfg_bg(a=0.0, b=10.0, L=14), 3),       # log2(10) = 3.32
    (W.cfg_bg(a=0.0, b=1.5, L=14), 1),        # log2(1.5) = 0.58: at least 1
    (W.cfg_bg(a=0.0, b=1000.0, M=4, L=9), 5),  # log4(1000) = 4.98
    (W.cfg_bg(a=0.0, b=1000.0, L=0), 0),      # L = 0
    (W.cfg_kd(eps=0.1), 6),                   # dt0 R = 0.5 / 0.01 = 50: log2 = 5.64
    (W.cfg_kd(eps=0.01), 8),                  # log2(5000) = 12.3: clamped to L
]


@pytest.mark.parametrize("prob,tau", DEPTH)
def test_warmup_depth_hand_cases(lib, prob, tau):
    assert OL.warmup_depth(prob) == tau
    assert pkg.mlmc_ap_warmup_depth(prob) == tau


def test_extrapolated_profile(lib):
    V = [2.0, 1.9, 1.7, 1.6]
    Vd = [0.0, 0.5, 0.7, 0.3]
    for M in (2, 3, 4):
        Vo, Vdo = OL.extrapolate(V, Vd, 3, M, 9)
        gV, gVd = pkg.mlmc_ap_extrapolate_variances(V, Vd, 3, M, 9)
        assert gV == Vo and gVd[1:] == Vdo[1:]
        assert Vo[:4] == V and Vdo[1:4] == Vd[1:]
        assert Vo[4:] == [1.6] * 6
        for l in range(4, 10):   # (dt_l / dt_{l-1})^3 = M^-3 per level
            assert Vdo[l] == pytest.approx(Vdo[l - 1] / M ** 3, rel=1e-15)
    # M = 2: exact powers of two
    assert OL.extrapolate(V, Vd, 3, 2, 5)[1][5] == 0.3 / 64.0
    with pytest.raises(pkg.MlmcApError):
        pkg.mlmc_ap_extrapolate_variances(V, Vd, 4, 2, 3)   # tau > L
    with pytest.raises(pkg.MlmcApError):
        pkg.mlmc_ap_extrapolate_variances([1.0, -1.0], [0.0, 1.0], 1, 2, 3)


def test_kd_difference_variance_decays_at_dt_cubed():
    """The rate the extrapolation assumes (Section 5.2: past dt = 1/R the
    difference variance of the KD levels falls as O(dt^3)), measured on the
    oracle's homogeneous KD background (a = 0, b = 100): successive ratios
    V_{l-1,l-2} / V_{l,l-1} at R dt_l = 0.024 .. 0.003 approach M^3 = 8."""
    p = W.cfg_bg(a=0.0, b=100.0, L=16)
    Vd = []
    for l in range(12, 16):
        r = O.simulate(p, l, 0, 40000)
        Vd.append(OM.sample_variance(OM.stats_of(r["xf"], r["xc"], l, W.QOI_X)))
    ratios = [a / b for a, b in zip(Vd[:-1], Vd[1:])]
    print("ratios", ratios)
    assert all(6.5 <= q <= 9.5 for q in ratios), ratios


def _splitting(M=2, L=2, stream=300, eps=1.0):
    return dict(eps=eps, T=1.0, dt0=0.5, M=M, L=L, x0_kind=1, x0_a=0.0, x0_b=1.0, eq_kind=1,
                coupling=1, seed=42, stream_id=stream, fp64_state=1)


@pytest.mark.parametrize("M", [2, 3, 4])
def test_bias_estimate_against_exact_level_means(M):
    """Where the splitting scheme's weak error is first order in dt (eps = 1),
    |E[Q_L - Q_c]| / (M^(L-c) - 1) from the exact level means matches the
    exact bias |E[Q_L] - E[Q]| within 2 % (c = L - 1 and L - 2); a factor
    M^(L-c) instead of M^(L-c) - 1 would miss by 25-50 %."""
    p = _splitting(M=M)
    top = {2: 24, 3: 15, 4: 12}[M]
    m = [CF.level_second_moment(p, l) for l in range(top + 1)]
    for L in range(3, top - 7):
        for k in (1, 2):
            b = OM.bias_estimate(m[L] - m[L - k], M, L, L - k)
            assert b == pytest.approx(abs(m[L] - m[-1]), rel=0.02), (M, L, k)


B1_CASE = dict(prob=W.cfg_bg(a=10.0, b=1000.0, L=12), tol=1e-3, n_warmup=100)


@pytest.fixture(scope="module")
def oracle_b1():
    c = B1_CASE
    return OM.estimate_adaptive(c["prob"], c["tol"], n_warmup=c["n_warmup"])


def _fresh_stats(prob, level, coarse, n):
    if level == 0:
        r = O.simulate(prob, 0, 0, n)
    elif coarse < 0:
        r = O.simulate(prob, level, 0, n, single=True)
    else:
        r = O.simulate(prob, level, 0, n, coarse_level=coarse)
    return OM.stats_of(r["xf"], r["xc"], 0 if coarse < 0 else level, prob.get("qoi", 0))


def test_oracle_protocol_b1(oracle_b1):
    prob, tol, nw = B1_CASE["prob"], B1_CASE["tol"], B1_CASE["n_warmup"]
    r = oracle_b1
    assert r["tau"] == 10 and r["L"] == 12 and r["added"] == 0
    # the set, recomputed from a fresh warm-up of levels 0..tau only
    V, Vd = [], []
    for l in range(r["tau"] + 1):
        st = _fresh_stats(prob, l, l - 1, nw)
        V.append(OM.sample_variance(st, "dq" if l == 0 else "qf"))
        Vd.append(OM.sample_variance(st))
    want = OL.heuristic(*OL.extrapolate(V, Vd, r["tau"], prob["M"], prob["L"]))
    assert r["levels"] == want
    assert r["levels"][-1] == prob["L"]
    assert r["coarse"] == [-1] + r["levels"][:-1]
    # every item's statistics are those of samples [0, N) of its pair
    est = 0.0
    for l, c, n, st in zip(r["levels"], r["coarse"], r["N"], r["stats"]):
        f = _fresh_stats(prob, l, c, n)
        assert f["n"] == n and f["mean_dq"] == st["mean_dq"] and f["m2_dq"] == st["m2_dq"]
        est += f["mean_dq"]
    assert est == r["estimate"]
    # statistical constraint, and E[x(T)] = 1 at every level (B1 is
    # symmetric about x(0) = 1)
    assert r["converged"] and r["var_estimator"] <= 0.5 * tol * tol
    assert abs(r["estimate"] - 1.0) <= 4.5 * math.sqrt(r["var_estimator"])
    assert r["bias"] == OM.bias_estimate(r["stats"][-1]["mean_dq"], prob["M"], prob["L"],
                                         r["coarse"][-1])


GROW_CASE = dict(prob=_splitting(L=2, stream=301), tol=1e-2, n_warmup=1000, L_max=10)


@pytest.fixture(scope="module")
def oracle_grow():
    c = GROW_CASE
    return OM.estimate_adaptive(c["prob"], c["tol"], n_warmup=c["n_warmup"], L_max=c["L_max"],
                                select="all")


def test_oracle_adaptive_L_meets_the_rmse(oracle_grow):
    """Splitting scheme, eps = 1: exact level differences d_L = 4.0e-2,
    2.0e-2, 1.0e-2, 5.0e-3, 2.5e-3 at L = 3..7 against the bias bound
    tol/sqrt(2) = 7.1e-3.  From L = 2 the loop must add levels at least up to
    5 (d_4 is 4 standard errors above the bound) and need not go past 8; the
    estimate is unbiased for its final level (exact E[Q_L]) and within the
    tolerance of the exact limit."""
    prob, tol = GROW_CASE["prob"], GROW_CASE["tol"]
    r = oracle_grow
    L = r["L"]
    assert 5 <= L <= 8 and r["added"] == L - prob["L"]
    assert r["levels"] == list(range(L + 1))
    assert r["converged"] and r["var_estimator"] <= 0.5 * tol * tol
    assert r["bias"] <= tol / math.sqrt(2.0)
    exact_L = CF.level_second_moment(dict(prob, L=L), L)
    limit = CF.level_second_moment(dict(prob, L=24), 24)
    assert abs(r["estimate"] - exact_L) <= 4.5 * math.sqrt(r["var_estimator"])
    assert abs(r["estimate"] - limit) <= 3.0 * tol
    for l, c, n, st in zip(r["levels"], r["coarse"], r["N"], r["stats"]):
        f = _fresh_stats(dict(prob, L=L), l, c, n)
        assert f["n"] == n and f["m2_dq"] == st["m2_dq"]


# ---------------------------------------------------------------------------
# Validation (CPU: rejected before any device work)
# ---------------------------------------------------------------------------
BAD_OPTIONS = [
    (W.cfg2(), dict(level_select=pkg.LEVELS_HEURISTIC_TAU)),          # splitting scheme
    (W.cfg_bg(L=8), dict(level_select=4)),
    (W.cfg_bg(L=8), dict(L_max=8)),                                  # not above L
    (W.cfg_bg(L=8), dict(L_max=31)),
    (W.cfg_bg(L=8), dict(L_max=12, level_select=pkg.LEVELS_HEURISTIC)),
    (W.cfg_bg(L=8), dict(L_max=12, level_select=pkg.LEVELS_OPTIMAL)),
    (dict(W.cfg2(), dt0=0.5, L=8), dict(L_max=30)),                  # n_L >= 2^31
]


@pytest.mark.parametrize("prob,kw", BAD_OPTIONS)
def test_estimate_rejects_bad_selection_options(lib, prob, kw):
    with pytest.raises(pkg.MlmcApError) as e:
        pkg.mlmc_ap_estimate(prob, 1e-2, pkg.options(**kw))
    assert e.value.name == "EINVAL", str(e.value)   # before any device call


def test_plain_mc_and_server_reject_adaptive_L(lib):
    with pytest.raises(pkg.MlmcApError):
        pkg.mlmc_ap_plain_mc(W.cfg_bg(L=8), 1e-2, pkg.options(L_max=10))
    with pytest.raises(pkg.MlmcApError):
        pkg.mlmc_ap_server_create(opt=pkg.options(L_max=10))
    with pytest.raises(pkg.MlmcApError):
        pkg.mlmc_ap_server_create(opt=pkg.options(level_select=pkg.LEVELS_HEURISTIC_TAU))


# ---------------------------------------------------------------------------
# GPU
# ---------------------------------------------------------------------------
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    pkg.mlmc_ap_init()
    return pkg


def _compare(g, o, prob):
    print("L %d tau %d levels %s N %s estimate %.8f bias %.3e" % (
        g["L"], g["tau"], g["level_set"], [g["N"][l] for l in g["level_set"]], g["estimate"],
        g["bias_estimate"]), flush=True)
    assert g["L"] == o["L"] and g["tau"] == o["tau"]
    assert g["levels_added"] == o["added"]
    assert g["level_set"] == o["levels"]
    assert [g["N"][l] for l in o["levels"]] == o["N"]
    assert g["converged"] == o["converged"]
    assert g["iterations"] == o["iterations"]
    assert abs(g["estimate"] - o["estimate"]) <= 1e-10 * (abs(o["estimate"]) + 1.0)
    assert g["var_estimator"] == pytest.approx(o["var_estimator"], rel=1e-9)
    assert g["bias_estimate"] == pytest.approx(o["bias"], rel=1e-6, abs=1e-13)


@pytest.mark.gpu
def test_gpu_protocol_b1_matches_oracle(oracle_b1):
    """KD in B1 (a = 10, b = 1000, L = 12): warm-up of levels 0..10 only, the
    extrapolated profile, the heuristic set, the on-line loop: the same tau,
    set, sample numbers and estimate as the oracle's loop (FP64 state: the
    statistics agree to about 1e-15, far from any ceil or comparison the
    loop takes)."""
    pkg = _gpu()
    c = B1_CASE
    g = pkg.mlmc_ap_estimate(c["prob"], c["tol"], pkg.options(
        level_select=pkg.LEVELS_HEURISTIC_TAU, n_warmup=c["n_warmup"]))
    _compare(g, oracle_b1, c["prob"])
    assert abs(g["estimate"] - 1.0) <= 4.5 * math.sqrt(g["var_estimator"])


@pytest.mark.gpu
def test_gpu_adaptive_L_matches_oracle(oracle_grow):
    pkg = _gpu()
    c = GROW_CASE
    g = pkg.mlmc_ap_estimate(c["prob"], c["tol"], pkg.options(
        n_warmup=c["n_warmup"], L_max=c["L_max"]))
    _compare(g, oracle_grow, c["prob"])


@pytest.mark.gpu
def test_gpu_protocol_with_adaptive_L_in_b2_matches_oracle():
    """KD in B2 (a = 10, b = 100), L = 4 growing up to 12: the set is chosen
    again from the same warm-up profile at every new L; the items that stay
    keep their samples."""
    pkg = _gpu()
    prob = W.cfg_bg(background=W.BG_B2, a=10.0, b=100.0, L=4, stream_id=17)
    o = OM.estimate_adaptive(prob, 2e-3, n_warmup=100, L_max=12)
    assert o["added"] >= 1
    g = pkg.mlmc_ap_estimate(prob, 2e-3, pkg.options(
        level_select=pkg.LEVELS_HEURISTIC_TAU, n_warmup=100, L_max=12))
    _compare(g, o, prob)
    # launch forms give the same result
    g2 = pkg.mlmc_ap_estimate(prob, 2e-3, pkg.options(
        level_select=pkg.LEVELS_HEURISTIC_TAU, n_warmup=100, L_max=12, batched=-1))
    assert g2["estimate"] == g["estimate"] and g2["N"] == g["N"]
