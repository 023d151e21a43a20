"""GPU parity of the KD scheme in the backgrounds B1 and B2 of Section 5
(piecewise-linear collision rate, Maxwellian N(0, 1), x(0) = 1) against the
FP64 oracle, through the C ABI.

Bars:
  * KD step counts, fine and coarse: bit-exact (collision times are decided on
    FP64 values on both sides; the device solves eq. intinv in closed form,
    the oracle by bisection on the rate integral, and the two roots agree to a
    few units of 1e-16, so a step count could only differ for a collision
    within that distance of a grid point);
  * positions: |x_gpu - x_oracle| <= 1e-12 max(|x_oracle|, rms(x_oracle));
  * statistics (QoI x(T) and x(T)^2): the device reduction against two-pass
    FP64 statistics of the device's own dump;
  * estimates of E[x(T)] in the symmetric background B1: within 4.5 standard
    errors of 1 (exact by symmetry).
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
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


def run(prob, level, n, begin=0, single=False, coarse_level=None):
    P = pkg.as_problem(prob)
    traj = torch.full((2 * n,), float("nan"), dtype=torch.float64, device="cuda")
    coll = torch.full((2 * n,), -1, dtype=torch.int32, device="cuda")
    if coarse_level is None:
        st = pkg.mlmc_ap_simulate_level(P, level, begin, n, single=single, traj=traj, coll=coll)
    else:
        st = pkg.mlmc_ap_simulate_pair(P, level, coarse_level, begin, n, traj=traj, coll=coll)
    torch.cuda.synchronize()
    x = traj.cpu().numpy()
    c = coll.cpu().numpy().astype(np.int64)
    return st, x[:n], x[n:], c[:n], c[n:]


def scaled_error(got, want):
    scale = np.maximum(np.abs(want), math.sqrt(np.mean(want ** 2)))
    return float(np.max(np.abs(got - want) / scale))


B1, B2 = W.BG_B1, W.BG_B2
CASES = [
    # name, problem, level, begin, n, single, coarse level
    ("b1_a10_b100_pair_l3", W.cfg_bg(B1, 10.0, 100.0, stream_id=701), 3, 0, 3001, False, None),
    ("b1_a10_b1000_pair_l5", W.cfg_bg(B1, 10.0, 1000.0, stream_id=702), 5, 7, 1500, False, None),
    ("b1_a10_b1_pair_l2_kinetic", W.cfg_bg(B1, 10.0, 1.0, stream_id=703), 2, 0, 4000, False, None),
    ("b2_a10_b100_pair_l4", W.cfg_bg(B2, 10.0, 100.0, stream_id=704), 4, 0, 2000, False, None),
    ("b2_a100_b10_pair_l1", W.cfg_bg(B2, 100.0, 10.0, stream_id=705), 1, 3, 3000, False, None),
    ("b1_a2_b100_single_l6", W.cfg_bg(B1, 2.0, 100.0, stream_id=706), 6, 0, 1000, True, None),
    ("b2_a50_b1000_l0", W.cfg_bg(B2, 50.0, 1000.0, stream_id=707), 0, 11, 2049, False, None),
    ("b1_a10_b100_M4_pair_l2", W.cfg_bg(B1, 10.0, 100.0, M=4, stream_id=708), 2, 0, 2000,
     False, None),
    ("b1_a10_b100_pair_5_2", W.cfg_bg(B1, 10.0, 100.0, stream_id=709), 5, 0, 1200, False, 2),
    ("b2_a20_b1_pair_l8_kinetic", W.cfg_bg(B2, 20.0, 1.0, stream_id=710), 8, 0, 1000, False, None),
    ("b1_a0_b100_homogeneous_pair_l3", W.cfg_bg(B1, 0.0, 100.0, stream_id=711), 3, 0, 2000,
     False, None),
    ("b1_a10_b100_last_samples", W.cfg_bg(B1, 10.0, 100.0, stream_id=712), 2, 2 ** 32 - 500,
     500, False, None),
    ("b1_a10_b100_one_sample", W.cfg_bg(B1, 10.0, 100.0, stream_id=713), 4, 0, 1, False, None),
    ("b2_a10_b100_normal_x0_l3", dict(W.cfg_bg(B2, 10.0, 100.0, stream_id=714),
                                      x0_kind=W.X0_NORMAL, x0_a=1.0, x0_b=0.3), 3, 0, 2000,
     False, None),
]


@pytest.mark.parametrize("name,prob,level,begin,n,single,lc", CASES, ids=[c[0] for c in CASES])
def test_background_trajectories_match_oracle(name, prob, level, begin, n, single, lc):
    say("case", name)
    st, xf, xc, cf, cc = run(prob, level, n, begin, single, lc)
    ref = O.simulate(prob, level, begin, n, single=single, coarse_level=lc)
    assert np.array_equal(cf, ref["cf"].astype(np.int64)), "fine KD step counts differ"
    assert np.array_equal(cc, ref["cc"].astype(np.int64)), "coarse KD step counts differ"
    coarse = level >= 1 and not single
    ef = scaled_error(xf, ref["xf"])
    ec = scaled_error(xc, ref["xc"]) if coarse else 0.0
    say("  max scaled error fine %.3e coarse %.3e, mean KD steps %.1f / %.1f"
        % (ef, ec, cf.mean(), cc.mean()))
    assert ef <= REL and ec <= REL
    dev = OM.stats_of(xf, xc, 0 if single else level, prob.get("qoi", 0))
    assert st["n"] == n and st["coll_f"] == int(cf.sum()) and st["coll_c"] == int(cc.sum())
    sd = math.sqrt(dev["m2_dq"] / max(n - 1, 1)) + 1e-300
    assert abs(st["mean_dq"] - dev["mean_dq"]) <= 1e-12 * (abs(dev["mean_dq"]) + sd)
    assert st["m2_dq"] == pytest.approx(dev["m2_dq"], rel=1e-9, abs=1e-18)


def test_position_qoi_statistics():
    """QoI x(T): dQ = x_f - x_c, with the same reduction as x^2."""
    prob = W.cfg_bg(B2, 10.0, 100.0, stream_id=720)
    for qoi in (pkg.QOI_X, pkg.QOI_X2):
        p = dict(prob, qoi=qoi)
        st, xf, xc, _, _ = run(p, 4, 5000)
        dev = OM.stats_of(xf, xc, 4, qoi)
        for k in ("mean_dq", "mean_qf", "mean_qc"):
            assert abs(st[k] - dev[k]) <= 1e-12 * (1.0 + abs(dev[k]))
        for k in ("m2_dq", "m2_qf", "m2_qc", "c_fc"):
            assert st[k] == pytest.approx(dev[k], rel=1e-9, abs=1e-15)
    # the splitting scheme takes the position QoI too
    sp = dict(W.cfg2(eps=0.1, stream_id=721), qoi=pkg.QOI_X)
    P = pkg.as_problem(sp)
    traj = torch.empty(2 * 3000, dtype=torch.float32, device="cuda")
    st = pkg.mlmc_ap_simulate_level(P, 3, 0, 3000, traj=traj)
    x = traj.cpu().double().numpy()
    dev = OM.stats_of(x[:3000], x[3000:], 3, pkg.QOI_X)
    assert abs(st["mean_dq"] - dev["mean_dq"]) <= 1e-12 * (1.0 + abs(dev["mean_dq"]))


@pytest.mark.parametrize("kind,a,b", [(B1, 10.0, 100.0), (B1, 10.0, 1000.0), (B1, 100.0, 10.0)])
def test_symmetric_background_estimate(kind, a, b):
    """MLMC estimate of E[x(T)] in B1 (levels dt = 2^-l, l = 0..L): the exact
    value is 1 (symmetry), and every level's correction has mean 0."""
    prob = dict(W.cfg_bg(kind, a, b, stream_id=730), L=6)
    res = pkg.mlmc_ap_estimate(prob, 2e-3)
    sd = math.sqrt(res["var_estimator"])
    say("B1 a=%g b=%g: estimate %.6f sd %.2e N %s" % (a, b, res["estimate"], sd, res["N"]))
    assert res["converged"] and abs(res["estimate"] - 1.0) <= 4.5 * sd
    for l in range(1, prob["L"] + 1):
        lv = res["levels"][l]
        s = math.sqrt(lv["m2_dq"] / max(lv["n"] - 1, 1) / lv["n"])
        assert abs(lv["mean_dq"]) <= 4.5 * s + 1e-15


def test_background_estimate_launch_forms_and_oracle():
    """An estimate in B2 (no symmetry): bitwise the same in every launch
    form, and level by level equal to the oracle on the same sample ranges
    (KD step totals exact, means to 1e-10)."""
    prob = dict(W.cfg_bg(B2, 10.0, 100.0, stream_id=740), L=5)
    ref = pkg.mlmc_ap_estimate(prob, 5e-3, pkg.options(batched=0))
    for batched in (-1, 1, 2):
        r = pkg.mlmc_ap_estimate(prob, 5e-3, pkg.options(batched=batched))
        assert r["estimate"] == ref["estimate"] and r["N"] == ref["N"]
        assert r["levels"] == ref["levels"]
    est, levels = OM.estimate_fixed(prob, ref["N"])
    for l, (g, o) in enumerate(zip(ref["levels"], levels)):
        assert g["coll_f"] == o["coll_f"] and g["coll_c"] == o["coll_c"], l
        assert abs(g["mean_dq"] - o["mean_dq"]) <= 1e-10 * (1.0 + abs(o["mean_qf"])), l
    say("B2 a=10 b=100 L=5: estimate %.6f oracle %.6f" % (ref["estimate"], est))
