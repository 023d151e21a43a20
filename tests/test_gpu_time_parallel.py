"""Time-parallel path (one trajectory per wavefront, its fine steps across the
lanes) against the one-trajectory-per-lane loop, through the C ABI.

Both forms apply the same floating-point operations in the same order, so
trajectories, collision counts, histograms and statistics must be bitwise
equal; the library picks the form per launch (few long trajectories run
time-parallel), and mlmc_ap_set_tuning(tp_max_samples=-1) switches it off.
The oracle parity of the time-parallel form itself is covered by the
trajectory cases of the parity tests, whose small long-level runs take it."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2004_04071_amd")

pytestmark = pytest.mark.gpu

DEFAULT_TP = 4096


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    pkg.mlmc_ap_init()
    yield
    pkg.mlmc_ap_set_tuning(tp_max_samples=DEFAULT_TP)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run(prob, level, begin, n, single, tp):
    pkg.mlmc_ap_set_tuning(tp_max_samples=DEFAULT_TP if tp else -1)
    P = pkg.as_problem(prob)
    dt = torch.float64 if P.fp64_state else torch.float32
    traj = torch.full((2 * n,), float("nan"), dtype=dt, device="cuda")
    coll = torch.full((2 * n,), -1, dtype=torch.int32, device="cuda")
    hist = P.qoi == pkg.QOI_X2_HIST
    out = pkg.mlmc_ap_simulate_level(P, level, begin, n, single=single, traj=traj, coll=coll,
                                     hist=bool(hist))
    torch.cuda.synchronize()
    st, h = out if hist else (out, None)
    return st, traj.cpu(), coll.cpu(), h


CASES = [
    ("agg_m2_l6", W.cfg2(eps=0.01, stream_id=71), 6, 17, 300, False),
    ("agg_m2_l5_one_tile", W.cfg2(eps=1.0, stream_id=72), 5, 0, 64, False),
    ("agg_m2_l7_ragged", W.cfg2(eps=1e-4, stream_id=73), 7, 5, 129, False),
    ("kicksum_l6", W.cfg2(eps=0.1, coupling=W.COUPLING_KICK_SUM, stream_id=74), 6, 3, 200, False),
    ("twopoint_l6", dict(W.cfg1(), M=2, L=8, dt0=0.125, T=1.0, fp64_state=0), 6, 0, 150, False),
    ("twopoint_fp64_l6", dict(W.cfg1(), M=2, L=8, dt0=0.125, T=1.0), 6, 9, 70, False),
    ("m4_l3", dict(W.cfg2(eps=0.05, stream_id=75), M=4, L=4), 3, 11, 200, False),
    ("cosine_hist_fp32_l6", W.cfg4(0), 6, 0, 100, False),
    ("cosine_hist_fp64_l6", W.cfg4(1), 6, 0, 100, False),
    ("single_l6", W.cfg2(eps=0.02, stream_id=76), 6, 40, 150, True),
    ("wide_threshold_l6", W.cfg2(eps=1e6, stream_id=77), 6, 0, 100, False),
    ("steps_96_l5", dict(W.cfg2(eps=0.3, stream_id=78), T=1.5, dt0=0.5), 5, 2, 77, False),
    ("agg_fp64_l6", dict(W.cfg2(eps=0.3, stream_id=79), fp64_state=1), 6, 0, 100, False),
]


@pytest.mark.parametrize("name,prob,level,begin,n,single", CASES, ids=[c[0] for c in CASES])
def test_time_parallel_equals_per_lane(name, prob, level, begin, n, single):
    say("case", name)
    a = run(prob, level, begin, n, single, tp=True)
    b = run(prob, level, begin, n, single, tp=False)
    assert a[0] == b[0], "statistics differ"
    assert torch.equal(a[1], b[1]), "positions differ"
    assert torch.equal(a[2], b[2]), "collision counts differ"
    assert a[3] == b[3], "histograms differ"
    assert a[0]["n"] == n and not torch.isnan(a[1]).any()


def test_time_parallel_case_matches_oracle():
    """A time-parallel run against the oracle directly (positions to the
    FP32 bar, collision counts exactly)."""
    prob = W.cfg2(eps=0.01, stream_id=80)
    st, traj, coll, _ = run(prob, 8, 123, 40, False, tp=True)
    ref = O.simulate(prob, 8, 123, 40)
    x = traj.double().numpy()
    c = coll.numpy().astype(np.int64)
    assert np.array_equal(c[:40], ref["cf"].astype(np.int64))
    assert np.array_equal(c[40:], ref["cc"].astype(np.int64))
    for got, want in ((x[:40], ref["xf"]), (x[40:], ref["xc"])):
        scale = np.maximum(np.abs(want), np.sqrt(np.mean(want ** 2)))
        assert np.max(np.abs(got - want) / scale) <= 1e-5


def key(r):
    return (r["estimate"], r["var_estimator"], tuple(r["N"]),
            tuple(tuple(sorted(l.items())) for l in r["levels"]))


@pytest.mark.parametrize("batched", [-1, 0, 1, 2])
def test_estimates_equal_with_and_without_time_parallel(batched):
    """The warm-up of an L = 8 estimate runs its long levels time-parallel;
    the estimate is bitwise the same with the path switched off."""
    pkg.mlmc_ap_set_tuning(tp_max_samples=DEFAULT_TP)
    prob = W.cfg2(eps=0.01, stream_id=81)
    on = pkg.mlmc_ap_estimate(prob, 1e-2, pkg.options(batched=batched))
    off = pkg.mlmc_ap_estimate(prob, 1e-2, pkg.options(batched=batched, tp_max_samples=-1))
    assert key(on) == key(off)


# Kinetic-diffusion items (homogeneous background): the time-parallel form
# walks the collision-time chain on wave-uniform values and sums the step
# increments in the per-lane loop's order.
KD_CASES = [
    ("kd_pair_l6", W.cfg_kd(eps=0.01, stream_id=91), 6, 0, 100, False),
    ("kd_pair_l8_ragged", W.cfg_kd(eps=0.01, stream_id=92), 8, 5, 70, False),
    ("kd_single_l6", W.cfg_kd(eps=0.01, stream_id=93), 6, 3, 100, True),
    ("kd_fine_l0_long", dict(W.cfg_kd(eps=0.01, stream_id=94), dt0=1.0 / 128), 0, 0, 65, False),
    ("kd_pair_l7_sparse", W.cfg_kd(eps=0.3, stream_id=95), 7, 0, 130, False),
    ("kd_pair_l6_flights_past_T", W.cfg_kd(eps=2.0, stream_id=96), 6, 9, 64, False),
    ("kd_pair_l10_many_windows", dict(W.cfg_kd(eps=0.01, stream_id=97), L=10), 10, 0, 20, False),
    ("kd_pair_m3_l4", dict(W.cfg_kd(eps=0.05, stream_id=98), M=3, L=5), 4, 0, 90, False),
    ("kd_pair_m4_l4", dict(W.cfg_kd(eps=0.05, stream_id=99), M=4, L=5), 4, 1, 90, False),
    ("kd_cosine_x0_l6", dict(W.cfg_kd(eps=0.05, stream_id=100), x0_kind=2), 6, 0, 80, False),
    ("kd_bg_a0_l10", W.cfg_bg(a=0.0, b=1000.0, L=12, stream_id=101), 10, 0, 64, False),
    # collision rates where some windows keep their guessed chain and others
    # walk it serially (flights crossing grid points now and then)
    ("kd_pair_l8_mixed_windows", W.cfg_kd(eps=0.05, stream_id=105), 8, 0, 100, False),
    ("kd_pair_l8_mixed_windows_2", W.cfg_kd(eps=0.03, stream_id=106), 8, 3, 70, False),
    ("kd_single_l8_mixed_windows", W.cfg_kd(eps=0.1, stream_id=107), 8, 0, 64, True),
    ("kd_pair_l8_windows_cut_short", W.cfg_kd(eps=0.02, stream_id=108), 8, 0, 80, False),
]


@pytest.mark.parametrize("name,prob,level,begin,n,single", KD_CASES, ids=[c[0] for c in KD_CASES])
def test_kd_time_parallel_equals_per_lane(name, prob, level, begin, n, single):
    say("case", name)
    a = run(prob, level, begin, n, single, tp=True)
    b = run(prob, level, begin, n, single, tp=False)
    assert a[0] == b[0], "statistics differ"
    assert torch.equal(a[1], b[1]), "positions differ"
    assert torch.equal(a[2], b[2]), "KD step counts differ"
    assert a[0]["n"] == n and not torch.isnan(a[1]).any()


def test_kd_time_parallel_nonadjacent_pair_equals_per_lane():
    """Levels 7 and 4 (block factor 8): coarse steps of up to 8 fine steps,
    carried across the 64-step windows."""
    prob = W.cfg_kd(eps=0.05, stream_id=102)
    res = []
    for tp in (DEFAULT_TP, -1):
        pkg.mlmc_ap_set_tuning(tp_max_samples=tp)
        traj = torch.zeros(2 * 100, dtype=torch.float64, device="cuda")
        coll = torch.zeros(2 * 100, dtype=torch.int32, device="cuda")
        st = pkg.mlmc_ap_simulate_pair(prob, 7, 4, 0, 100, traj=traj, coll=coll)
        torch.cuda.synchronize()
        res.append((st, traj.cpu(), coll.cpu()))
    pkg.mlmc_ap_set_tuning(tp_max_samples=DEFAULT_TP)
    assert res[0][0] == res[1][0]
    assert torch.equal(res[0][1], res[1][1]) and torch.equal(res[0][2], res[1][2])


def test_kd_time_parallel_case_matches_oracle():
    """A time-parallel KD run against the oracle directly (positions within
    1e-12 of the R12 scale, KD step counts exactly)."""
    prob = W.cfg_kd(eps=0.01, stream_id=103)
    st, traj, coll, _ = run(prob, 8, 11, 30, False, tp=True)
    ref = O.simulate(prob, 8, 11, 30)
    x = traj.numpy()
    c = coll.numpy().astype(np.int64)
    assert np.array_equal(c[:30], ref["cf"].astype(np.int64))
    assert np.array_equal(c[30:], ref["cc"].astype(np.int64))
    for got, want in ((x[:30], ref["xf"]), (x[30:], ref["xc"])):
        scale = np.maximum(np.abs(want), np.sqrt(np.mean(want ** 2)))
        assert np.max(np.abs(got - want) / scale) <= 1e-12


@pytest.mark.parametrize("batched", [-1, 0, 1])
def test_kd_estimates_equal_with_and_without_time_parallel(batched):
    """The KD estimate's warm-up runs its long levels time-parallel; the
    estimate is bitwise the same with the path switched off."""
    pkg.mlmc_ap_set_tuning(tp_max_samples=DEFAULT_TP)
    prob = W.cfg_kd(eps=0.01, stream_id=104)
    on = pkg.mlmc_ap_estimate(prob, 1e-2, pkg.options(batched=batched))
    off = pkg.mlmc_ap_estimate(prob, 1e-2, pkg.options(batched=batched, tp_max_samples=-1))
    assert key(on) == key(off)


# KD items in the backgrounds of Section 5: the time-parallel form walks the
# fine path's state chain on wave-uniform values and, for a pair, the coarse
# KD steps in a second in-order pass over each window.
BG_CASES = [
    ("bg_b1_a10_b1000_pair_l10", W.cfg_bg(W.BG_B1, 10.0, 1000.0, L=10, stream_id=111), 10, 3,
     70, False),
    ("bg_b1_a10_b100_pair_l8", W.cfg_bg(W.BG_B1, 10.0, 100.0, stream_id=112), 8, 0, 100, False),
    ("bg_b2_a10_b100_pair_l9", W.cfg_bg(W.BG_B2, 10.0, 100.0, L=9, stream_id=113), 9, 0, 64,
     False),
    ("bg_b1_a10_b1000_single_l12", W.cfg_bg(W.BG_B1, 10.0, 1000.0, L=12, stream_id=114), 12, 0,
     40, True),
    ("bg_b2_a20_b1_pair_l8_flights_past_T", W.cfg_bg(W.BG_B2, 20.0, 1.0, stream_id=115), 8, 0,
     130, False),
    ("bg_b1_a10_b100_M4_pair_l4", W.cfg_bg(W.BG_B1, 10.0, 100.0, M=4, L=4, stream_id=116), 4, 0,
     80, False),
    ("bg_b1_a100_b10_pair_l7", W.cfg_bg(W.BG_B1, 100.0, 10.0, stream_id=117), 7, 0, 90, False),
    ("bg_b2_a10_b100_normal_x0_l7", dict(W.cfg_bg(W.BG_B2, 10.0, 100.0, stream_id=118),
                                         x0_kind=W.X0_NORMAL, x0_a=1.0, x0_b=0.3), 7, 0, 64,
     False),
    ("bg_b1_a10_b1000_pair_l14_long", W.cfg_bg(W.BG_B1, 10.0, 1000.0, L=14, stream_id=119), 14,
     0, 8, False),
    ("bg_b1_a10_b1000_last_samples", W.cfg_bg(W.BG_B1, 10.0, 1000.0, L=8, stream_id=120), 8,
     2 ** 32 - 65, 65, False),
]


@pytest.mark.parametrize("name,prob,level,begin,n,single", BG_CASES, ids=[c[0] for c in BG_CASES])
def test_kd_background_time_parallel_equals_per_lane(name, prob, level, begin, n, single):
    say("case", name)
    a = run(prob, level, begin, n, single, tp=True)
    b = run(prob, level, begin, n, single, tp=False)
    assert a[0] == b[0], "statistics differ"
    assert torch.equal(a[1], b[1]), "positions differ"
    assert torch.equal(a[2], b[2]), "KD step counts differ"
    assert a[0]["n"] == n and not torch.isnan(a[1]).any()


def test_kd_background_time_parallel_nonadjacent_pair_equals_per_lane():
    """Levels 11 and 3 in B1 (block factor 256): coarse KD steps that gather
    hundreds of fine steps across many windows."""
    prob = W.cfg_bg(W.BG_B1, 10.0, 1000.0, L=11, stream_id=121)
    res = []
    for tp in (DEFAULT_TP, -1):
        pkg.mlmc_ap_set_tuning(tp_max_samples=tp)
        traj = torch.zeros(2 * 50, dtype=torch.float64, device="cuda")
        coll = torch.zeros(2 * 50, dtype=torch.int32, device="cuda")
        st = pkg.mlmc_ap_simulate_pair(prob, 11, 3, 0, 50, traj=traj, coll=coll)
        torch.cuda.synchronize()
        res.append((st, traj.cpu(), coll.cpu()))
    pkg.mlmc_ap_set_tuning(tp_max_samples=DEFAULT_TP)
    assert res[0][0] == res[1][0]
    assert torch.equal(res[0][1], res[1][1]) and torch.equal(res[0][2], res[1][2])


def test_kd_background_time_parallel_case_matches_oracle():
    """A time-parallel run in B1 against the oracle directly (positions within
    1e-12 of the R12 scale, KD step counts exactly)."""
    prob = W.cfg_bg(W.BG_B1, 10.0, 1000.0, L=9, stream_id=122)
    st, traj, coll, _ = run(prob, 9, 5, 24, False, tp=True)
    ref = O.simulate(prob, 9, 5, 24)
    x = traj.numpy()
    c = coll.numpy().astype(np.int64)
    assert np.array_equal(c[:24], ref["cf"].astype(np.int64))
    assert np.array_equal(c[24:], ref["cc"].astype(np.int64))
    for got, want in ((x[:24], ref["xf"]), (x[24:], ref["xc"])):
        scale = np.maximum(np.abs(want), np.sqrt(np.mean(want ** 2)))
        assert np.max(np.abs(got - want) / scale) <= 1e-12


@pytest.mark.parametrize("batched", [-1, 0, 1])
def test_kd_background_estimates_equal_with_and_without_time_parallel(batched):
    """An estimate in B1 whose warm-up runs its long levels time-parallel;
    bitwise the same with the path switched off."""
    pkg.mlmc_ap_set_tuning(tp_max_samples=DEFAULT_TP)
    prob = W.cfg_bg(W.BG_B1, 10.0, 1000.0, L=10, stream_id=123)
    on = pkg.mlmc_ap_estimate(prob, 1e-2, pkg.options(batched=batched))
    off = pkg.mlmc_ap_estimate(prob, 1e-2, pkg.options(batched=batched, tp_max_samples=-1))
    assert key(on) == key(off)
