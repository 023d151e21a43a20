"""Serving loop, batching and autotuner on the GPU, through the C ABI.

A request's sample ranges depend only on its own statistics and the server's
per-tick cap, and every statistic is reduced by a tree fixed by the sample
count, so results must be bitwise equal alone, in a mix, under a tight
memory budget, and to mlmc_ap_estimate with the same cap."""
import math

import pytest

import workloads as W
from oracle import closed_form as CF

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


def key(r):
    return (r["estimate"], r["var_estimator"], tuple(r["N"]),
            tuple(tuple(sorted(l.items())) for l in r["levels"]))


REQS = [(W.cfg2(eps=1e-3, stream_id=51), 1e-2), (W.cfg2(eps=0.1, stream_id=52), 5e-3),
        (W.cfg2(eps=1.0, stream_id=53), 1e-2), (dict(W.cfg2(eps=0.02, stream_id=54), T=0.5,
                                                      dt0=0.25), 8e-3)]


def serve(reqs, **cfg):
    srv = pkg.mlmc_ap_server_create(**cfg)
    try:
        tickets = [pkg.mlmc_ap_server_submit(srv, p, t) for p, t in reqs]
        out = {}
        for _ in range(10000):
            pkg.mlmc_ap_server_step(srv)
            for tk in tickets:
                if tk not in out:
                    r = pkg.mlmc_ap_server_poll(srv, tk)
                    if r is not None:
                        out[tk] = r
            if len(out) == len(tickets):
                break
        stats = pkg.mlmc_ap_server_get_stats(srv)
    finally:
        pkg.mlmc_ap_server_destroy(srv)
    return [out[t] for t in tickets], stats


def test_alone_equals_mix_equals_estimate():
    mixed, st = serve(REQS)
    assert st["completed"] == len(REQS)
    for (p, t), m in zip(REQS, mixed):
        alone, _ = serve([(p, t)])
        assert key(alone[0]) == key(m)
        direct = pkg.mlmc_ap_estimate(p, t)
        if max(m["N"]) <= 2 ** 24:  # no level split across ticks by the per-tick cap
            assert key(direct) == key(m)
        else:  # the same samples, merged in more pieces: equal up to rounding
            assert direct["N"] == m["N"]
            assert direct["estimate"] == pytest.approx(m["estimate"], rel=1e-13)
        assert m["converged"]
        exact = CF.level_second_moment(p, p["L"])
        assert abs(m["estimate"] - exact) <= 4.0 * math.sqrt(m["var_estimator"])


def test_tight_budget_queues_and_keeps_results():
    cap = 4096
    ref, _ = serve(REQS, max_samples_per_tick=cap)
    # with the time-parallel path off, each request needs about 9 levels x 65
    # tiles x 80 B per tick: two fit at once (results do not depend on the path)
    budget = 120 * 1024
    tight, st = serve(REQS, hbm_budget_bytes=budget, max_samples_per_tick=cap,
                      opt=pkg.options(tp_max_samples=-1))
    assert st["bytes_peak"] <= budget
    assert st["completed"] == len(REQS)
    for a, b in zip(ref, tight):
        assert key(a) == key(b)


def test_oversized_request_is_rejected():
    srv = pkg.mlmc_ap_server_create(hbm_budget_bytes=8 * 1024)
    try:
        with pytest.raises(pkg.MlmcApError) as e:
            pkg.mlmc_ap_server_submit(srv, W.cfg2(), 1e-2)
        assert e.value.name == "EBUSY"
        assert pkg.mlmc_ap_server_get_stats(srv)["rejected"] == 1
    finally:
        pkg.mlmc_ap_server_destroy(srv)


MIXED = [(W.cfg2(eps=0.1, stream_id=55), 1e-2),
         (dict(W.cfg2(eps=0.05, stream_id=56), fp64_state=1), 1e-2),
         (W.cfg_kd(eps=0.05, stream_id=57), 1e-2),
         (dict(W.cfg_kd(eps=0.3, stream_id=58), L=5), 1e-2)]


def test_mixed_precisions_and_schemes_in_one_server():
    """FP32 and FP64 splitting requests and KD requests served together (one
    launch per particle kernel and tick): each result equals the request
    served alone and is close to its exact value."""
    mixed, st = serve(MIXED)
    assert st["completed"] == len(MIXED)
    for (p, t), m in zip(MIXED, mixed):
        alone, _ = serve([(p, t)])
        assert key(alone[0]) == key(m)
        kd = p.get("scheme", 0) == W.SCHEME_KD
        exact = (CF.kinetic_limit(p["eps"], p["T"], 1.0) if kd
                 else CF.level_second_moment(p, p["L"]))
        assert m["converged"]
        assert abs(m["estimate"] - exact) <= 4.5 * math.sqrt(m["var_estimator"])


def test_invalid_requests_are_refused():
    srv = pkg.mlmc_ap_server_create()
    try:
        with pytest.raises(pkg.MlmcApError):
            pkg.mlmc_ap_server_submit(srv, W.cfg2(), 0.0)
        with pytest.raises(pkg.MlmcApError):
            pkg.mlmc_ap_server_submit(srv, dict(W.cfg2(), M=1), 1e-2)
        with pytest.raises(pkg.MlmcApError):   # histograms are not served
            pkg.mlmc_ap_server_submit(srv, W.cfg4(), 1e-2)
        with pytest.raises(pkg.MlmcApError) as e:
            pkg.mlmc_ap_server_poll(srv, 12345)
        assert e.value.name == "ENOTFOUND"
    finally:
        pkg.mlmc_ap_server_destroy(srv)


def test_cancel():
    srv = pkg.mlmc_ap_server_create()
    try:
        t1 = pkg.mlmc_ap_server_submit(srv, REQS[0][0], REQS[0][1])
        t2 = pkg.mlmc_ap_server_submit(srv, REQS[1][0], REQS[1][1])
        pkg.mlmc_ap_server_cancel(srv, t1)  # still queued
        pkg.mlmc_ap_server_step(srv)
        t3 = pkg.mlmc_ap_server_submit(srv, REQS[2][0], REQS[2][1])
        pkg.mlmc_ap_server_step(srv)
        pkg.mlmc_ap_server_cancel(srv, t3)  # admitted, in flight
        done = None
        for _ in range(1000):
            pkg.mlmc_ap_server_step(srv)
            done = pkg.mlmc_ap_server_poll(srv, t2)
            if done is not None:
                break
        assert done is not None and done["converged"]
        for t in (t1, t3):
            with pytest.raises(pkg.MlmcApError) as e:
                pkg.mlmc_ap_server_poll(srv, t)
            assert e.value.name == "ECANCELLED"
        st = pkg.mlmc_ap_server_get_stats(srv)
        assert st["cancelled"] == 2 and st["active"] == 0
    finally:
        pkg.mlmc_ap_server_destroy(srv)


def test_trace_replay_overlaps_requests():
    arr, probs, tols = W.cfg5_trace(40, rate=2000.0, seed=7)
    srv = pkg.mlmc_ap_server_create()
    try:
        lat, res = pkg.mlmc_ap_server_run_trace(srv, arr, probs, tols)
        st = pkg.mlmc_ap_server_get_stats(srv)
    finally:
        pkg.mlmc_ap_server_destroy(srv)
    assert all(l > 0 for l in lat) and all(r["converged"] for r in res)
    # continuous batching: far fewer launches than requests x iterations
    assert st["ticks"] < sum(r["launches"] for r in res)
    # requests whose levels never exceeded the per-tick cap ran the same
    # sample ranges as a stand-alone estimate
    same = [(p, t, r) for p, t, r in zip(probs, tols, res) if max(r["N"]) <= 2 ** 24][:5]
    assert same
    for p, t, r in same:
        assert key(r) == key(pkg.mlmc_ap_estimate(p, t))


def test_autotune_keeps_results(tmp_path):
    prob = W.cfg2(eps=0.05, stream_id=61)
    before = pkg.mlmc_ap_estimate(prob, 1e-2)
    cache = str(tmp_path / "tune.json")
    t = pkg.mlmc_ap_autotune(prob, 2e-2, cache)
    assert t["block"] in (64, 128, 256) and t["ppt"] in (1, 2, 4)
    again = pkg.mlmc_ap_autotune(prob, 2e-2, cache)  # served from the cache
    assert again == t
    after = pkg.mlmc_ap_estimate(prob, 1e-2)
    assert key(before) == key(after)


def test_serving_workload_full_trace():
    """The benchmark's serving workload (400 Poisson requests at 200/s, 4 GiB
    budget): every request converges, meets the statistical constraint at its
    own tolerance and lies within 4.5 standard errors of its exact E[Q_L]
    (eps, T and the tolerance differ per request)."""
    arr, probs, tols = W.cfg5_trace(400)
    srv = pkg.mlmc_ap_server_create(hbm_budget_bytes=4 << 30)
    try:
        lat, res = pkg.mlmc_ap_server_run_trace(srv, arr, probs, tols)
    finally:
        pkg.mlmc_ap_server_destroy(srv)
    worst = 0.0
    for p, t, r in zip(probs, tols, res):
        assert r["converged"] and r["var_estimator"] <= 0.5 * t * t * (1 + 1e-12)
        z = abs(r["estimate"] - CF.level_second_moment(p, p["L"])) / math.sqrt(r["var_estimator"])
        worst = max(worst, z)
        assert z <= 4.5, (p, t, r["estimate"])
    lat = sorted(lat)
    print("400 requests: worst |z| %.2f, p50 %.3f ms, p99 %.3f ms" % (
        worst, lat[200] * 1e3, lat[396] * 1e3), flush=True)
