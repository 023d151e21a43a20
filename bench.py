#!/usr/bin/env python3
"""Benchmark of the multilevel asymptotic-preserving Monte Carlo hot path on
one MI355X.

One step = one complete MLMC estimate of E[x_8(T)^2] for the MLMC-AP
workload (x0 ~ N(0,1), Maxwellian equilibrium, eps = 0.01, T = 1, dt0 = 0.5,
M = 2, levels 0..8, RMSE 1e-3, FP32 particle state with FP64 statistics):
warm-up samples on every level, optimal sample numbers, top-ups until the
statistical constraint holds -- every level of an iteration in one persistent
kernel launch (issued directly, the library's default).

Printed: one JSON line.  ``value`` = particle-steps (fine + coarse) per
second over the K timed estimates.  Extra fields: time-to-RMSE of the same
launches replayed from captured hipGraphs, of plain per-level launches and of
plain Monte Carlo at level 8; the estimate on the level set the heuristic
level selection picks; the eps-sweep batch; serving latency; the same
estimate with the kinetic-diffusion scheme (all levels and selected levels);
the roofline of the particle kernel; the FP64 oracle timed on the host cores
on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Roofline of the particle kernels: VALU instruction issue.  MI355X issues one
# wave64 VALU instruction per SIMD every four cycles (16 lanes per cycle), so
# the peak is 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 3.93e13 lane-instructions/s:
# the non-packed FP32 FMA rate (78.6 TFLOP/s) and the FP64 FMA rate alike.
# (The kernels are built without packed FP32, whose 157.3 TFLOP/s does not apply.)
PEAK_LANE_INSTR = 256 * 4 * 16 * 2.4e9

# Per-unit work: VALU lane-instructions per sample of each level of the
# benchmarked workloads, as issued by the built gfx950 persistent kernels
# (unit = one sample of level l, i.e. one fine/coarse pair for l >= 1).
# Measured with rocprofv3 SQ_INSTS_VALU on launches of one size each
# (bench.py --valu-probe); kept with the kernel source hash they were taken on
# in profiles/valu_instructions_per_sample.json.  The long levels agree with
# the static count of the hot loop in the gfx950 assembly (221 instructions
# per four fine steps of an aggregated M = 2 pair, i.e. 55 per fine step;
# level 8 measures 53.4 per fine step including the per-sample work).
VALU_RECORD = os.path.join(ROOT, "profiles", "valu_instructions_per_sample.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def valu_per_sample(scheme):
    """(per-level VALU lane-instructions per sample, record is current)."""
    with open(VALU_RECORD) as f:
        rec = json.load(f)
    return rec[scheme], rec.get("kernel_source_hash") == kernel_source_hash()


def algorithmic_lane_instructions(table, N):
    """VALU lane-instructions of an estimate with N[l] samples at level l."""
    return sum(n * table[l] for l, n in enumerate(N))


def fine_steps(prob, N):
    """Fine-path particle steps of an estimate (coarse steps left out)."""
    n0 = int(round(prob["T"] / prob["dt0"]))
    return sum(n * n0 * prob["M"] ** l for l, n in enumerate(N))


KERNEL_SOURCES = ("kernels.hip", "kernels.hpp", "kd.hpp", "device.hpp", "types.hpp", "stats.hpp",
                  "unit_math.hpp", "plan.hpp")
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "persistent_kernel_hbm_traffic.json")


def exact_second_moment(prob, level):
    """Exact E[x(T)^2] of the splitting scheme at `level` (reported beside the
    estimate; x0 ~ N(a, b^2)): with n steps of the level and its h, s, p, the
    velocity chain has correlation q^d (q = 1 - p) at lag d, so
    E[x^2] = E[x0^2] + n s^2 + h^2 (n + 2 sum_{d=1}^{n-1} (n - d) q^d)."""
    dt = prob["dt0"] / float(prob["M"]) ** level
    n = int(round(prob["T"] / prob["dt0"])) * int(prob["M"]) ** level
    eps = prob["eps"]
    den = eps * eps + dt
    h, s2, q = dt * eps / den, 2.0 * dt * dt / den, 1.0 - dt / den
    lag = sum((n - d) * q ** d for d in range(1, n))
    return prob["x0_a"] ** 2 + prob["x0_b"] ** 2 + n * s2 + h * h * (n + 2.0 * lag)


def kd_exact_second_moment(prob):
    """Exact E[x(T)^2] of the kinetic-diffusion scheme in a homogeneous
    background at every time step: the kinetic value E[x0^2] +
    2 (T - eps^2 (1 - e^{-T/eps^2}))."""
    eps, T = prob["eps"], prob["T"]
    return prob["x0_a"] ** 2 + prob["x0_b"] ** 2 + 2.0 * (T + eps * eps * math.expm1(-T / (eps * eps)))


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2004_04071_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_traffic(tuning):
    """HBM bytes per launch of the particle kernel from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE record, if it was taken on the current
    kernel sources and launch shape; else None."""
    try:
        with open(TRAFFIC_RECORD) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_model():
    """Model name of the host CPU (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(prob, N, seconds):
    """FP64 oracle on the host cores, on the MLMC sample numbers N scaled
    down so the run takes about `seconds`."""
    import oracle
    from oracle import mlmc as OM
    threads = oracle.default_threads()
    # calibrate on a tiny slice
    frac = 1e-4
    for _ in range(6):
        t0 = time.perf_counter()
        steps = 0
        for l, n in enumerate(N):
            k = max(1, int(n * frac))
            oracle.simulate(prob, l, 0, k, threads=threads)
            steps += k * OM.level_cost(prob, l)
        dt = time.perf_counter() - t0
        if dt > 0.5:
            break
        frac *= 4
    frac = min(1.0, frac * seconds / max(dt, 1e-3))
    # passes over the (scaled) sample ranges until `seconds` have elapsed: at
    # frac = 1 one pass is the whole estimate's samples
    t0 = time.perf_counter()
    steps = 0
    passes = 0
    while passes == 0 or time.perf_counter() - t0 < seconds:
        for l, n in enumerate(N):
            k = max(1, int(n * frac))
            oracle.simulate(prob, l, 0, k, threads=threads)
            steps += k * OM.level_cost(prob, l)
        passes += 1
    dt = time.perf_counter() - t0
    return dict(value=steps / dt, unit="particle-steps/s", cores=threads, kind="oracle",
                cpu_model=cpu_model(), host_logical_cpus=os.cpu_count(),
                sample="MLMC-AP eps=0.01 L=8: %d pass(es) over the estimate's sample numbers "
                       "scaled by %.3g (%d particle-steps, %.1f s)" % (passes, frac, steps, dt))


def valu_probe():
    """The launches behind profiles/valu_instructions_per_sample.json (run it
    under rocprofv3 --pmc SQ_INSTS_VALU): per workload and finest level L,
    one persistent launch over levels 0..L with VALU_PROBE_SAMPLES samples at
    every level and the tuning the benchmark times (host-planned direct form,
    so that no device-planned top-up follows the launch); the time-parallel
    path is off so that every sample runs the per-lane loop."""
    import torch
    import paper_2004_04071_amd as pkg
    import workloads as W
    torch.cuda.set_device(0)
    pkg.mlmc_ap_init()
    for name, base in (("ap", W.cfg2()), ("kd", W.cfg_kd())):
        n = VALU_PROBE_SAMPLES[name]
        for L in range(base["L"] + 1):
            r = pkg.mlmc_ap_estimate(dict(base, L=L), 100.0, pkg.options(
                batched=3, n_warmup=n, max_iter=1, tp_max_samples=-1, block=256, ppt=1,
                waves_per_simd=8))
            assert r["launches"] == 1 and r["N"] == [n] * (L + 1)
            print(json.dumps(dict(workload=name, L=L, samples_per_level=n)), flush=True)


VALU_PROBE_SAMPLES = {"ap": 1 << 24, "kd": 1 << 20}
VALU_PROBE_COMMAND = ("rocprofv3 --pmc SQ_INSTS_VALU SQ_WAVES --output-format csv -d <dir> "
                      "-o pmc -- python3 bench.py --valu-probe")


def _counter_per_dispatch(csv_path, counter):
    """(kernel name, value) of `counter` per dispatch, in dispatch order."""
    import csv
    rows = {}
    with open(csv_path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                rows[int(r["Dispatch_Id"])] = (r["Kernel_Name"], float(r["Counter_Value"]))
    return [rows[k] for k in sorted(rows)]


def write_traffic_record(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv):
    """HBM bytes per launch of the particle kernel: FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch) scaled by what they read for a plain copy of known
    size (--copy-probe 256: each copy reads and writes 256 MiB)."""
    copy_bytes = 256.0 * 1024 * 1024
    def factor(path, counter):
        # the three copies (the probe's fill of the source is not a copy)
        vals = [v for name, v in _counter_per_dispatch(path, counter) if "copy" in name.lower()]
        assert len(vals) == 3, vals
        return copy_bytes / (1024.0 * (sum(vals) / len(vals)))
    ff = factor(copy_fetch_csv, "FETCH_SIZE")
    fw = factor(copy_write_csv, "WRITE_SIZE")
    def mean_kib(path, counter):
        vals = [v for name, v in _counter_per_dispatch(path, counter)
                if "persistent_kernel<float" in name]
        return sum(vals) / len(vals), len(vals)
    fk, n = mean_kib(fetch_csv, "FETCH_SIZE")
    wk, _ = mean_kib(write_csv, "WRITE_SIZE")
    rec = {"kernel": "persistent_kernel<float, 1, false>",
           "workload": "MLMC-AP eps=0.01 L=8 RMSE 1e-3 (bench timed region)",
           "kernel_source_hash": kernel_source_hash(),
           "tuning": {"block": 256, "ppt": 1, "waves_per_simd": 8},
           "dispatches": n, "fetch_kib_per_launch": fk, "write_kib_per_launch": wk,
           "fetch_factor": ff, "write_factor": fw,
           "bytes_per_launch": fk * 1024.0 * ff + wk * 1024.0 * fw,
           "commands": ["rocprofv3 --pmc FETCH_SIZE -- python3 bench.py --no-extras "
                        "--no-cpu-baseline --steps 5 --warmup 1 --tuning 256,1,8",
                        "rocprofv3 --pmc WRITE_SIZE -- (the same)",
                        "rocprofv3 --pmc FETCH_SIZE -- python3 bench.py --copy-probe 256",
                        "rocprofv3 --pmc WRITE_SIZE -- python3 bench.py --copy-probe 256"]}
    with open(TRAFFIC_RECORD, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps(rec))


def write_valu_record(csv_path):
    """Per-level VALU lane-instructions per sample from the counters of the
    --valu-probe launches (persistent kernels only, in dispatch order): the
    launch over levels 0..L minus the launch over levels 0..L-1, times 64
    lanes, over the samples per level."""
    import csv
    by_dispatch = {}
    with open(csv_path) as f:
        for r in csv.DictReader(f):
            if "persistent_kernel" in r["Kernel_Name"] and r["Counter_Name"] == "SQ_INSTS_VALU":
                by_dispatch[int(r["Dispatch_Id"])] = (r["Kernel_Name"], float(r["Counter_Value"]))
    launches = [by_dispatch[k] for k in sorted(by_dispatch)]
    rec = {"kernel_source_hash": kernel_source_hash(), "command": VALU_PROBE_COMMAND,
           "unit": "VALU lane-instructions per sample of level l (SQ_INSTS_VALU x 64)",
           "samples_per_level": VALU_PROBE_SAMPLES}
    k = 0
    for name, kernel in (("ap", "persistent_kernel<float, 1, false>"),
                         ("kd", "persistent_kernel<double, 1, true>")):
        prev, per = 0.0, []
        for L in range(9):
            kname, v = launches[k]
            k += 1
            assert kernel in kname, (kname, kernel)
            per.append(round((v - prev) * 64.0 / VALU_PROBE_SAMPLES[name], 2))
            prev = v
        rec[name] = per
        rec[name + "_kernel"] = kernel
    with open(VALU_RECORD, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps(rec))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--serving-requests", type=int, default=2100,
                    help="Poisson requests of the serving trace (the first "
                         "--serving-warmup of them are left out of p50/p99)")
    ap.add_argument("--serving-warmup", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=("ap", "kd"), default="ap",
                    help="kd: time the same estimate with the kinetic-diffusion scheme instead "
                         "(FP64 state; value = KD steps per second; for profiling its kernel)")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the timed estimates (for profiler runs)")
    ap.add_argument("--tuning", default=None,
                    help="block,ppt,waves_per_simd instead of running the autotuner")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (the known-size "
                         "kernel that calibrates the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--valu-probe", action="store_true",
                    help="only run, for each finest level L = 0..8 of the benchmarked "
                         "splitting and KD workloads, one warm-up-only estimate over levels "
                         "0..L with the same sample number everywhere (one persistent launch "
                         "each): differences of SQ_INSTS_VALU between consecutive launches "
                         "give the VALU instructions per sample of level L")
    ap.add_argument("--valu-record", metavar="CSV",
                    help="write profiles/valu_instructions_per_sample.json from the "
                         "rocprofv3 counter CSV of a --valu-probe run (no GPU needed)")
    ap.add_argument("--traffic-record", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH",
                                                          "COPY_WRITE"),
                    help="write profiles/persistent_kernel_hbm_traffic.json from the rocprofv3 "
                         "FETCH_SIZE and WRITE_SIZE CSVs of the benchmark (--no-extras) and of "
                         "--copy-probe 256 (no GPU needed)")
    args = ap.parse_args()
    if args.traffic_record:
        write_traffic_record(*args.traffic_record)
        return
    if args.valu_record:
        write_valu_record(args.valu_record)
        return
    if args.valu_probe:
        valu_probe()
        return
    if args.copy_probe:
        import torch
        n = args.copy_probe * 1024 * 1024 // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4, "copies": 3}), flush=True)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the estimator would shard by sample ranges with "
              "one statistics merge per iteration, which is not implemented across GPUs; "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2004_04071_amd as pkg
    import workloads as W

    torch.cuda.set_device(0)
    pkg.mlmc_ap_init()
    kd_mode = args.workload == "kd"
    prob = W.cfg_kd() if kd_mode else W.cfg2()
    tol = W.CFG2_TOL
    stream = torch.cuda.current_stream()

    if args.tuning:
        b, p_, w = (int(v) for v in args.tuning.split(","))
        tuning = dict(block=b, ppt=p_, waves_per_simd=w)
    else:
        tuning = pkg.mlmc_ap_autotune(prob, tol, None)
    log("tuning", tuning)
    tk = dict(block=tuning["block"], ppt=tuning["ppt"], waves_per_simd=tuning["waves_per_simd"])

    opt = pkg.options(batched=0, **tk)
    P = pkg.as_problem(prob)           # marshalled once, as a serving client would
    hs = stream.cuda_stream
    for _ in range(args.warmup):
        pkg.mlmc_ap_estimate(P, tol, opt, stream=hs)
    torch.cuda.synchronize()
    raw = [pkg.Result() for _ in range(args.steps)]
    t0 = time.perf_counter()
    for r in raw:
        pkg.mlmc_ap_estimate_into(P, tol, opt, r, stream=hs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    results = [pkg.result_dict(r) for r in raw]
    if kd_mode:   # KD steps actually taken (fine + coarse)
        steps_total = sum(int(l["coll_f"]) + int(l["coll_c"]) for r in results for l in r["levels"])
        fine_total = sum(int(l["coll_f"]) for r in results for l in r["levels"])
    else:
        steps_total = sum(r["particle_steps"] for r in results)
        fine_total = sum(fine_steps(prob, r["N"]) for r in results)
    value = steps_total / elapsed
    ms_per = elapsed / args.steps * 1e3
    last = results[-1]
    exact = kd_exact_second_moment(prob) if kd_mode else exact_second_moment(prob, prob["L"])
    log("estimate %.6f exact %.6f sd %.2e N %s" % (last["estimate"], exact,
                                                   math.sqrt(last["var_estimator"]), last["N"]))

    # Dominant kernel: the persistent particle kernel (which also runs a
    # warm-up launch's few long trajectories time-parallel), launched directly
    # so that HIP events on the launch stream time it.  Work = the per-sample
    # table times the samples of every level (the time-parallel schedule of a
    # warm-up's long trajectories is counted as the same per-sample work).
    direct = pkg.mlmc_ap_estimate(prob, tol, pkg.options(batched=2, **tk))
    kern_s = direct["kernel_seconds"]
    launches = direct["launches"]
    table, current = valu_per_sample("kd" if kd_mode else "ap")
    work = algorithmic_lane_instructions(table, direct["N"])
    achieved = work / kern_s
    roofline = dict(bound="alu", achieved=achieved / 1e12, peak=PEAK_LANE_INSTR / 1e12,
                    unit="T VALU lane-instructions/s", frac=achieved / PEAK_LANE_INSTR,
                    traffic=recorded_traffic(tuning) if not kd_mode else None,
                    kernel=("persistent_kernel<double,1,true>" if kd_mode else
                            "persistent_kernel<float,%d,false>" % tuning["ppt"]),
                    avg_launch_ms=kern_s / launches * 1e3, launches=launches,
                    lane_instructions_per_estimate=work, per_unit_record_current=current)
    out = {
        "metric": "particle-steps/s; MLMC time-to-RMSE 1e-3 vs plain MC; p50/p99 request latency",
        "value": value,
        "unit": "KD steps/s" if kd_mode else "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if kd_mode else "f32",
        "data": "synthetic",
        "config": {"workload": ("MLMC-KD eps=0.01 T=1 dt0=0.5 M=2 L=0..8 RMSE=1e-3 x0~N(0,1), "
                                "homogeneous background, FP64 state") if kd_mode else
                               ("MLMC-AP eps=0.01 T=1 dt0=0.5 M=2 L=0..8 RMSE=1e-3 "
                                "x0~N(0,1) Maxwellian, FP32 state / FP64 statistics"),
                   "rmse_tol": tol, "levels": prob["L"] + 1,
                   "particle_steps_per_estimate": last["particle_steps"],
                   "N": last["N"], "tuning": tuning},
        "time_to_rmse_ms": ms_per,
        "fine_steps_per_s": fine_total / elapsed,
        "estimate": last["estimate"],
        "estimate_exact": exact,
        "roofline": roofline,
    }
    if kd_mode:
        out["kernel_ms_per_estimate"] = kern_s * 1e3
    if not args.no_extras and not kd_mode:
        # plain per-level launches (same estimator, one kernel launch per level)
        t0 = time.perf_counter()
        reps = 3
        for _ in range(reps):
            pkg.mlmc_ap_estimate(prob, tol, pkg.options(batched=-1, **tk))
        per_level_ms = (time.perf_counter() - t0) / reps * 1e3
        # plain Monte Carlo at level 8
        t0 = time.perf_counter()
        mc = pkg.mlmc_ap_plain_mc(prob, tol)
        plain_ms = (time.perf_counter() - t0) * 1e3
        # the same persistent launches replayed from captured hipGraphs
        t0 = time.perf_counter()
        for _ in range(reps):
            pkg.mlmc_ap_estimate(prob, tol, pkg.options(batched=1, **tk))
        graph_ms = (time.perf_counter() - t0) / reps * 1e3
        # the same direct launches with every launch planned by the host (no
        # device-planned first top-up)
        hopt = pkg.options(batched=3, **tk)
        hraw = pkg.Result()
        pkg.mlmc_ap_estimate_into(P, tol, hopt, hraw, stream=hs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            pkg.mlmc_ap_estimate_into(P, tol, hopt, hraw, stream=hs)
        torch.cuda.synchronize()
        out["host_planned_time_to_rmse_ms"] = (time.perf_counter() - t0) / args.steps * 1e3
        out["graph_replay_time_to_rmse_ms"] = graph_ms
        out["per_level_launch_time_to_rmse_ms"] = per_level_ms
        out["plain_mc_time_to_rmse_ms"] = plain_ms
        out["plain_mc_particle_steps"] = mc["particle_steps"]
        out["mlmc_speedup_vs_plain_mc"] = plain_ms / ms_per
        out["batched_speedup_vs_per_level"] = per_level_ms / ms_per
        log("per-level %.2f ms, batched %.2f ms (graph replay %.2f ms), plain MC %.2f ms"
            % (per_level_ms, ms_per, graph_ms, plain_ms))

        # the same estimate on the level set the heuristic of Section 5.2 picks
        sopt = pkg.options(batched=0, level_select=pkg.LEVELS_HEURISTIC, **tk)
        pkg.mlmc_ap_estimate(P, tol, sopt, stream=hs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            sel = pkg.mlmc_ap_estimate(P, tol, sopt, stream=hs)
        torch.cuda.synchronize()
        sel_ms = (time.perf_counter() - t0) / reps * 1e3
        out["level_selection"] = dict(levels=sel["level_set"], time_to_rmse_ms=sel_ms,
                                      particle_steps=sel["particle_steps"],
                                      N=[sel["N"][l] for l in sel["level_set"]],
                                      estimate=sel["estimate"],
                                      sd=math.sqrt(sel["var_estimator"]))
        log("level selection", out["level_selection"])

        # the epsilon-adaptive on-line phase of Section 5.3: tolerances
        # tol0 / sqrt(2^r), r = 0..20, ending at the same RMSE target
        R = 20
        sq_opt = pkg.options(batched=0, **tk)
        pkg.mlmc_ap_estimate_sequence(P, tol * 2.0 ** (R / 2), R, sq_opt, stream=hs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sq = pkg.mlmc_ap_estimate_sequence(P, tol * 2.0 ** (R / 2), R, sq_opt, stream=hs)
        torch.cuda.synchronize()
        sq_ms = (time.perf_counter() - t0) * 1e3
        out["tolerance_sequence"] = dict(
            stages=R + 1, tol_first=tol * 2.0 ** (R / 2), tol_last=tol, time_ms=sq_ms,
            particle_steps=sq[-1]["particle_steps"],
            last_stage_particle_steps=sq[-1]["particle_steps"] - sq[-2]["particle_steps"],
            launches=sq[-1]["launches"], estimate=sq[-1]["estimate"],
            sd=math.sqrt(sq[-1]["var_estimator"]),
            level_correction=sq[-1]["levels"][prob["L"]]["mean_dq"],
            level_correction_sd=math.sqrt(sq[-1]["levels"][prob["L"]]["m2_dq"]
                                          / max(sq[-1]["N"][prob["L"]] - 1, 1)
                                          / max(sq[-1]["N"][prob["L"]], 1)))
        log("tolerance sequence", out["tolerance_sequence"])

        # eps sweep: 15 requests in one batched launch per iteration vs one by one
        probs, tols = W.cfg3()
        pkg.mlmc_ap_estimate_batch(probs, tols)
        t0 = time.perf_counter()
        batch = pkg.mlmc_ap_estimate_batch(probs, tols)
        batch_ms = (time.perf_counter() - t0) * 1e3
        t0 = time.perf_counter()
        for p, t in zip(probs, tols):
            pkg.mlmc_ap_estimate(p, t, pkg.options(batched=-1))
        seq_ms = (time.perf_counter() - t0) * 1e3
        out["eps_sweep"] = dict(requests=len(probs), batched_ms=batch_ms,
                                per_level_sequential_ms=seq_ms,
                                particle_steps=sum(b["particle_steps"] for b in batch))

        # serving: Poisson arrivals
        n = args.serving_requests
        arr, sprobs, stols = W.cfg5_trace(n)
        srv = pkg.mlmc_ap_server_create(hbm_budget_bytes=4 << 30)
        try:
            lat, res = pkg.mlmc_ap_server_run_trace(srv, arr, sprobs, stols)
            sstats = pkg.mlmc_ap_server_get_stats(srv)
        finally:
            pkg.mlmc_ap_server_destroy(srv)
        w = min(args.serving_warmup, n - 1)
        lat_sorted = sorted(lat[w:])
        m = len(lat_sorted)
        # makespan: first arrival to the last completion (not the completion
        # of the last-submitted request, which an earlier long one can outlast)
        makespan = max(a + l for a, l in zip(arr, lat)) - arr[0]
        out["serving"] = dict(requests=n, warmup_requests=w, measured_requests=m,
                              rate_per_s=200.0,
                              p50_ms=lat_sorted[m // 2] * 1e3,
                              p99_ms=lat_sorted[min(m - 1, int(math.ceil(0.99 * m)) - 1)] * 1e3,
                              max_ms=lat_sorted[-1] * 1e3,
                              particle_steps=sstats["particle_steps"],
                              makespan_s=makespan,
                              particle_steps_per_s=sstats["particle_steps"] / makespan,
                              ticks=sstats["ticks"],
                              # the trace offers less work than the GPU can do:
                              # time inside ticks, and the rate while in them
                              busy_s=sstats["busy_seconds"],
                              busy_fraction=sstats["busy_seconds"] / makespan,
                              particle_steps_per_busy_s=(sstats["particle_steps"]
                                                         / max(sstats["busy_seconds"], 1e-12)))
        log("serving", out["serving"])

        # the paper's kinetic-diffusion scheme on the same estimate (FP64 state)
        kprob = W.cfg_kd()
        KP = pkg.as_problem(kprob)
        kopt = pkg.options(batched=2, **tk)
        pkg.mlmc_ap_estimate(KP, tol, kopt, stream=hs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kres = [pkg.mlmc_ap_estimate(KP, tol, kopt, stream=hs) for _ in range(reps)]
        torch.cuda.synchronize()
        kd_ms = (time.perf_counter() - t0) / reps * 1e3
        kr = kres[-1]
        kd_steps = sum(int(l["coll_f"]) + int(l["coll_c"]) for l in kr["levels"])
        ktable, kcur = valu_per_sample("kd")
        kwork = algorithmic_lane_instructions(ktable, kr["N"])
        kach = kwork / kr["kernel_seconds"]
        ksopt = pkg.options(batched=2, level_select=pkg.LEVELS_HEURISTIC, **tk)
        pkg.mlmc_ap_estimate(KP, tol, ksopt, stream=hs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ks = pkg.mlmc_ap_estimate(KP, tol, ksopt, stream=hs)
        torch.cuda.synchronize()
        kd_sel_ms = (time.perf_counter() - t0) / reps * 1e3
        out["kd"] = dict(
            workload="MLMC-KD eps=0.01 T=1 dt0=0.5 M=2 L=0..8 RMSE=1e-3 x0~N(0,1), "
                     "homogeneous background, FP64 state",
            time_to_rmse_ms=kd_ms, kernel_ms=kr["kernel_seconds"] * 1e3,
            roofline=dict(bound="alu", achieved=kach / 1e12, peak=PEAK_LANE_INSTR / 1e12,
                          unit="T VALU lane-instructions/s", frac=kach / PEAK_LANE_INSTR,
                          kernel="persistent_kernel<double,1,true>",
                          lane_instructions_per_estimate=kwork,
                          per_unit_record_current=kcur),
            kd_steps=kd_steps, kd_steps_per_s=kd_steps / (kd_ms * 1e-3),
            N=kr["N"], estimate=kr["estimate"],
            estimate_exact=kd_exact_second_moment(kprob),
            sd=math.sqrt(kr["var_estimator"]),
            level_selection=dict(levels=ks["level_set"], time_to_rmse_ms=kd_sel_ms,
                                 N=[ks["N"][l] for l in ks["level_set"]],
                                 estimate=ks["estimate"], sd=math.sqrt(ks["var_estimator"])))
        log("kd", out["kd"])

        # the test case of Section 5: KD in background B1 with a = 10, b = 1000
        # (x(0) = 1, dt_l = 2^-l, QoI E[x(T)], exact value 1 by symmetry), the
        # case of the paper's cost-complexity study; multilevel estimates (all
        # levels, heuristic and cost-optimal level sets) against single-level
        # KDMC at the finest level, at the same RMSE
        bprob = W.cfg_bg(W.BG_B1, 10.0, 1000.0, L=14)
        BP = pkg.as_problem(bprob)
        btol = 1e-4
        bres = {}
        for name, fn, bopt in (
                ("mlmc_all_levels", pkg.mlmc_ap_estimate, pkg.options(batched=2, **tk)),
                ("mlmc_heuristic_levels", pkg.mlmc_ap_estimate,
                 pkg.options(batched=2, level_select=pkg.LEVELS_HEURISTIC, **tk)),
                ("mlmc_optimal_levels", pkg.mlmc_ap_estimate,
                 pkg.options(batched=2, level_select=pkg.LEVELS_OPTIMAL, **tk)),
                # Section 5.3's protocol: 100 warm-up samples on levels 0..tau
                # only, the O(dt^3) profile beyond, the heuristic set
                ("mlmc_section53_protocol", pkg.mlmc_ap_estimate,
                 pkg.options(batched=2, level_select=pkg.LEVELS_HEURISTIC_TAU, n_warmup=100,
                             **tk)),
                ("single_level_kdmc", pkg.mlmc_ap_plain_mc, pkg.options(batched=2, **tk))):
            fn(BP, btol, bopt, stream=hs)
            torch.cuda.synchronize()
            times = []
            for _ in range(3):  # the median of three: single launches here last milliseconds
                t0 = time.perf_counter()
                r = fn(BP, btol, bopt, stream=hs)
                torch.cuda.synchronize()
                times.append((time.perf_counter() - t0) * 1e3)
            bres[name] = dict(time_ms=sorted(times)[1], estimate=r["estimate"],
                              sd=math.sqrt(r["var_estimator"]), levels=r["level_set"],
                              N=[r["N"][l] for l in r["level_set"]],
                              kd_steps=sum(int(l["coll_f"]) + int(l["coll_c"])
                                           for l in r["levels"]),
                              tau=r["tau"], cost_model_steps=r["particle_steps"])
        out["background_b1"] = dict(
            workload="KD, background B1 a=10 b=1000, x(0)=1, T=1, dt_l=2^-l, L=14, "
                     "QoI E[x(T)] (exact 1), RMSE 1e-4",
            exact=1.0, **bres,
            speedup_heuristic_vs_single_level=(bres["single_level_kdmc"]["time_ms"]
                                               / bres["mlmc_heuristic_levels"]["time_ms"]),
            speedup_all_levels_vs_single_level=(bres["single_level_kdmc"]["time_ms"]
                                                / bres["mlmc_all_levels"]["time_ms"]),
            speedup_protocol_vs_single_level=(bres["single_level_kdmc"]["time_ms"]
                                              / bres["mlmc_section53_protocol"]["time_ms"]))
        # the cost complexity of Section 5.3 in the same case: time and KD
        # steps of the protocol's estimate and of single-level KDMC over a
        # sequence of tolerances (each tolerance a fresh estimate after an
        # untimed one, L = 14)
        sweep = []
        for btol_r in (1e-3, 5e-4, 2.5e-4, 1.25e-4, 6.25e-5, 3.125e-5, 1.5625e-5):
            row = dict(rmse_tol=btol_r)
            for name, fn, bopt in (
                    ("protocol", pkg.mlmc_ap_estimate,
                     pkg.options(batched=2, level_select=pkg.LEVELS_HEURISTIC_TAU, n_warmup=100,
                                 **tk)),
                    ("single_level", pkg.mlmc_ap_plain_mc, pkg.options(batched=2, **tk))):
                fn(BP, btol_r, bopt, stream=hs)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = fn(BP, btol_r, bopt, stream=hs)
                torch.cuda.synchronize()
                row[name + "_ms"] = (time.perf_counter() - t0) * 1e3
                row[name + "_kd_steps"] = sum(int(l["coll_f"]) + int(l["coll_c"])
                                              for l in r["levels"])
                row[name + "_estimate"] = r["estimate"]
                row[name + "_sd"] = math.sqrt(r["var_estimator"])
            row["speedup"] = row["single_level_ms"] / row["protocol_ms"]
            row["work_ratio"] = row["single_level_kd_steps"] / row["protocol_kd_steps"]
            sweep.append(row)
        out["background_b1"]["tolerance_sweep"] = sweep
        log("background_b1", out["background_b1"])
    if not args.no_cpu_baseline and not kd_mode:
        out["cpu_baseline"] = cpu_baseline(prob, last["N"], args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
