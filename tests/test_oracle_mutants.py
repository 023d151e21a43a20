"""Plants plausible mistakes in a copy of the oracle and checks that the pins
catch every one of them (CPU only; the real oracle source is never edited).

Each mutant is one textual substitution in ``oracle/oracle.c``; the copy is
compiled into a temporary directory and the pins run in a subprocess that
loads it through ORACLE_LIB_PATH.
"""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = [
    ("philox_multiplier", "0xD2511F53u * (uint64_t)x0", "0xD2511F57u * (uint64_t)x0"),
    ("philox_no_key_bump", "k0 += 0x9E3779B9u;", "k0 += 0u;"),
    ("uniform_shift", "(double)(w >> 9)", "(double)(w >> 10)"),
    ("box_muller_angle", "double theta = 2.0 * M_PI * u2;", "double theta = 2.0 * M_PI * u1;"),
    ("box_muller_radius", "sqrt(-2.0 * log(u1))", "sqrt(-log(u1))"),
    ("kick_std_missing_2", "c.s = sqrt(2.0 * c.dt * c.dt / denom);", "c.s = sqrt(c.dt * c.dt / denom);"),
    ("collision_prob_swapped", "c.p = c.dt / denom;", "c.p = eps * eps / denom;"),
    ("drift_missing_eps", "c.h = c.dt * eps / denom;", "c.h = c.dt / denom;"),
    ("level_dt_shifted", "c.dt = dt0 / pow((double)M, (double)l);",
     "c.dt = dt0 / pow((double)M, (double)(l + 1));"),
    ("coarse_any_collision", "int chit = ((uint64_t)min_word < thr_c2);",
     "int chit = ((uint64_t)min_word < F.thr);"),
    ("coarse_threshold_unadjusted", "int chit = ((uint64_t)min_word < thr_c2);",
     "int chit = ((uint64_t)min_word < C.thr);"),
    ("kick_sum_unnormalised", "kick = sum_xi / sqrt((double)P->M);", "kick = sum_xi;"),
    ("aggregate_norm_wrong", "sqrt((double)P->M * F.s * F.s + F.h * F.h * den)",
     "sqrt((double)P->M * F.s * F.s + F.h * den)"),
    ("coarse_uses_fine_drift", "xc = xc + C.h * vc + C.s * kick;", "xc = xc + F.h * vc + C.s * kick;"),
    ("coarse_uses_fine_kick_std", "xc = xc + C.h * vc + C.s * kick;", "xc = xc + C.h * vc + F.s * kick;"),
    ("block_boundary_misaligned", "(n % (uint64_t)P->M) == (uint64_t)(P->M - 1)",
     "(n % (uint64_t)P->M) == 0"),
    ("block_sum_not_reset", "sum_xi = 0.0; vel_num = 0.0;", "vel_num = 0.0;"),
    ("coarse_velocity_not_updated", "if (chit) { vc = vf; cc++; }", "if (chit) { cc++; }"),
    ("cosine_icdf_sign", "double F = mid + sin(2.0 * M_PI * mid) / (2.0 * M_PI);",
     "double F = mid - sin(2.0 * M_PI * mid) / (2.0 * M_PI);"),
    ("normal_x0_ignores_std", "x0 = P->x0_a + P->x0_b * nc;", "x0 = P->x0_a + nc * 0.5;"),
    ("velocity_not_resampled", "vf = v_new;", "vf = vf;"),
    ("coarse_threshold_linearised", "-expm1(log1p(-pc) / (double)M)", "(pc / (double)M)"),
    ("block_min_not_reset", "            min_word = 0xFFFFFFFFu;\n", "\n"),
]


@pytest.fixture(scope="module")
def source():
    with open(os.path.join(ROOT, "oracle", "oracle.c")) as f:
        return f.read()


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(source, tmp_path, name, old, new):
    assert source.count(old) == 1, "mutation anchor must occur exactly once: %r" % old
    src = tmp_path / "oracle_mut.c"
    src.write_text(source.replace(old, new))
    lib = tmp_path / "liboracle_mut.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC",
                           "-w", str(src), "-o", str(lib), "-lm"])
    env = dict(os.environ, ORACLE_LIB_PATH=str(lib),
               PYTHONPATH=os.pathsep.join([ROOT, os.environ.get("PYTHONPATH", "")]))
    out = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "oracle_pins.py"), "--first"],
                         env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr[-2000:]
    failed = json.loads(out.stdout.strip().splitlines()[-1])
    assert failed, "mutant %s passed every pin" % name
