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
    ("kick_sum_unnormalised", "kick = sum_xi / sqrt((double)Mb);", "kick = sum_xi;"),
    ("aggregate_norm_wrong", "sqrt((double)Mb * F.s * F.s + F.h * F.h * den)",
     "sqrt((double)Mb * F.s * F.s + F.h * den)"),
    ("coarse_uses_fine_drift", "xc = xc + C.h * vc + C.s * kick;", "xc = xc + F.h * vc + C.s * kick;"),
    ("coarse_uses_fine_kick_std", "xc = xc + C.h * vc + C.s * kick;", "xc = xc + C.h * vc + F.s * kick;"),
    ("block_boundary_misaligned", "(n % (uint64_t)Mb) == (uint64_t)(Mb - 1)",
     "(n % (uint64_t)Mb) == 0"),
    ("block_sum_not_reset", "sum_xi = 0.0; vel_num = 0.0;", "vel_num = 0.0;"),
    ("coarse_velocity_not_updated", "if (chit) { vc = vf; cc++; }", "if (chit) { cc++; }"),
    ("cosine_icdf_sign", "double F = mid + sin(2.0 * M_PI * mid) / (2.0 * M_PI);",
     "double F = mid - sin(2.0 * M_PI * mid) / (2.0 * M_PI);"),
    ("normal_x0_ignores_std", "x0 = P->x0_a + P->x0_b * nc;", "x0 = P->x0_a + nc * 0.5;"),
    ("velocity_not_resampled", "vf = v_new;", "vf = vf;"),
    ("coarse_threshold_linearised", "-expm1(log1p(-pc) / (double)M)", "(pc / (double)M)"),
    ("block_min_not_reset", "            min_word = 0xFFFFFFFFu;\n", "\n"),
    ("aggregate_draw_counts_its_collision_step",
     "have_draw = 1; last_nu = v_new; last_uses = 0.0;",
     "have_draw = 1; last_nu = v_new; last_uses = 1.0;"),
    ("aggregate_unweighted_velocity", "vel_num += last_uses * last_nu;", "vel_num += last_nu;"),
    ("aggregate_last_draw_never_in_kick", "if (have_draw && !chit) {", "if (0) {"),
    ("aggregate_last_draw_always_in_kick", "if (have_draw && !chit) {", "if (have_draw) {"),
    ("nonadjacent_block_is_M",
     "const int Mb = coarse ? (int)llround(pow((double)P->M, (double)(l - P->coarse_level))) : 1;",
     "const int Mb = coarse ? P->M : 1;"),
]


# Mistakes in the kinetic-diffusion scheme; these run the KD pins only.
KD_MUTANTS = [
    ("kd_diffusion_missing_2", "double d2 = 2.0 * sigma * sigma / (R * R) * kd_f(y)",
     "double d2 = sigma * sigma / (R * R) * kd_f(y)"),
    ("kd_advection_mean_dropped", "double a = mu * theta + dv", "double a = dv"),
    ("kd_advection_rate_inverted", "double a = mu * theta + dv * (-expm1(-y)) / R;",
     "double a = mu * theta + dv * (-expm1(-y)) * R;"),
    ("kd_f_sign", "return 2.0 * (e - 1.0) + y * (e + 1.0);", "return 2.0 * (e - 1.0) + y * (e - 1.0);"),
    ("kd_g_series_coefficient", "(ldexp(1.0, m) - 2.0 * (double)m)", "(ldexp(1.0, m) - (double)m)"),
    ("kd_g_direct_sign", "return 1.0 - 2.0 * y * e - e * e;", "return 1.0 - 2.0 * y * e + e * e;"),
    ("kd_flight_rate_inverted", "tf = 0.0, tauf = E / R;", "tf = 0.0, tauf = E * R;"),
    ("kd_theta_full_step", "double theta = t_next - cfine;                /* eq. diffusive-time */",
     "double theta = dtf;"),
    ("kd_step_grid_ceil", "return floor(c / dt);", "return ceil(c / dt);"),
    ("kd_chi_not_normalised", "double chi_c = den > 0.0 ? num / sqrt(den) : 0.0;",
     "double chi_c = den > 0.0 ? num / den : 0.0;"),
    ("kd_nu_update_initial", "double nu_c = nu_f;", "double nu_c = nu;"),
    ("kd_one_fine_step_per_window", "} while (!(kd_step_of(cfine, dtf) + 1.0 > end_c_fine));",
     "} while (0);"),
    ("kd_alpha_includes_own_flight", "if (!first) {", "if (1) {"),
    ("kd_nonadjacent_block_is_M",
     "const double Mb = coarse ? (double)llround(pow((double)P->M, (double)(l - P->coarse_level))) : 1.0;",
     "const double Mb = coarse ? (double)P->M : 1.0;"),
    ("kd_beta_over_theta", "kd_h(R * theta_p));", "kd_h(R * theta));"),
    ("kd_alpha_without_zeta_shift", "alpha = (tauf + zeta_prev) * sigma;", "alpha = tauf * sigma;"),
    ("kd_alpha_pairs_next_velocity", "num += alpha * nu_f;", "num += alpha * nu_next;"),
    ("kd_zeta_full_phase", "double zeta = -expm1(-y) / R;", "double zeta = theta;"),
    ("kd_exponential_from_wrong_word", "*E_next = -log(oracle_uniform(w[2]));",
     "*E_next = -log(oracle_uniform(w[0]));"),
]


# Mistakes in the KD scheme in the backgrounds of Section 5; these run the
# background pins only.
BG_MUTANTS = [
    ("bg_kink_ignored", "if ((x - 1.0) * (xe - 1.0) < 0.0) {            /* crosses the kink */",
     "if (0) {"),
    ("bg_b1_rate_not_symmetric", "if (g->kind == BG_B1) return g->b * (g->a * fabs(u) + 1.0);",
     "if (g->kind == BG_B1) return g->b * (g->a * fmax(u, 0.0) + 1.0);"),
    ("bg_flight_frozen_rate", "double lo = 0.0, hi = E / g->b;\n    if (!(E > 0.0)) return 0.0;",
     "double lo = 0.0, hi = E / g->b;\n    if (!(E > 0.0) || 1) return E / bg_rate(g, x);"),
    ("bg_epsilon_not_reduced", "double E_c = Ef - bg_rate_integral(g, xf, vf, tc - tf);",
     "double E_c = Ef;"),
    ("bg_epsilon_reduced_along_coarse", "double E_c = Ef - bg_rate_integral(g, xf, vf, tc - tf);",
     "double E_c = Ef - bg_rate_integral(g, xc, vf, tc - tf) * 0.5;"),
    ("bg_fine_steps_beyond_T_kept", "if (cfine >= T && !fine_done) {", "if (0) {"),
    ("bg_trapezoid_half_missing", "return 0.5 * t * (bg_rate(g, x) + bg_rate(g, xe));",
     "return t * bg_rate(g, x);"),
]


@pytest.fixture(scope="module")
def source():
    with open(os.path.join(ROOT, "oracle", "oracle.c")) as f:
        return f.read()


def _run_mutant(source, tmp_path, name, old, new, extra, first_of=None):
    """first_of = n: the anchor occurs n times (the same line in the KD
    functions of the homogeneous background and of the Section 5
    backgrounds) and only its first occurrence, in the homogeneous one, is
    mutated; otherwise it must occur exactly once."""
    if first_of is None:
        assert source.count(old) == 1, "mutation anchor must occur exactly once: %r" % old
        mutated = source.replace(old, new)
    else:
        assert source.count(old) == first_of, (old, source.count(old))
        mutated = source.replace(old, new, 1)
    src = tmp_path / "oracle_mut.c"
    src.write_text(mutated)
    lib = tmp_path / "liboracle_mut.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC",
                           "-w", str(src), "-o", str(lib), "-lm"])
    env = dict(os.environ, ORACLE_LIB_PATH=str(lib),
               PYTHONPATH=os.pathsep.join([ROOT, os.environ.get("PYTHONPATH", "")]))
    out = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "oracle_pins.py"), "--first"]
                         + extra,
                         env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr[-2000:]
    failed = json.loads(out.stdout.strip().splitlines()[-1])
    assert failed, "mutant %s passed every pin" % name


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(source, tmp_path, name, old, new):
    _run_mutant(source, tmp_path, name, old, new, [])


@pytest.mark.parametrize("name,old,new", KD_MUTANTS, ids=[m[0] for m in KD_MUTANTS])
def test_kd_mutant_is_caught(source, tmp_path, name, old, new):
    n = source.count(old)
    _run_mutant(source, tmp_path, name, old, new, ["--kd"], first_of=n if n == 2 else None)


@pytest.mark.parametrize("name,old,new", BG_MUTANTS, ids=[m[0] for m in BG_MUTANTS])
def test_bg_mutant_is_caught(source, tmp_path, name, old, new):
    _run_mutant(source, tmp_path, name, old, new, ["--bg"])
