"""Consistency of the coarse KD random numbers (the paper's Section 5.1, on
the CPU oracle): for fine steps dt = T/2^l and coarse steps K dt, the first
1000 aggregated coarse numbers nu~, E~ and chi~ follow N(0,1), Exp(1) and
N(0,1) (eq. null_hypothesis) by the Anderson-Darling test of eq. anderson at
the paper's 1 % level.  Over many cells some rejections happen by chance even
for exact laws, so the bar is on their number: at most 4 of the 90 tests of
each background (binomial(90, 0.01) exceeds 4 with probability 0.002), and no
A^2 beyond the 1e-4 level.  The GPU harness (tests/test_gpu_consistency.py)
runs the paper's full table on the device's own numbers."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as O
from oracle_pins import AD_CRIT_1PCT, ad_pvalue, anderson_darling

LEVELS = (2, 5, 8, 11, 14)
KS = (2, 4, 8, 16, 32, 64)


def cell_problem(level, K, background):
    """Fine step 2^-l, coarse step K 2^-l, as (dt0, M, level 1, coarse level 0)."""
    p = dict(eps=0.1, T=1.0, dt0=K * 2.0 ** -level, M=K, x0_kind=0, x0_a=1.0, x0_b=0.0,
             eq_kind=1, coupling=1, seed=7, stream_id=1000 + 31 * level + K, scheme=O.SCHEME_KD)
    if background:
        p.update(background=O.BG_B1, bg_a=10.0, bg_b=1000.0)
    return p


def first_numbers(prob, n=1000):
    rows, s = [], 0
    while sum(r.shape[0] for r in rows) < n:
        if prob.get("background", 0):
            rows.append(O.kd_bg_phases(prob, 1, s, coarse_level=0)[1])
        else:
            rows.append(O.kd_coarse_numbers(prob, 1, s, coarse_level=0)[0])
        s += 1
    return np.concatenate(rows)[:n]


def test_ad_pvalue_reproduces_published_critical_values():
    """Case 0 (fully specified law) critical values of the AD statistic."""
    for a2, p in ((1.933, 0.10), (2.492, 0.05), (3.070, 0.025), (3.857, 0.01)):
        assert abs(ad_pvalue(a2) - p) < 0.05 * p


@pytest.mark.parametrize("background", [False, True], ids=["homogeneous_eps0.1", "B1_a10_b1000"])
def test_coarse_numbers_follow_their_laws(oracle_lib, background):
    rejected, worst = [], 1.0
    for level in LEVELS:
        for K in KS:
            rows = first_numbers(cell_problem(level, K, background))
            a2 = (anderson_darling(rows[:, 1], stats.norm.cdf),
                  anderson_darling(rows[:, 2], stats.expon.cdf),
                  anderson_darling(rows[:, 0], stats.norm.cdf))
            print("l=%2d K=%2d: A^2 nu %.3f E %.3f chi %.3f" % ((level, K) + a2))
            for name, a in zip(("nu", "E", "chi"), a2):
                worst = min(worst, ad_pvalue(a))
                if a >= AD_CRIT_1PCT:
                    rejected.append((level, K, name, a))
    print("rejected at 1 %%: %s; smallest p %.3g" % (rejected, worst))
    assert len(rejected) <= 4
    assert worst > 1e-4
