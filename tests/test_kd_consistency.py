"""Consistency of the coarse KD random numbers (the paper's Section 5.1
check, in a homogeneous background): for fine steps dt = T/2^l and coarse
steps K dt, the aggregated coarse numbers nu~, E~ and chi~ of 1000 pairs
follow N(0,1), Exp(1) and N(0,1) (eq. null_hypothesis), by the
Anderson-Darling distance of eq. anderson (CPU, oracle only)."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as O
from oracle_pins import AD_MAX, anderson_darling

CASES = [(l, K) for l in (2, 5, 8, 11, 14) for K in (2, 4, 8, 16, 32, 64) if 2 ** l >= K]


@pytest.mark.parametrize("level,K", CASES, ids=["l%d_K%d" % c for c in CASES])
def test_coarse_numbers_follow_their_laws(oracle_lib, level, K):
    # dt0 = T and M = 2: level l has dt = T/2^l; the coarse level l - log2 K
    prob = dict(eps=0.1, T=1.0, dt0=1.0, M=2, x0_kind=0, x0_a=0.0, x0_b=0.0, eq_kind=1,
                coupling=1, seed=7, stream_id=1000 + 31 * level + K, scheme=O.SCHEME_KD)
    lc = level - int(round(math.log2(K)))
    rows = np.concatenate([O.kd_coarse_numbers(prob, level, s, coarse_level=lc)[0]
                           for s in range(1000)])
    a_nu = anderson_darling(rows[:, 1], stats.norm.cdf)
    a_e = anderson_darling(rows[:, 2], stats.expon.cdf)
    a_chi = anderson_darling(rows[:, 0], stats.norm.cdf)
    print("l=%d K=%d: %d coarse steps, A^2 nu %.2f E %.2f chi %.2f"
          % (level, K, rows.shape[0], a_nu, a_e, a_chi))
    assert max(a_nu, a_e, a_chi) < AD_MAX
