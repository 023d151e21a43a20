"""Level selection of the C ABI (host-only entry points) against the
oracle: the heuristic of Section 5.2 on hand-derived cases and random
variance profiles, and the cost-optimal set of eq. level_selection against
plain enumeration (CPU only)."""
import math

import numpy as np
import pytest

from oracle import levels as OL

pkg = pytest.importorskip("paper_2004_04071_amd")


@pytest.fixture(scope="module")
def lib():
    try:
        return pkg.lib()
    except Exception as e:  # pragma: no cover
        pytest.skip("library not built: %s" % e)


# Hand-derived from the algorithm's steps: the first level whose difference
# variance is below its own variance starts the set with the level before it;
# a later level joins when its difference variance is below half of the last
# one taken.
HAND = [
    # V, Vdiff (index 0 unused), selected
    ([1.0] * 9, [0, 1.5, 1.2, 0.8, 0.5, 0.3, 0.1, 0.03, 0.004], [2, 3, 5, 6, 7, 8]),
    ([1.0] * 5, [0, 0.5, 0.2, 0.09, 0.04], [0, 1, 2, 3, 4]),
    ([1.0] * 5, [0, 0.5, 0.4, 0.3, 0.3], [0, 1, 4]),          # L added at the end
    ([1.0] * 4, [0, 2.0, 3.0, 1.5], [3]),                    # no pair pays: level L alone
    ([2.0], [0], [0]),                                       # L = 0
    ([1.0, 1.0, 1.0], [0, 1.0, 0.2], [0, 1, 2]),             # V_{l,l-1} = V_l ends the search
]


@pytest.mark.parametrize("V,Vd,want", HAND)
def test_heuristic_hand_cases(lib, V, Vd, want):
    assert OL.heuristic(V, Vd) == want
    assert pkg.mlmc_ap_select_levels_heuristic(V, Vd) == want


def test_heuristic_random_profiles(lib):
    rng = np.random.default_rng(5)
    for _ in range(300):
        L = int(rng.integers(0, 12))
        V = list(rng.uniform(0.5, 2.0, L + 1))
        # a bump then a decay, as for the kinetic-diffusion levels
        Vd = [0.0] + list(np.exp(rng.normal(0, 1.5, L)) * np.geomspace(2, 1e-3, L))
        assert pkg.mlmc_ap_select_levels_heuristic(V, Vd) == OL.heuristic(V, Vd)


def _random_instance(rng, L):
    V = rng.uniform(0.1, 2.0, L + 1)
    C = np.array([2.0 ** l for l in range(L + 1)])
    Vp = np.zeros((L + 1, L + 1))
    Cp = np.zeros((L + 1, L + 1))
    for i in range(L + 1):
        for j in range(i):
            Vp[i, j] = V[i] * rng.uniform(1e-3, 1.5) * 0.5 ** (i - j > 1)
            Cp[i, j] = C[i] + C[j]
    return V, C, Vp, Cp


def test_optimal_against_enumeration(lib):
    rng = np.random.default_rng(11)
    for _ in range(150):
        L = int(rng.integers(0, 9))
        V, C, Vp, Cp = _random_instance(rng, L)
        best, args = OL.optimal(V, C, Vp, Cp)
        got, cost = pkg.mlmc_ap_select_levels_optimal(V, C, Vp, Cp)
        assert cost == pytest.approx(best, rel=1e-12)
        assert got in args
        assert OL.hierarchy_cost(got, V, C, Vp, Cp) == pytest.approx(best, rel=1e-12)


def test_optimal_special_cases(lib):
    # all pairs useless: level L alone
    V = [1.0, 1.0, 1.0]
    C = [1.0, 2.0, 4.0]
    big = [[0, 0, 0], [9.0, 0, 0], [9.0, 9.0, 0]]
    Cp = [[1, 1, 1], [3.0, 1, 1], [5.0, 6.0, 1]]
    assert pkg.mlmc_ap_select_levels_optimal(V, C, big, Cp)[0] == [2]
    # free corrections: every level pays
    tiny = [[0, 0, 0], [1e-30, 0, 0], [1e-30, 1e-30, 0]]
    levels, cost = pkg.mlmc_ap_select_levels_optimal(V, C, tiny, Cp)
    assert levels[0] == 0 and levels[-1] == 2 and cost == pytest.approx(1.0, rel=1e-9)


def test_selectors_reject_bad_input(lib):
    with pytest.raises(pkg.MlmcApError):
        pkg.mlmc_ap_select_levels_heuristic([1.0, -1.0], [0.0, 0.5])
    with pytest.raises(pkg.MlmcApError):
        pkg.mlmc_ap_select_levels_optimal([1.0, 1.0], [1.0, 0.0], [[0, 0], [1, 0]],
                                          [[1, 1], [1, 1]])


def test_heuristic_sets_are_nested_in_L(lib):
    """Section 5.2: the heuristic is level-adaptive; raising the finest level
    L keeps every level chosen below the old L (the set for L, without the
    level L that is always added, is contained in the set for L + 1)."""
    rng = np.random.default_rng(9)
    for _ in range(200):
        Lmax = int(rng.integers(2, 14))
        V = list(rng.uniform(0.5, 2.0, Lmax + 1))
        Vd = [0.0] + list(np.exp(rng.normal(0, 1.5, Lmax)) * np.geomspace(2, 1e-3, Lmax))
        prev = None
        for L in range(0, Lmax + 1):
            cur = pkg.mlmc_ap_select_levels_heuristic(V[:L + 1], Vd[:L + 1])
            assert cur == OL.heuristic(V[:L + 1], Vd[:L + 1])
            if prev is not None:
                assert set(prev) - {L - 1} <= set(cur), (L, prev, cur)
            prev = cur


def _kd_like_profiles(rng, count):
    for _ in range(count):
        L = int(rng.integers(1, 14))
        V = list(rng.uniform(0.5, 2.0, L + 1))
        Vd = [0.0] + list(np.exp(rng.normal(0, 1.5, L)) * np.geomspace(2, 1e-3, L))
        yield V, Vd


def test_heuristic_set_properties(lib):
    """What the description of Section 5.2 fixes about the set, checked on
    the library's sets: it opens with the adjacent pair (l-1, l) at the first
    l whose difference is no more variable than level l; past that pair every
    level taken (but the closing L) at least halves the difference variance of
    the level taken before it, and no level left out would have; L closes it;
    with no such pair the set is {L}."""
    rng = np.random.default_rng(21)
    for V, Vd in _kd_like_profiles(rng, 400):
        L = len(V) - 1
        got = pkg.mlmc_ap_select_levels_heuristic(V, Vd)
        assert got[-1] == L and got == sorted(set(got))
        opening = [l for l in range(1, L + 1) if Vd[l] <= V[l]]
        if not opening:
            assert got == [L]
            continue
        first = opening[0]
        assert got[:2] == [first - 1, first]
        last = Vd[first]
        for k in range(first + 1, L + 1):
            if k in got and (k != L or Vd[k] < 0.5 * last):
                assert Vd[k] < 0.5 * last, (k, got)
                last = Vd[k]
            else:
                assert k == L or Vd[k] >= 0.5 * last, (k, got)


def test_heuristic_cost_is_never_below_the_optimum(lib):
    """Eq. level_selection's optimum is a lower bound on the cost of any set
    that ends at L, the heuristic's included (pair variances of a model with
    independent level increments, Var[Q_i - Q_j] = sum of the adjacent ones
    between; costs 2^i and 2^i + 2^j)."""
    rng = np.random.default_rng(22)
    for V, Vd in _kd_like_profiles(rng, 200):
        L = len(V) - 1
        C = [2.0 ** l for l in range(L + 1)]
        Vp = [[sum(Vd[j + 1:i + 1]) if i > j else 0.0 for j in range(L + 1)]
              for i in range(L + 1)]
        Cp = [[C[i] + C[j] if i > j else 1.0 for j in range(L + 1)] for i in range(L + 1)]
        h = pkg.mlmc_ap_select_levels_heuristic(V, Vd)
        _, best = pkg.mlmc_ap_select_levels_optimal(V, C, Vp, Cp)
        assert OL.hierarchy_cost(h, V, C, Vp, Cp) >= best * (1 - 1e-12)
