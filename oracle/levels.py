"""Level selection (Section 4.2, eq. level_selection; Section 5.2, Algorithm
"Heuristic level selection approach").

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* ``heuristic``: the algorithm's steps in order, with two readings: the
  scan for further levels starts after the first selected pair (the printed
  loop starts at level 0, where V_{0,-1} does not exist), and level L is
  always added (the estimator targets E[Q_L]); if no level qualifies the set
  is {L}.
* ``optimal``: eq. level_selection by plain enumeration of every subset of
  {0..L} that contains L.
* ``warmup_depth`` and ``extrapolate``: the off-line part of Section 5.3
  (warm-up of the levels with dt_l down to about the mean free time, the
  O(dt^3) rate beyond it).
"""
import itertools
import math


def heuristic(V, Vdiff):
    L = len(V) - 1
    if L == 0:
        return [0]
    l = 1
    while l <= L and Vdiff[l] > V[l]:
        l += 1
    if l > L:
        return [L]
    chosen = [l - 1, l]
    vmin = Vdiff[l]
    for k in range(l + 1, L + 1):
        if Vdiff[k] < vmin / 2:
            chosen.append(k)
            vmin = Vdiff[k]
    if chosen[-1] != L:
        chosen.append(L)
    return chosen


def hierarchy_cost(levels, V, C, Vpair, Cpair):
    """sqrt(V_{l_1} C_{l_1}) + sum_j sqrt(V_{l_j,l_{j-1}} C_{l_j,l_{j-1}})."""
    cost = math.sqrt(V[levels[0]] * C[levels[0]])
    for a, b in zip(levels[1:], levels[:-1]):
        cost += math.sqrt(Vpair[a][b] * Cpair[a][b])
    return cost


def optimal(V, C, Vpair, Cpair):
    """(minimum cost, list of every minimising level set)."""
    L = len(V) - 1
    best, arg = math.inf, []
    for r in range(L + 1):
        for head in itertools.combinations(range(L), r):
            levels = list(head) + [L]
            c = hierarchy_cost(levels, V, C, Vpair, Cpair)
            if c < best * (1 - 1e-12):
                best, arg = c, [levels]
            elif c <= best * (1 + 1e-12):
                arg.append(levels)
    return best, arg


def warmup_depth(prob):
    """Section 5.3: the warm-up runs the levels 0..tau, tau the level whose
    step dt_tau = dt0 M^-tau is nearest (in log scale) to the mean free time
    1/R; R is the constant b of the Section 5 backgrounds, 1/eps^2 in the
    diffusive scaling.  At least one difference is measured (tau >= 1) and
    none beyond L (tau = 0 if L = 0)."""
    L = int(prob["L"])
    if L <= 0:
        return 0
    if int(prob.get("background", 0)) != 0:
        R = float(prob["bg_b"])
    else:
        R = 1.0 / (prob["eps"] * prob["eps"])
    t = math.log(prob["dt0"] * R) / math.log(prob["M"])
    if not t < L:
        return L
    return max(1, min(L, int(math.floor(t + 0.5))))


def extrapolate(V, Vdiff, tau, M, L):
    """Section 5.3: the profile of levels 0..L from the warm-up's levels
    0..tau.  Beyond tau the difference variance follows the asymptotic rate
    O(dt^3): V_{l,l-1} = V_{tau,tau-1} (dt_l / dt_tau)^3, and the level
    variance is taken as V_tau (the level variances converge with l).
    Returns (V, Vdiff) of length L + 1."""
    Vo = [float(V[l]) if l <= tau else float(V[tau]) for l in range(L + 1)]
    Vd = [float(Vdiff[l]) if l <= tau else
          float(Vdiff[tau]) / math.pow(M, 3.0 * (l - tau)) for l in range(L + 1)]
    return Vo, Vd
