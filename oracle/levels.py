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
