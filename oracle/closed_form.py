"""Closed-form moments of the discrete asymptotic-preserving particle scheme.

TEST INFRASTRUCTURE ONLY (pins for the oracle; see ``oracle/__init__.py``).

Scheme at fixed time step dt (unit-variance equilibrium, sigma^2 = 1):
    x_{k+1} = x_k + h v_k + s xi_k,   xi_k ~ N(0,1) independent,
    v_{k+1} = v_k with probability q = 1 - p, else a fresh equilibrium draw,
with h = dt eps/(eps^2+dt), s^2 = 2 dt^2/(eps^2+dt), p = dt/(eps^2+dt) and
v_0 drawn from the equilibrium.  The velocity chain is stationary with
Cov(v_j, v_k) = q^|j-k|, so after n steps

    E[x_n^2] = E[x_0^2] + n s^2 + h^2 (n + 2 sum_{d=1}^{n-1} (n-d) q^d).

Limits used as independent pins:
  * eps -> 0 (diffusion limit): h -> 0, s^2 -> 2 dt, so x_T ~ N(x_0, 2T), the
    heat kernel of d rho/dt = d^2 rho/dx^2;
  * dt -> 0 (kinetic limit): the displacement variance tends to
    2 (T - eps^2 (1 - exp(-T/eps^2))), the unconditional kinetic displacement
    variance the paper gives as the square of its weight beta (eq.
    weights-beta) with collision rate R = 1/eps^2 and velocity variance
    sigma_v^2 = 1/eps^2.
"""
import math

import numpy as np


def level_dt(dt0, M, level):
    return dt0 / float(M) ** level


def scheme_coeffs(eps, dt):
    den = eps * eps + dt
    return dict(h=dt * eps / den, s2=2.0 * dt * dt / den, p=dt / den)


def x0_second_moment(x0_kind, a=0.0, b=0.0):
    """E[x_0^2]: delta at a; normal(a, b^2); density 1+cos(2 pi x) on [0,1]."""
    if x0_kind == 0:
        return a * a
    if x0_kind == 1:
        return a * a + b * b
    if x0_kind == 2:
        return 1.0 / 3.0 + 1.0 / (2.0 * math.pi ** 2)
    raise ValueError(x0_kind)


def x0_mean(x0_kind, a=0.0, b=0.0):
    if x0_kind in (0, 1):
        return a
    return 0.5


def second_moment(eps, dt, n, ex0sq, p=None):
    """Exact E[x_n^2] of the discrete scheme after n steps.  ``p`` overrides
    the collision probability (e.g. the quantised threshold / 2^32)."""
    c = scheme_coeffs(eps, dt)
    q = 1.0 - (c["p"] if p is None else p)
    d = np.arange(1, n, dtype=np.float64)
    corr = float(np.sum((n - d) * q ** d)) if n > 1 else 0.0
    return ex0sq + n * c["s2"] + c["h"] ** 2 * (n + 2.0 * corr)


def second_moment_closed(eps, dt, n, ex0sq):
    """Same quantity with the geometric sum in closed form (for p not tiny)."""
    c = scheme_coeffs(eps, dt)
    q = 1.0 - c["p"]
    S = q * (n * (1.0 - q) - 1.0 + q ** n) / (1.0 - q) ** 2
    return ex0sq + n * c["s2"] + c["h"] ** 2 * (n + 2.0 * S)


def kinetic_limit(eps, T, ex0sq):
    """dt -> 0 limit: E[x_0^2] + 2 (T - eps^2 (1 - exp(-T/eps^2)))."""
    if eps == 0.0:
        return ex0sq + 2.0 * T
    return ex0sq + 2.0 * (T - eps * eps * (-math.expm1(-T / (eps * eps))))


def heat_limit(T, ex0sq):
    return ex0sq + 2.0 * T


def level_second_moment(prob, level):
    """Exact E[Q_l] = E[x^2] at time T for level ``level`` of ``prob``."""
    dt = level_dt(prob["dt0"], prob["M"], level)
    n = int(round(prob["T"] / prob["dt0"])) * int(prob["M"]) ** level
    ex0 = x0_second_moment(prob["x0_kind"], prob.get("x0_a", 0.0), prob.get("x0_b", 0.0))
    return second_moment(prob["eps"], dt, n, ex0)


def two_point_mixture_cdf(x, x0, eps, dt, n):
    """Exact CDF of x_n for velocities +-1 (each with probability 1/2, also at
    collisions), by enumerating all 2^n velocity sequences: given the
    sequence, x_n ~ N(x0 + h sum v, n s^2).  A collision redraws the sign, so
    consecutive velocities agree with probability q + p/2."""
    from scipy.stats import norm
    c = scheme_coeffs(eps, dt)
    h, s2, p = c["h"], c["s2"], c["p"]
    stay = 1.0 - p + 0.5 * p
    flip = 0.5 * p
    # distribution of sum v over sequences: dynamic programming on (sum, last v)
    probs = {(1, 1): 0.5, (-1, -1): 0.5}
    for _ in range(1, n):
        nxt = {}
        for (tot, v), pr in probs.items():
            for nv, t in ((v, stay), (-v, flip)):
                key = (tot + nv, nv)
                nxt[key] = nxt.get(key, 0.0) + pr * t
        probs = nxt
    sums = {}
    for (tot, _), pr in probs.items():
        sums[tot] = sums.get(tot, 0.0) + pr
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    sd = math.sqrt(n * s2)
    for tot, pr in sums.items():
        out += pr * norm.cdf((x - x0 - h * tot) / sd)
    return out
