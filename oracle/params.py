"""Parameter criteria of the paper, written out plainly — TEST INFRASTRUCTURE ONLY.

Each function states one printed criterion of Mirjalili, Ivey & Mani (arXiv:1803.01262).
u stands for the advection speed the criterion names (|u| in 1D, |u|_max or the largest
velocity component in several dimensions).
"""
from __future__ import annotations

import math


def euler_amplification(alpha: float, beta: float, kdx: float) -> float:
    """|sigma| of Eq. 5: forward Euler applied to the advective rewrite (Eq. 2) of Eq. 1,
    with alpha = (u+gamma) dt/dx and beta = 2 gamma eps / ((u+gamma) dx)."""
    return abs(complex(1.0 - alpha * beta * (1.0 - math.cos(kdx)), -alpha * math.sin(kdx)))


def alpha_bound_eq6(beta: float, kdx: float) -> float:
    """Right-hand side of Eq. 6: the largest stable alpha at wavenumber k."""
    c, s = math.cos(kdx / 2.0), math.sin(kdx / 2.0)
    return beta / (c * c + beta * beta * s * s)


def alpha_bound_eq7(beta: float) -> float:
    """Eq. 7: the bound over all wavenumbers, min(1/beta, beta)."""
    return min(1.0 / beta, beta)


def dt_mod_1d(dx: float, gamma: float, eps: float, u: float) -> float:
    """Eq. 8: min(dx^2 / (2 gamma eps), 2 gamma eps / (u + gamma)^2)."""
    return min(dx * dx / (2.0 * gamma * eps), 2.0 * gamma * eps / (u + gamma) ** 2)


def crossover_eps_over_dx(gamma_over_u: float) -> float:
    """Eq. 9 / Eq. 17 / Eq. 35: eps/dx on the crossover line, (gamma/u + 1) / (2 gamma/u)."""
    return (gamma_over_u + 1.0) / (2.0 * gamma_over_u)


def dt_mod_max_eq10(dx: float, u: float, gamma: float) -> float:
    """Eq. 10: the largest stable step, reached on the crossover line: dx / (u + gamma)."""
    return dx / (u + gamma)


def margin_eq17(eps: float, dx: float, gamma: float, umax: float) -> float:
    """eps/dx minus the Eq. 17 threshold built from |u|_max (>= 0: bounded regime)."""
    return eps / dx - crossover_eps_over_dx(gamma / umax)


def margin_eq24(eps: float, dx: float, gamma: float, comp_max: float) -> float:
    """eps/dx minus the relaxed threshold of Eqs. 23-24, built from the largest component."""
    return eps / dx - crossover_eps_over_dx(gamma / comp_max)


def dt_max(scheme: str, dims: int, dx: float, gamma: float, eps: float) -> float:
    """Eqs. 25-28: diffusion-limited step for Euler, RK2, RK3 (Wray) and RK4 in D_f dims."""
    base = dx * dx / (gamma * eps)
    return {"euler": base / (2 * dims), "rk2": base / (2 * dims),
            "rk3": 2.51 * base / (4 * dims), "rk4": 2.79 * base / (4 * dims)}[scheme]


def dt_rk4_2d_eq31(dx: float, gamma: float, eps: float) -> float:
    """Eq. 31: 2.79 dx^2 / (8 gamma eps)."""
    return 2.79 * dx * dx / (8.0 * gamma * eps)


def dt_rk4_2d_eq32(dx: float, umax: float, vmax: float, gamma: float) -> float:
    """Eq. 32: mixed advective-diffusive step used below the crossover line."""
    return 2.83 * dx / (umax + vmax + 2.0 * gamma)
