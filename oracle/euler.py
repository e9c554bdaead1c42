"""2-D Euler system: conserved/primitive variables, equation of state, fluxes.

Follows the system in Sec. 2 (equation "euler 2d equation") with the
ideal-gas energy relation E = p/(gamma-1) + rho |u|^2 / 2 that follows it;
gamma = 1.4 in every test case of the paper.
Conserved vector e = (rho, rho u, rho v, E); arrays carry it on axis 0.
"""
from __future__ import annotations

import numpy as np

GAMMA = 1.4


def prim_to_cons(w: np.ndarray, gamma: float = GAMMA) -> np.ndarray:
    rho, u, v, p = w
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def pressure(e: np.ndarray, gamma: float = GAMMA) -> np.ndarray:
    rho, m, n, E = e
    return (gamma - 1.0) * (E - 0.5 * (m * m + n * n) / rho)


def cons_to_prim(e: np.ndarray, gamma: float = GAMMA) -> np.ndarray:
    rho, m, n, E = e
    return np.stack([rho, m / rho, n / rho, pressure(e, gamma)])


def sound_speed(e: np.ndarray, gamma: float = GAMMA) -> np.ndarray:
    return np.sqrt(gamma * pressure(e, gamma) / e[0])


def fluxes(e: np.ndarray, gamma: float = GAMMA):
    """Return (f_x, f_y), the x- and y-flux vectors of the Euler system."""
    rho, m, n, E = e
    p = pressure(e, gamma)
    u = m / rho
    v = n / rho
    fx = np.stack([m, m * u + p, m * v, u * (E + p)])
    fy = np.stack([n, n * u, n * v + p, v * (E + p)])
    return fx, fy


def mach(e: np.ndarray, gamma: float = GAMMA) -> np.ndarray:
    """Proxy variable Phi(e) = |u| sqrt(rho / (gamma p)) (Sec. 5, item 2)."""
    rho, m, n, _ = e
    speed = np.sqrt(m * m + n * n) / rho
    return speed * np.sqrt(rho / (gamma * pressure(e, gamma)))


def temperature_like(e: np.ndarray, gamma: float = GAMMA) -> np.ndarray:
    """theta = p / ((gamma - 1) rho): the quantity through which the energy
    is filtered (Sec. 5, item 3; reading of relation I-(4) with c_v = 1)."""
    return pressure(e, gamma) / ((gamma - 1.0) * e[0])
