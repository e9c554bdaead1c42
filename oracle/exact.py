"""Closed-form solutions and relations used to pin the oracle.

* Isentropic vortex advected by a uniform flow (standard test; not in the
  paper, used for the single-patch FP64 configuration).
* Oblique-shock deflection relation, equation "deflection" of Sec. 7.
* Mach-M flow and Mach-M shock states, equations "mach_flow_ic" and
  "mach_shock_ic" of Sec. 7 (density taken from the Rankine-Hugoniot
  relation; see the reading on the shock density).
* Exact Riemann solution of the 1-D Euler equations (Toro, ch. 4), own
  implementation, for the Sod problem used as a shock test.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import brentq

from .euler import GAMMA


def isentropic_vortex(x, y, t, beta=5.0, x0=5.0, y0=5.0, u0=1.0, v0=1.0, gamma=GAMMA):
    """Primitive (rho, u, v, p) of the isentropic vortex of strength beta,
    centred at (x0, y0) at t = 0 and carried by the background flow
    (rho, u, v, p) = (1, u0, v0, 1)."""
    dx = x - x0 - u0 * t
    dy = y - y0 - v0 * t
    r2 = dx * dx + dy * dy
    g = np.exp(0.5 * (1.0 - r2))
    du = -beta / (2 * np.pi) * g * dy
    dv = beta / (2 * np.pi) * g * dx
    T = 1.0 - (gamma - 1.0) * beta ** 2 / (8 * gamma * np.pi ** 2) * np.exp(1.0 - r2)
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho ** gamma
    return np.stack([rho, u0 + du, v0 + dv, p])


def deflection_angle(beta_shock, M, gamma=GAMMA):
    """Flow deflection alpha_t for shock angle alpha_d at Mach M, from
    tan(alpha_t/2)... written as tan(theta) = 2 cot(b) (M^2 sin^2 b - 1) /
    (M^2 (gamma + cos 2b) + 2) with theta the wedge half-angle (Sec. 7,
    equation "deflection")."""
    b = beta_shock
    return np.arctan(2.0 / np.tan(b) * (M * M * np.sin(b) ** 2 - 1.0)
                     / (M * M * (gamma + np.cos(2 * b)) + 2.0))


def weak_shock_angle(theta, M, gamma=GAMMA):
    """Weak-branch oblique shock angle for deflection theta (radians)."""
    mu = np.arcsin(1.0 / M)
    bs = np.linspace(mu + 1e-9, np.pi / 2, 20001)
    th = deflection_angle(bs, M, gamma)
    k = int(np.argmax(th))
    return brentq(lambda b: deflection_angle(b, M, gamma) - theta, mu + 1e-12, bs[k])


def mach_flow_state(M, gamma=GAMMA):
    """Uniform Mach-M flow (rho, u, v, p) = (gamma, M, 0, 1): sound speed 1
    (Sec. 7, equation "mach_flow_ic")."""
    return np.array([gamma, M, 0.0, 1.0])


def mach_shock_state(M, rho1=GAMMA, p1=1.0, gamma=GAMMA):
    """Post-shock state of a Mach-M normal shock moving into (rho1, 0, 0, p1)
    (Sec. 7, equation "mach_shock_ic"), from the Rankine-Hugoniot relations."""
    a1 = np.sqrt(gamma * p1 / rho1)
    rho2 = rho1 * (gamma + 1) * M * M / ((gamma - 1) * M * M + 2)
    p2 = p1 * (2 * gamma * M * M - (gamma - 1)) / (gamma + 1)
    u2 = 2.0 / (gamma + 1) * (M - 1.0 / M) * a1
    return np.array([rho2, u2, 0.0, p2])


def riemann_exact(WL, WR, xi, gamma=GAMMA):
    """Exact solution (rho, u, p) of the 1-D Riemann problem at similarity
    coordinates xi = x / t (Toro, ch. 4)."""
    rl, ul, pl = WL
    rr, ur, pr = WR
    al, ar = np.sqrt(gamma * pl / rl), np.sqrt(gamma * pr / rr)

    def fk(p, rk, pk, ak):
        if p > pk:
            A = 2.0 / ((gamma + 1) * rk)
            B = (gamma - 1) / (gamma + 1) * pk
            return (p - pk) * np.sqrt(A / (p + B))
        return 2 * ak / (gamma - 1) * ((p / pk) ** ((gamma - 1) / (2 * gamma)) - 1)

    g = lambda p: fk(p, rl, pl, al) + fk(p, rr, pr, ar) + ur - ul
    ps = brentq(g, 1e-12, 10 * max(pl, pr) + 10)
    us = 0.5 * (ul + ur) + 0.5 * (fk(ps, rr, pr, ar) - fk(ps, rl, pl, al))
    xi = np.asarray(xi, dtype=float)
    out = np.zeros((3,) + xi.shape)
    for idx, s in np.ndenumerate(xi):
        if s <= us:  # left of contact
            if ps > pl:
                SL = ul - al * np.sqrt((gamma + 1) / (2 * gamma) * ps / pl + (gamma - 1) / (2 * gamma))
                if s <= SL:
                    w = (rl, ul, pl)
                else:
                    r = rl * ((ps / pl + (gamma - 1) / (gamma + 1)) / ((gamma - 1) / (gamma + 1) * ps / pl + 1))
                    w = (r, us, ps)
            else:
                SHL = ul - al
                asl = al * (ps / pl) ** ((gamma - 1) / (2 * gamma))
                STL = us - asl
                if s <= SHL:
                    w = (rl, ul, pl)
                elif s > STL:
                    w = (rl * (ps / pl) ** (1 / gamma), us, ps)
                else:
                    c = 2 / (gamma + 1) + (gamma - 1) / ((gamma + 1) * al) * (ul - s)
                    w = (rl * c ** (2 / (gamma - 1)), 2 / (gamma + 1) * (al + (gamma - 1) / 2 * ul + s),
                         pl * c ** (2 * gamma / (gamma - 1)))
        else:
            if ps > pr:
                SR = ur + ar * np.sqrt((gamma + 1) / (2 * gamma) * ps / pr + (gamma - 1) / (2 * gamma))
                if s >= SR:
                    w = (rr, ur, pr)
                else:
                    r = rr * ((ps / pr + (gamma - 1) / (gamma + 1)) / ((gamma - 1) / (gamma + 1) * ps / pr + 1))
                    w = (r, us, ps)
            else:
                SHR = ur + ar
                asr = ar * (ps / pr) ** ((gamma - 1) / (2 * gamma))
                STR = us + asr
                if s >= SHR:
                    w = (rr, ur, pr)
                elif s < STR:
                    w = (rr * (ps / pr) ** (1 / gamma), us, ps)
                else:
                    c = 2 / (gamma + 1) - (gamma - 1) / ((gamma + 1) * ar) * (ur - s)
                    w = (rr * c ** (2 / (gamma - 1)), 2 / (gamma + 1) * (-ar + (gamma - 1) / 2 * ur + s),
                         pr * c ** (2 * gamma / (gamma - 1)))
        out[(slice(None),) + idx] = w
    return out
