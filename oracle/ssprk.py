"""Strong-stability-preserving Runge-Kutta scheme of order 4.

The paper time-steps with "SSPRK-4" (Sec. 2 and Sec. 5, item 4, citing
Gottlieb 2005).  Reading: the five-stage, fourth-order SSP scheme of
Spiteri & Ruuth in Shu-Osher form; its coefficients are checked against the
eight fourth-order conditions by the test suite.
"""
from __future__ import annotations

import numpy as np

# u1 = u0 + A0 dt L(u0)
A0 = 0.391752226571890
# u2 = B20 u0 + B21 u1 + A1 dt L(u1)
B20, B21, A1 = 0.444370493651235, 0.555629506348765, 0.368410593050371
# u3 = B30 u0 + B32 u2 + A2 dt L(u2)
B30, B32, A2 = 0.620101851488403, 0.379898148511597, 0.251891774271694
# u4 = B40 u0 + B43 u3 + A3 dt L(u3)
B40, B43, A3 = 0.178079954393132, 0.821920045606868, 0.544974750228521
# u5 = C2 u2 + C3 u3 + D3 dt L(u3) + C4 u4 + D4 dt L(u4)
C2, C3, D3, C4, D4 = (0.517231671970585, 0.096059710526147, 0.063692468666290,
                      0.386708617503269, 0.226007483236906)


def butcher():
    """Butcher tableau (a, b, c) equivalent to the Shu-Osher form above,
    obtained by expanding each stage in terms of dt L(u_k)."""
    # Each stage u_k = u0 + dt sum_j a[k, j] L(u_j)
    a = np.zeros((5, 5))
    a[1, 0] = A0
    a[2] = B21 * a[1]; a[2, 1] += A1
    a[3] = B32 * a[2]; a[3, 2] += A2
    a[4] = B43 * a[3]; a[4, 3] += A3
    b = C2 * a[2] + C3 * a[3] + C4 * a[4]
    b[3] += D3
    b[4] += D4
    c = a.sum(axis=1)
    return a, b, c


def stage_times():
    """Fraction of dt at which each stage's output approximates the solution:
    outputs of stages 1..5 (u1..u4, u5)."""
    _, _, c = butcher()
    return np.array([c[1], c[2], c[3], c[4], 1.0])


def step(u0, dt, L, enforce=None):
    """One SSPRK(5,4) step.  ``L(u, k)`` evaluates the spatial operator for
    stage k; ``enforce(u, k)`` applies boundary conditions and inter-patch
    communication to the output of stage k (Alg. 1, stage loop)."""
    enforce = enforce or (lambda u, k: u)
    u1 = enforce(u0 + A0 * dt * L(u0, 0), 0)
    u2 = enforce(B20 * u0 + B21 * u1 + A1 * dt * L(u1, 1), 1)
    L2 = L(u2, 2)
    u3 = enforce(B30 * u0 + B32 * u2 + A2 * dt * L2, 2)
    L3 = L(u3, 3)
    u4 = enforce(B40 * u0 + B43 * u3 + A3 * dt * L3, 3)
    L4 = L(u4, 4)
    u5 = enforce(C2 * u2 + C3 * u3 + D3 * dt * L3 + C4 * u4 + D4 * dt * L4, 4)
    return u5
