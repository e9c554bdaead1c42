"""Pins of the oracle's physics, time stepping and closed forms (CPU only)."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import euler, exact, ssprk, solver

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_prim_cons_roundtrip_and_eos():
    rng = np.random.default_rng(0)
    w = np.stack([rng.uniform(0.5, 2, 50), rng.normal(0, 2, 50), rng.normal(0, 2, 50), rng.uniform(0.5, 3, 50)])
    e = euler.prim_to_cons(w)
    assert np.allclose(euler.cons_to_prim(e), w, rtol=1e-14, atol=1e-14)
    # E = p/(gamma-1) + rho |u|^2 / 2 for a hand-computed state
    e1 = euler.prim_to_cons(np.array([[2.0], [3.0], [4.0], [5.0]]))
    assert np.allclose(e1[:, 0], [2.0, 6.0, 8.0, 5.0 / 0.4 + 0.5 * 2.0 * 25.0])


def test_flux_identities():
    rng = np.random.default_rng(1)
    w = np.stack([rng.uniform(0.5, 2, 20), rng.normal(0, 2, 20), rng.normal(0, 2, 20), rng.uniform(0.5, 3, 20)])
    e = euler.prim_to_cons(w)
    fx, fy = euler.fluxes(e)
    rho, u, v, p = w
    assert np.allclose(fx[0], rho * u) and np.allclose(fy[0], rho * v)
    assert np.allclose(fx[1], rho * u * u + p) and np.allclose(fy[2], rho * v * v + p)
    assert np.allclose(fx[2], fy[1])
    # rotational invariance: f_y of a state equals the rotated f_x of the
    # state rotated by -90 degrees
    wr = np.stack([rho, v, -u, p])
    fxr, _ = euler.fluxes(euler.prim_to_cons(wr))
    assert np.allclose(fy[0], fxr[0]) and np.allclose(fy[2], fxr[1]) and np.allclose(fy[1], -fxr[2])
    assert np.allclose(fy[3], fxr[3])


def test_mach_proxy():
    # Mach-M flow state has unit sound speed, so Phi = M (Sec. 7)
    for M in (3.0, 10.0):
        e = euler.prim_to_cons(exact.mach_flow_state(M)[:, None])
        assert abs(euler.mach(e)[0] - M) < 1e-14
        assert abs(euler.sound_speed(e)[0] - 1.0) < 1e-14


def test_ssprk_order_conditions():
    a, b, c = ssprk.butcher()
    assert abs(b.sum() - 1) < 1e-14
    assert abs(b @ c - 1 / 2) < 1e-14
    assert abs(b @ c ** 2 - 1 / 3) < 1e-14
    assert abs(b @ (a @ c) - 1 / 6) < 1e-14
    assert abs(b @ c ** 3 - 1 / 4) < 1e-14
    assert abs((b * c) @ (a @ c) - 1 / 8) < 1e-14
    assert abs(b @ (a @ c ** 2) - 1 / 12) < 1e-14
    assert abs(b @ (a @ (a @ c)) - 1 / 24) < 1e-14
    # Shu-Osher convex combinations
    for s in ((ssprk.B20, ssprk.B21), (ssprk.B30, ssprk.B32), (ssprk.B40, ssprk.B43)):
        assert abs(sum(s) - 1) < 1e-14
    assert abs(ssprk.C2 + ssprk.C3 + ssprk.C4 - 1) < 1e-14


def test_ssprk_fourth_order_on_linear_ode():
    lam = -1.0 + 2.0j
    errs = []
    for n in (20, 40, 80):
        dt = 1.0 / n
        y = np.array([1.0 + 0j])
        for _ in range(n):
            y = ssprk.step(y, dt, lambda u, k: lam * u)
        errs.append(abs(y[0] - np.exp(lam)))
    o = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert (o > 3.8).all() and (o < 4.3).all()


def test_deflection_table():
    g = json.load(open(os.path.join(GOLD, "deflection_table.json")))
    th = np.radians(g["half_angle_deg"])
    for c in g["cases"]:
        b = np.degrees(exact.weak_shock_angle(th, c["mach"]))
        assert abs(b - c["shock_angle_deg"]) <= g["printed_precision_deg"] + 1e-9


def test_sod_exact_star_state():
    g = json.load(open(os.path.join(GOLD, "sod_star_state.json")))
    xi = np.array([0.0, 0.9, 1.0])  # left of / right of the contact (u* = 0.927)
    w = exact.riemann_exact(g["left"], g["right"], xi)
    tol = g["printed_precision"]
    assert abs(w[2, 0] - g["p_star"]) < tol and abs(w[1, 0] - g["u_star"]) < tol
    assert abs(w[0, 0] - g["rho_star_left"]) < tol
    assert abs(w[0, 2] - g["rho_star_right"]) < tol


def test_vortex_is_exact_solution():
    """The vortex solves the Euler system: centred finite-difference residual
    of the closed form vanishes at second order."""
    res = []
    for h in (0.02, 0.01):
        x, y = np.meshgrid(np.linspace(3, 7, 41), np.linspace(3, 7, 41))
        e = lambda xx, yy, t: euler.prim_to_cons(exact.isentropic_vortex(xx, yy, t))
        dt = h
        et = (e(x, y, dt) - e(x, y, -dt)) / (2 * dt)
        fxp, _ = euler.fluxes(e(x + h, y, 0))
        fxm, _ = euler.fluxes(e(x - h, y, 0))
        _, fyp = euler.fluxes(e(x, y + h, 0))
        _, fym = euler.fluxes(e(x, y - h, 0))
        r = et + (fxp - fxm) / (2 * h) + (fyp - fym) / (2 * h)
        res.append(np.abs(r).max())
    assert res[1] < res[0] / 3.5 and res[1] < 1e-3


def test_mach_shock_rankine_hugoniot():
    """Post-shock state conserves mass, momentum and energy fluxes in the
    shock frame."""
    M = 10.0
    w1 = np.array([1.4, 0.0, 0.0, 1.0])
    w2 = exact.mach_shock_state(M)
    s = M * 1.0  # shock speed (sound speed 1)
    e1 = euler.prim_to_cons(w1[:, None])[:, 0]
    e2 = euler.prim_to_cons(w2[:, None])[:, 0]
    f1, _ = euler.fluxes(e1[:, None])
    f2, _ = euler.fluxes(e2[:, None])
    jump = (f2[:, 0] - f1[:, 0]) - s * (e2 - e1)
    assert np.abs(jump).max() < 1e-10 * np.abs(f2).max()


def _vortex_error(n, steps_time):
    specs = W.vortex_box(n)
    S = solver.Solver(solver.patches_from_specs(specs), solver.Params(fc_d=5, fc_C=27),
                      exact=lambda x, y, t: exact.isentropic_vortex(x, y, t))
    S.set_prim([exact.isentropic_vortex(specs[0].x, specs[0].y, 0.0)])
    while S.t < steps_time - 1e-12:
        S.prm.dt_fixed = min(0.25 * 10.0 / (n - 1) / 2.6, steps_time - S.t)
        S.step()
    return np.abs(S.prim(0) - exact.isentropic_vortex(specs[0].x, specs[0].y, S.t)).max()


def test_vortex_convergence():
    e1 = _vortex_error(41, 0.5)
    e2 = _vortex_error(81, 0.5)
    assert e2 < e1 / 8.0, (e1, e2)  # order >= 3 (min(d, 4) expected)
    assert e2 < 1e-4


def test_freestream_preserved_on_curved_patches():
    for specs in (W.curved_patch(), W.annular_sector()):
        S = solver.Solver(solver.patches_from_specs(specs), solver.Params(fc_d=5, fc_C=27))
        w = np.broadcast_to(np.array([1.4, 3.0, 0.5, 1.0])[:, None, None], (4,) + specs[0].shape)
        S.set_prim([w])
        assert not S.grids[0].affine
        L = S.rhs(S.U)
        assert np.abs(L).max() < 1e-10 * np.abs(S.U).max()
