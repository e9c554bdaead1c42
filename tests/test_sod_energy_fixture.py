"""The energy-conservation fixture (Sec. 7.2.2) against its closed form: the
exact mean energy of the Sod data in a closed box is the area-weighted mean
of E = p / (gamma - 1) + rho |u|^2 / 2 of the two states, and the lattice
initial data of the workload converge to it."""
import json
import os

import numpy as np

import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden", "sod_reflect_energy.json")


def _energy(prim, gamma):
    rho, u, v, p = prim
    return p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)


def test_exact_mean_energy_closed_form():
    g = json.load(open(GOLD))
    xs = g["interface_x"] / g["domain"][0]
    mean = xs * _energy(g["left"], g["gamma"]) + (1 - xs) * _energy(g["right"], g["gamma"])
    assert abs(mean - g["exact_mean_energy"]) < 1e-15
    assert abs(g["reported_mean_energy"] - g["exact_mean_energy"]) <= g["reported_band"]


def _lattice_mean_energy(h_index):
    specs = W.sod_reflect(h_index)
    w = W.sod_state(specs)
    cols = []
    for s, wp, (c0, c1) in zip(specs, w, W.sod_reflect_cores(h_index)):
        X0 = int(round(s.x[0, 0] * h_index))
        cols.append(_energy(wp, 1.4)[:, c0 - X0:c1 - X0])
    E = np.concatenate(cols, axis=1)
    ny, nx = E.shape
    wx = np.ones(nx); wx[[0, -1]] = 0.5
    wy = np.ones(ny); wy[[0, -1]] = 0.5
    return (wy[:, None] * wx[None, :] * E).sum() / ((nx - 1) * (ny - 1)), nx


def test_workload_covers_the_box_once():
    for hidx in (200, 400):
        specs = W.sod_reflect(hidx)
        cores = W.sod_reflect_cores(hidx)
        assert cores[0][0] == 0 and cores[-1][1] == hidx + 1
        assert all(a[1] == b[0] for a, b in zip(cores, cores[1:]))
        for s, (c0, c1) in zip(specs, cores):
            X = np.rint(s.x[0] * hidx).astype(int)
            assert X[0] <= c0 and X[-1] >= c1 - 1  # the core lies inside the subpatch
        assert abs(specs[0].y.max() - 0.25) < 1e-15 and abs(specs[-1].x.max() - 1.0) < 1e-15


def test_lattice_initial_energy_converges():
    g = json.load(open(GOLD))
    # the jump sits on a lattice node (right state there): the trapezoid rule
    # misses half a cell of the left state, (E_l - E_r) h / 2 over the unit length
    for hidx in (200, 400, 800):
        m, nx = _lattice_mean_energy(hidx)
        expect = g["exact_mean_energy"] - 0.5 * (2.5 - 0.25) / hidx
        assert abs(m - expect) < 1e-12, (hidx, m, expect)
