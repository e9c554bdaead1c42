"""GPU runs of the wedge tunnel (MI355X, gfx950): the obstacle with C1
corner subpatches at the tip (30-degree obstacle angle) and at the two rear
corners (75 degrees), skewed-affine subpatches on the faces and seeded
lattice subpatches, at the Mach number of the headline configuration, the
initial data smeared in the first step (Alg. 4 at t = 0).

- oracle parity on the small decomposition (h = 1/600, 72 subpatches):
  modal viscosity and filter, two steps, classes equal and the state to
  FP64 rounding;
- the oblique shock off the upper face at Mach 5: its angle against the
  weak branch of the theta-beta-M relation (Sec. 7, equation "deflection");
- the Mach-10 flow to t = 0.06: physical state, attached shock;
- the full-size set (244 subpatches, 1.15e7 points): graph replay equals
  eager launches bit for bit, and one split-BF16 step stays within the
  split-BF16 contraction bound of the FP64 step.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import os  # noqa: E402

import paper_2506_19370_amd as F  # noqa: E402
import workloads as W  # noqa: E402
from oracle import exact, solver as osolver  # noqa: E402

GOLD = os.path.join(os.path.dirname(__file__), "golden", "sdnn_oracle_weights.npz")
M = W.WEDGE_MACH


def _rel(S, O, n):
    scale = np.abs(O.U).max()
    return max(np.abs(S.cons(p) - O.view(O.U, p)).max() for p in range(n)) / scale


def test_wedge_small_matches_oracle():
    specs = W.wedge_tunnel(600, 48, 96, mach=M)
    w = W.wedge_state(specs, quiescent_wake=True, mach=M)
    S = F.Solver(specs, F.SolverParams(fc_d=2, fc_C=27, cfl=0.5, av="modal", filter=True, smear=True))
    for p in range(len(specs)):
        S.set_state(p, w[p])
    O = osolver.Solver(osolver.patches_from_specs(specs),
                       osolver.Params(fc_d=2, fc_C=27, cfl=0.5, av="modal", filter=True, smear=True))
    O.set_prim(w)
    for step in range(2):
        t = S.advance(5, sync=True)
        O.step()
        assert abs(t - O.t) < 1e-12 * O.t
        for p in range(len(specs)):
            assert np.array_equal(S.field(p, "tau0"), O.last_tau[p][0]), (step, p)
            assert np.array_equal(S.field(p, "tau1"), O.last_tau[p][1]), (step, p)
        assert _rel(S, O, len(specs)) < 1e-11, step


def _shock_angle(S, specs, xs, face, rho_mid):
    """Least-squares angle (degrees) of the points above the face where the
    density falls through rho_mid, on vertical lines x = xs."""
    X, Y, R = [], [], []
    for p, s in enumerate(specs):
        act = np.ones(s.shape, bool) if s.mask is None else s.mask
        X.append(s.x[act])
        Y.append(s.y[act])
        R.append(S.field(p, "rho")[act])
    X, Y, R = map(np.concatenate, (X, Y, R))
    h = 1.0 / 600
    ys = []
    for x0 in xs:
        sel = (np.abs(X - x0) < 0.6 * h) & (Y > face(x0) + 2 * h) & (Y < 0.5)
        y, r = Y[sel], R[sel]
        o = np.argsort(y)
        y, r = y[o], r[o]
        above = np.flatnonzero(r >= rho_mid)
        k = above.max()  # last point of the shock layer going up
        y0 = y[k] + (y[k + 1] - y[k]) * (r[k] - rho_mid) / (r[k] - r[k + 1])
        ys.append(y0)
    slope = np.polyfit(xs, ys, 1)[0]
    return np.rad2deg(np.arctan(slope))


def _wedge_run(mach, t_end):
    specs = W.wedge_tunnel(600, 48, 96, mach=mach)
    w = W.wedge_state(specs, quiescent_wake=True, mach=mach)
    blob = np.load(GOLD)["params"]
    S = F.Solver(specs, F.SolverParams(fc_d=2, fc_C=27, cfl=0.5, av="sdnn", filter=True, sdnn_weights=blob,
                                       smear=True))
    for p in range(len(specs)):
        S.set_state(p, w[p])
    t = 0.0
    while t < t_end:
        t = S.advance(5 * 1000, sync=True)  # raises if the state turns non-finite or non-physical
    return S, specs, t


def test_wedge_shock_angle():
    """Small decomposition at Mach 5 run to t = 0.06 (the stream passes the
    face length 1.5 times): the shock off the upper face between 30 % and
    90 % of the face lies within 2 degrees of the inviscid weak-branch angle
    for the face's 15-degree deflection.  (At Mach 10 the shock layer over
    the face, 0.094 of the distance from the tip, is 3 to 10 points high at
    h = 1/600, thinner than the smeared shock: the angle is not resolved
    there; the Mach-10 run below checks the flow stays physical and the
    shock attached.)"""
    mach = 5.0
    S, specs, t = _wedge_run(mach, 0.06)
    geo = W.wedge_geometry(1.0)
    face = lambda x: geo["Yc"] + (x - geo["Xt"]) * np.tan(geo["theta"])
    beta = np.rad2deg(exact.weak_shock_angle(geo["theta"], mach))
    Mn = mach * np.sin(np.deg2rad(beta))
    rho2 = 1.4 * 2.4 * Mn ** 2 / (0.4 * Mn ** 2 + 2.0)
    xs = geo["Xt"] + (geo["Xr"] - geo["Xt"]) * np.linspace(0.3, 0.9, 13)
    ang = _shock_angle(S, specs, xs, face, 0.5 * (1.4 + rho2))
    print(f"Mach {mach}: shock angle {ang:.2f} deg at t = {t:.4f}, theta-beta-M {beta:.2f} deg")
    assert abs(ang - beta) < 2.0


def test_wedge_mach10_long_run():
    """The headline Mach number on the small decomposition to t = 0.06 with
    the SDNN viscosity and the smeared start: the state stays finite and
    physical, and on vertical lines over 50 % .. 90 % of the upper face the
    shock is attached: a compressed layer next to the face (density above
    twice the free stream's) and the free stream restored (3 %) a quarter of
    the face length above the weak-branch shock (the smeared shock reaches
    well above its inviscid position at this resolution)."""
    S, specs, t = _wedge_run(M, 0.06)
    geo = W.wedge_geometry(1.0)
    face = lambda x: geo["Yc"] + (x - geo["Xt"]) * np.tan(geo["theta"])
    beta = exact.weak_shock_angle(geo["theta"], M)
    X, Y, R = [], [], []
    for p, s in enumerate(specs):
        act = np.ones(s.shape, bool) if s.mask is None else s.mask
        X.append(s.x[act])
        Y.append(s.y[act])
        R.append(S.field(p, "rho")[act])
    X, Y, R = map(np.concatenate, (X, Y, R))
    h = 1.0 / 600
    for x0 in geo["Xt"] + (geo["Xr"] - geo["Xt"]) * np.linspace(0.5, 0.9, 5):
        shock = geo["Yc"] + (x0 - geo["Xt"]) * np.tan(beta)
        line = np.abs(X - x0) < 0.6 * h
        layer = line & (Y > face(x0)) & (Y < shock)
        free = line & (Y > shock + 0.25 * (geo["Xr"] - geo["Xt"])) & (Y < 0.5)
        assert R[layer].max() > 2.8, (x0, R[layer].max())
        assert np.abs(R[free] - 1.4).max() < 0.042, (x0, np.abs(R[free] - 1.4).max())


def test_wedge_full_size_graph_and_split_bf16():
    specs = W.wedge_tunnel(mach=M)
    assert 230 <= len(specs) <= 260
    w = W.wedge_state(specs, quiescent_wake=True, mach=M)
    res = {}
    for name, prec, graph in (("graph", "fp64", True), ("eager", "fp64", False), ("bf16x3", "bf16x3", True)):
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            S = F.Solver(specs, F.SolverParams(fc_d=2, fc_C=27, cfl=0.5, av="modal", filter=True, use_graph=graph,
                                               precision=prec, smear=True), stream=stream)
            for p in range(len(specs)):
                S.set_state(p, w[p])
            S.advance(5, sync=True)
            res[name] = [S.cons(p) for p in range(len(specs))]
            if name == "graph":
                S.advance(10, sync=True)  # raises if the state turns non-finite or non-physical
            del S
        torch.cuda.synchronize()
    for p in range(len(specs)):
        assert np.array_equal(res["graph"][p], res["eager"][p]), p
    scale = max(np.abs(r).max() for r in res["graph"])
    err = max(np.abs(a - b).max() for a, b in zip(res["bf16x3"], res["graph"])) / scale
    assert err < 1e-4, err
