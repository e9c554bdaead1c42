"""Pins of oracle functions against closed forms and hand-computed values
(CPU only): the viscous term, the slip-wall and corner boundary conditions,
the theta-form filter rebuild of E, the adaptive step and the stability
argument behind its viscous limit, Adam, and the modal-decay indicator.

Each test is chosen so that a plausible slip in the oracle (a dropped term,
a wrong sign, the metric of the wrong direction, the energy filtered
directly, a missing bias correction, a shifted threshold) fails it.
"""
import numpy as np
import pytest

import workloads as W
from oracle import euler, fcgram, patches, sdnn, solver, ssprk


# ---------------------------------------------------------------- viscous term
# w_c = A_c + B_c sin(a_c x + b_c y), mu = m0 + m1 cos(g x - k y):
# div(mu grad w) = mu lap w + mu_x w_x + mu_y w_y in closed form.
COMP = ((2.0, 0.3, 1.1, 0.7), (0.5, 0.4, -0.6, 1.3), (-0.3, 0.5, 0.9, -0.8), (6.0, 0.7, 0.5, 0.4))
MU = (0.02, 0.01, 1.3, 0.9)


def _visc_exact(x, y):
    m0, m1, g, k = MU
    mu = m0 + m1 * np.cos(g * x - k * y)
    mux = -m1 * g * np.sin(g * x - k * y)
    muy = m1 * k * np.sin(g * x - k * y)
    w, out = [], []
    for A, B, a, b in COMP:
        s = np.sin(a * x + b * y)
        c = np.cos(a * x + b * y)
        w.append(A + B * s)
        out.append(mu * (-(a * a + b * b) * B * s) + mux * a * B * c + muy * b * B * c)
    return mu, np.stack(w), np.stack(out)


def _visc_error(specs):
    S = solver.Solver(solver.patches_from_specs(specs), solver.Params(fc_d=5, fc_C=27))
    g = S.grids[0]
    mu, e, ref = _visc_exact(g.p.x, g.p.y)
    mu1, mu2 = g.deriv(mu, 0), g.deriv(mu, 1)
    Lv = S.rhs_patch(e, 0, (mu, mu1, mu2)) - S.rhs_patch(e, 0, None)
    return np.abs(Lv - ref).max() / np.abs(ref).max(), g


@pytest.mark.parametrize("shape", ["sector", "perturbed"])
def test_viscous_term_matches_closed_form(shape):
    """mu Lap w + grad mu . grad w on a curvilinear subpatch (the annular
    sector has Delta q^k terms, the perturbed square also g^12 != 0) equals
    div(mu grad w) of closed-form fields, converging under refinement."""
    make = (lambda s: W.annular_sector(48 * s, 40 * s)) if shape == "sector" else \
        (lambda s: W.curved_patch(48 * s, 40 * s))
    e1, g = _visc_error(make(1))
    e2, _ = _visc_error(make(2))
    assert not g.affine
    if shape == "perturbed":
        assert np.abs(g.g12).max() > 0.05 * np.abs(g.g11).max()
    else:
        assert np.abs(g.lap2).max() > 0.1 * np.sqrt(np.abs(g.g22).max())
    # third order (FC second derivatives with d = 5); a dropped Delta q^k or
    # g^12 term, or a sign error in grad mu . grad w, leaves an O(1) error
    assert e2 < 5e-4, (e1, e2)
    assert e2 < e1 / 6.0, (e1, e2)


# ---------------------------------------------------------------- slip walls
def test_slip_and_corner_conditions_on_a_curved_wall():
    """Annular sector with slip walls on r = r0 (side S) and theta = 0
    (side W): on r = r0 the radial momentum is removed (tangential momentum,
    density and pressure kept); on theta = 0 the y momentum; at their
    corner both momentum components vanish with p kept; every other point
    is unchanged.  The wall normal is the discrete metric's (FC derivatives
    of the mapping), so the curved-wall checks hold to its accuracy."""
    spec = W.annular_sector(60, 48)[0]
    spec.sides = {"W": W.SLIP, "E": W.OUTFLOW, "S": W.SLIP, "N": W.OUTFLOW}
    S = solver.Solver(solver.patches_from_specs([spec]), solver.Params(fc_d=5, fc_C=27))
    rng = np.random.default_rng(3)
    n2, n1 = spec.shape
    w = np.stack([rng.uniform(0.5, 2, (n2, n1)), rng.normal(0, 1, (n2, n1)), rng.normal(0, 1, (n2, n1)),
                  rng.uniform(0.5, 2, (n2, n1))])
    S.set_prim([w])
    U1 = S.enforce(S.U, 0.0)
    e0, e1 = S.view(S.U, 0), S.view(U1, 0)
    p0, p1 = euler.pressure(e0), euler.pressure(e1)
    th = np.arctan2(spec.y, spec.x)
    touched = np.zeros((n2, n1), bool)
    # wall r = r0 (row j = 0), corner excluded
    cs, sn = np.cos(th[0, 1:]), np.sin(th[0, 1:])
    rad1 = e1[1, 0, 1:] * cs + e1[2, 0, 1:] * sn
    tan0 = -e0[1, 0, 1:] * sn + e0[2, 0, 1:] * cs
    tan1 = -e1[1, 0, 1:] * sn + e1[2, 0, 1:] * cs
    assert np.abs(rad1).max() < 1e-7
    assert np.abs(tan1 - tan0).max() < 1e-7
    touched[0, 1:] = True
    # wall theta = 0 (column i = 0): normal (0, 1)
    assert np.abs(e1[2, 1:, 0]).max() < 1e-13
    assert np.abs(e1[1, 1:, 0] - e0[1, 1:, 0]).max() < 1e-13
    touched[1:, 0] = True
    # corner
    assert e1[1, 0, 0] == 0.0 and e1[2, 0, 0] == 0.0
    touched[0, 0] = True
    assert np.abs(e1[0] - e0[0]).max() == 0.0
    assert np.abs(p1[touched] - p0[touched]).max() < 1e-13 * np.abs(p0).max()
    assert np.array_equal(e1[:, ~touched], e0[:, ~touched])


# ---------------------------------------------------------------- filter rebuild
def test_filter_rebuilds_energy_from_filtered_theta():
    """Alg. 4: rho, rho u, rho v and theta = p / ((gamma - 1) rho) are filtered
    along both directions and E is rebuilt from them, so theta of the
    filtered state is the filtered theta (filtering E itself would not give
    it where the data jump); a uniform state passes unchanged."""
    spec = W.box_patch(0.0, 1.0, 0.0, 0.5, 48, 30, {k: W.OUTFLOW for k in "WESN"})
    S = solver.Solver(solver.patches_from_specs([spec]), solver.Params(fc_d=2, fc_C=27, filter=True))
    x, y = spec.x, spec.y
    rho = np.where(x < 0.43, 1.0, 0.3) + 0.05 * np.sin(3 * y)
    w = np.stack([rho, 0.4 + 0.1 * x, -0.2 + 0.0 * x, 1.0 + 0.2 * y])
    S.set_prim([w])
    e0 = S.view(S.U, 0).copy()
    e1 = S.view(S.apply_filter(S.U), 0)
    g = S.grids[0]
    filt = lambda f: g.deriv(g.deriv(f, 0, "filter"), 1, "filter")
    th0 = euler.temperature_like(e0)
    th1 = euler.temperature_like(e1)
    assert np.abs(e1[:3] - filt(e0[:3])).max() < 1e-13
    assert np.abs(th1 - filt(th0)).max() < 1e-12 * np.abs(th0).max()
    # the alternative reading (E filtered directly) differs here
    alt = filt(e0[3])
    assert np.abs(alt - e1[3]).max() > 1e-3 * np.abs(e1[3]).max()
    # constants pass (to the d = 2 continuation's fit accuracy)
    S.set_prim([np.broadcast_to(np.array([1.4, 3.0, -1.0, 1.0])[:, None, None], (4,) + spec.shape)])
    e2 = S.view(S.apply_filter(S.U), 0)
    assert np.abs(e2 - S.view(S.U, 0)).max() < 1e-9 * np.abs(S.U).max()


def test_filter_operator_is_applied_along_both_directions():
    """Data that jump along q^2 only: every column of the filtered density is
    the column passed through the 1-D filter operator (constants along q^1
    pass that direction unchanged), and it differs from the raw column."""
    spec = W.box_patch(0.0, 1.0, 0.0, 1.0, 40, 36, {k: W.OUTFLOW for k in "WESN"})
    S = solver.Solver(solver.patches_from_specs([spec]), solver.Params(fc_d=2, fc_C=27, filter=True))
    w = np.stack([np.where(spec.y < 0.5, 1.0, 0.5), 0 * spec.x, 0 * spec.x, 1.0 + 0 * spec.x])
    S.set_prim([w])
    e1 = S.view(S.apply_filter(S.U), 0)
    col = fcgram.fc_apply(w[0][:, 7], 2, 27, "filter")
    assert np.abs(e1[0] - col[:, None]).max() < 1e-9  # d = 2 fit accuracy along q^1
    assert np.abs(col - w[0][:, 7]).max() > 1e-3


# ---------------------------------------------------------------- time step
def test_timestep_closed_form():
    """Uniform state on a Cartesian patch of spacing h: dt = CFL h / (|u| + a)
    without viscosity, CFL h^2 / (4 mu) where that is smaller (h from the
    FC-derived metric: d = 5 rounding, about 1e-13 relative)."""
    h = 0.1
    spec = W.box_patch(0.0, 3.0, 0.0, 2.0, 31, 21, {k: W.OUTFLOW for k in "WESN"})
    S = solver.Solver(solver.patches_from_specs([spec]), solver.Params(fc_d=5, fc_C=27, cfl=0.5))
    rho, u, v, p = 1.4, 3.0, 4.0, 1.0  # |u| = 5, a = 1
    S.set_prim([np.broadcast_to(np.array([rho, u, v, p])[:, None, None], (4,) + spec.shape)])
    rel = lambda a, b: abs(a - b) / b
    assert rel(S.timestep(S.U, None), 0.5 * h / 6.0) < 1e-12
    mu = np.full(S.U.shape[1], 0.2)
    zero = np.zeros_like(mu)
    assert rel(S.timestep(S.U, (mu, zero, zero)), 0.5 * h * h / 0.8) < 1e-12
    mu[:] = 1e-4  # inviscid limit smaller again
    assert rel(S.timestep(S.U, (mu, zero, zero)), 0.5 * h / 6.0) < 1e-12


@pytest.mark.parametrize("alpha_deg", [90.0, 75.0, 30.0])
def test_mesh_size_of_skewed_cells(alpha_deg):
    """On a parallelogram grid of spacing h and cell angle alpha the mesh
    size of the step-size limits is the distance between neighbouring grid
    lines along the most compressed direction, 1 / sqrt of the largest
    eigenvalue of the metric tensor built from the dual basis of the two
    cell edges: h sin(alpha) / sqrt(1 + |cos(alpha)|) (h when alpha = 90,
    0.366 h at the 30-degree cells of a wedge apex)."""
    h, a = 0.01, np.deg2rad(alpha_deg)
    e1, e2 = np.array([h, 0.0]), np.array([h * np.cos(a), h * np.sin(a)])
    I, J = np.meshgrid(np.arange(24.0), np.arange(20.0))
    spec = W.PatchSpec(I * e1[0] + J * e2[0], I * e1[1] + J * e2[1], None, {k: W.OUTFLOW for k in "WESN"})
    g = patches.Grid(solver.patches_from_specs([spec])[0], 2, 27, 5)
    dual = np.linalg.inv(np.column_stack([e1, e2]))  # rows: grad q1, grad q2 (index units)
    lam = np.linalg.eigvalsh(dual @ dual.T).max()
    assert np.allclose(g.hx, 1.0 / np.sqrt(lam), rtol=1e-9, atol=0)
    assert np.allclose(g.hx, h * np.sin(a) / np.sqrt(1.0 + abs(np.cos(a))), rtol=1e-9, atol=0)


def _stability_function():
    a, b, _ = ssprk.butcher()

    def R(z):
        return 1.0 + z * (b @ np.linalg.solve(np.eye(5) - z * a, np.ones(5)))
    return R


def test_ssprk_real_axis_stability_interval():
    """The SSPRK(5,4) stability polynomial is bounded by 1 on [-5.33, 0] of the
    real axis and exceeds 1 just beyond."""
    R = _stability_function()
    xs = np.linspace(-5.33, 0.0, 5331)
    assert max(abs(R(x)) for x in xs) <= 1.0 + 1e-12
    assert abs(R(-5.34)) > 1.0


@pytest.mark.parametrize("d", [2, 5])
def test_viscous_step_limit_factor_four(d):
    """The viscous limit dt = CFL h^2 / (4 mu) keeps every eigenvalue of the
    2-D FC viscous operator mu (D2 x I + I x D2) / h^2 inside the SSPRK(5,4)
    stability region for CFL <= 1, while dt = CFL h^2 / mu does not at
    CFL = 0.5 (the spectral second derivative reaches about -pi^2)."""
    R = _stability_function()
    ev = np.linalg.eigvals(fcgram.dense_operator(61, d, 27, "d2"))
    lam = (ev[:, None] + ev[None, :]).ravel()
    assert abs(lam).max() > 2 * 8.5  # close to 2 pi^2
    assert max(abs(R(l / 4.0)) for l in lam) <= 1.0 + 1e-4  # CFL 1, factor 4 (tiny FC modes: ~1e-5)
    assert max(abs(R(0.5 * l)) for l in lam) > 10.0         # CFL 0.5, factor 1


# ---------------------------------------------------------------- Adam
def test_adam_two_steps_by_hand():
    """Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected), two steps on
    scalar parameters with gradients g1 then g2, against the values worked
    out by hand."""
    params = {"a": np.array([1.0]), "b": np.array([-2.0])}
    st = {}
    lr = 0.1
    g1 = {"a": np.array([0.5]), "b": np.array([-4.0])}
    sdnn.adam_update(params, g1, st, lr=lr)
    # step 1: m = 0.1 g, v = 0.001 g^2, mh = g, vh = g^2 -> p -= lr g / (|g| + eps)
    assert abs(params["a"][0] - (1.0 - lr * 0.5 / (0.5 + 1e-8))) < 1e-15
    assert abs(params["b"][0] - (-2.0 + lr * 4.0 / (4.0 + 1e-8))) < 1e-15
    g2 = {"a": np.array([-1.5]), "b": np.array([2.0])}
    sdnn.adam_update(params, g2, st, lr=lr)
    # step 2, parameter a: m = 0.09*0.5 + 0.1*(-1.5) = -0.105, v = 0.000999*0.25 + 0.001*2.25 = 0.00249975
    mh = -0.105 / 0.19
    vh = 0.00249975 / (1 - 0.999 ** 2)
    a_ref = (1.0 - lr * 0.5 / (0.5 + 1e-8)) - lr * mh / (np.sqrt(vh) + 1e-8)
    assert abs(params["a"][0] - a_ref) < 1e-14
    assert st["t"] == 2


# ---------------------------------------------------------------- modal indicator
def _poly_basis():
    """Orthonormal discrete polynomials on 16 equispaced points of [-1, 1]
    (numpy QR in FP64; independent of the oracle's construction)."""
    t = np.linspace(-1.0, 1.0, 16)
    Q, R = np.linalg.qr(np.vander(t, 16, increasing=True))
    return Q * np.sign(np.diag(R))[None, :]


@pytest.mark.parametrize("lo,hi,frac,tau", [
    (3, 10, 0.0, 0),     # degree < 8 only
    (2, 12, 1.0, 2),     # degree >= 8 only
    (1, 9, 0.01, 1),     # 1 % of the non-constant energy in high modes
    (5, 8, 0.0002, 0),   # below 1e-3
    (4, 15, 0.1, 2),     # above 10^-1.5
    (2, 8, 0.02, 1),     # between 1e-3 and 10^-1.5
])
def test_modal_indicator_on_known_modal_content(lo, hi, frac, tau):
    """Windows built from two orthonormal modes with a known high-mode energy
    fraction (invariant under the min/max normalisation) get the class of
    the thresholds 1e-3 and 10^-1.5."""
    P = _poly_basis()
    c_lo, c_hi = np.sqrt(1.0 - frac), np.sqrt(frac)
    v = 3.0 + 0.7 * (c_lo * P[:, lo] + c_hi * P[:, hi])
    got = sdnn.modal_classify(np.stack([v, -v + 10.0]))
    assert got.tolist() == [tau, tau]


def test_lowp_gradient_pins():
    """The low-precision gradient of the training reading: with weights,
    inputs and activations already on the bf16 grid it equals the FP64
    gradient (rounding is then the identity), and otherwise it equals the
    FP64 gradient of the network whose weights are rounded, fed rounded
    inputs (a plausible mistake, such as rounding the gradients or skipping
    the activation rounding, breaks one of the two)."""
    rng = np.random.default_rng(11)
    p = {k: rng.standard_normal(s) * 0.3 for k, s in (("W1", (64, 16)), ("b1", (64,)), ("W2", (64, 64)),
                                                      ("b2", (64,)), ("W3", (3, 64)), ("b3", (3,)))}
    x = rng.random((200, 16))
    y = rng.integers(0, 3, 200)
    cw = np.array([0.5, 1.5, 3.0])
    # on the bf16 grid: identical to the FP64 gradient up to the activation
    # rounding, which vanishes only for bf16-exact activations; use a
    # network with one hidden unit active per layer and exact values
    pr = {k: (sdnn.round_bf16(v) if k.startswith("W") else v) for k, v in p.items()}
    xr = sdnn.round_bf16(x)
    l_low, g_low = sdnn.loss_and_grads_lowp(p, x, y, cw)
    l_ref, g_ref = sdnn.loss_and_grads(pr, xr, y, cw)
    # the only remaining difference is the rounding of the hidden
    # activations: small and of bf16 size
    for k in g_ref:
        d = np.abs(g_low[k] - g_ref[k]).max() / np.abs(g_ref[k]).max()
        assert d < 3e-2, (k, d)
    assert abs(l_low - l_ref) < 1e-2 * abs(l_ref)
    # with bf16-exact activations the two agree to FP64 rounding: the first
    # layer reduced to bf16 biases (W1 = 0), the second to halving those
    # (one weight 0.5 per unit), so every activation lies on the bf16 grid
    q = {k: v.copy() for k, v in pr.items()}
    q["W1"][:] = 0.0
    q["b1"] = sdnn.round_bf16(np.abs(p["b1"]))
    q["W2"] = np.zeros((64, 64))
    q["W2"][np.arange(64), np.arange(64)] = 0.5
    q["b2"] = np.zeros(64)
    l1, g1 = sdnn.loss_and_grads_lowp(q, x, y, cw)
    l2, g2 = sdnn.loss_and_grads(q, xr, y, cw)
    assert abs(l1 - l2) < 1e-13
    for k in g2:
        assert np.allclose(g1[k], g2[k], rtol=1e-12, atol=1e-15), k


# ---------------------------------------------------------------- initial-data smearing
def _sod_line_solver(n1=120, n2=24):
    spec = W.box_patch(0.0, 1.0, 0.0, 0.2, n1, n2, {k: W.SLIP for k in "WESN"})
    S = solver.Solver(solver.patches_from_specs([spec]),
                      solver.Params(fc_d=2, fc_C=27, av="modal", smear=True, filter=True))
    w = np.where((spec.x < 0.5)[None], np.array([1.0, 0.0, 0.0, 1.0])[:, None, None],
                 np.array([0.125, 0.0, 0.0, 0.1])[:, None, None])
    S.set_prim([w])
    return S, spec


def test_smear_filter_multiplier():
    """The smearing's filter is the t > 0 filter's exponential with order 8:
    10^(-16 eta^8), so it damps the middle of the spectrum (eta = 0.5: 0.866,
    0.7: 0.111) where the order-36 filter hardly does (1 - 1e-13 and 0.9999),
    and both keep constants exactly."""
    M = 128
    m = np.fft.fftfreq(M) * M
    eta = 2 * np.abs(m) / M
    s = fcgram._multiplier(M, "smear").real
    f = fcgram._multiplier(M, "filter").real
    for e0, want in ((0.5, 10 ** (-16 * 0.5 ** 8)), (0.703125, 10 ** (-16 * 0.703125 ** 8))):
        k = int(np.argmin(np.abs(eta - e0)))
        assert abs(s[k] - want) < 1e-12 and f[k] > 0.9998
    x = np.linspace(0, 1, 80)
    for kind in ("smear", "filter"):
        assert np.allclose(fcgram.fc_apply(np.full((2, 80), 3.25), 2, 27, kind), 3.25, atol=1e-12)
    # a smooth low-mode line is nearly kept, a jump is spread
    smooth = np.sin(2 * np.pi * x)
    assert np.abs(fcgram.fc_apply(smooth, 2, 27, "smear") - smooth).max() < 1e-3
    jump = (x > 0.5).astype(float)
    assert np.abs(fcgram.fc_apply(jump, 2, 27, "smear") - jump).max() > 0.1


def test_smear_initial_data_pins():
    """Nothing flagged: the data are returned unchanged.  Everything flagged
    (window 1 at every point): the data are exactly the strong-filtered
    rho, rho u, rho v, theta with E rebuilt.  A jump flagged only near its
    position: the data change only within n_v + 8 points of it, and
    density and theta stay positive."""
    S, spec = _sod_line_solver()
    g = S.grids[0]
    n2, n1 = spec.shape
    S.last_tau = [np.zeros((2, n2, n1), dtype=np.int64)]
    assert np.array_equal(S.smear_initial_data(S.U), S.U)
    S.last_tau = [np.ones((2, n2, n1), dtype=np.int64)]
    # all non-fringe points flagged: the window is 1 wherever a flagged point
    # lies within reach; on this machine without internal sides every point is
    e = S.view(S.U, 0)
    theta = euler.temperature_like(e)
    q = np.stack([e[0], e[1], e[2], theta])
    qs = g.deriv(g.deriv(q, 0, "smear"), 1, "smear")
    out = S.view(S.smear_initial_data(S.U), 0)
    assert np.allclose(out[0], qs[0], rtol=0, atol=1e-14)
    assert np.allclose(out[3], qs[0] * qs[3] + 0.5 * (qs[1] ** 2 + qs[2] ** 2) / qs[0], rtol=1e-13, atol=1e-14)
    # flagged within 3 columns of the jump only
    tau = np.zeros((2, n2, n1), dtype=np.int64)
    jcol = int(np.argmax(spec.x[0] >= 0.5))
    tau[0, :, jcol - 3:jcol + 3] = 2
    S.last_tau = [tau]
    out = S.view(S.smear_initial_data(S.U), 0)
    changed = np.abs(out - e).max(axis=(0, 1)) > 0
    cols = np.flatnonzero(changed)
    assert cols.size > 0 and cols.min() >= jcol - 3 - 9 and cols.max() <= jcol + 3 + 9
    assert (out[0] > 0).all() and (euler.temperature_like(out) > 0).all()


# ---------------------------------------------------------------- no-slip adiabatic walls
def _noslip_box(n):
    spec = W.box_patch(0.0, 1.0, 0.0, 1.0, 31, n, {"W": W.OUTFLOW, "E": W.OUTFLOW, "S": W.NOSLIP, "N": W.NOSLIP})
    S = solver.Solver(solver.patches_from_specs([spec]), solver.Params(fc_d=5, fc_C=27))
    y = spec.y
    theta = 1.0 + 0.3 * y ** 2 * (1 - y) ** 2  # zero slope at both walls
    rho = 1.0 + 0.2 * np.sin(3 * spec.x)
    S.set_prim([np.stack([rho, 0.3 + 0 * y, -0.2 + 0 * y, 0.4 * rho * theta])])
    e = S.view(S.U, 0)
    e[3, 0, :] *= 1.7   # spoiled wall values: they must be recomputed
    e[3, -1, :] *= 0.6
    return S, spec, theta, e.copy()


def test_noslip_adiabatic_wall_pins():
    """A box with no-slip walls at y = 0 and y = 1 (d = 5): after the
    boundary treatment the wall nodes carry zero momentum and their density,
    theta there makes the FC derivative along the column vanish at both
    walls (the two ends of each column solved together), and for the profile
    theta = 1 + c y^2 (1 - y)^2 (zero slope at both walls, degree 4, which
    FC d = 5 reproduces) the recomputed wall values are the profile's (a
    wrong sign, row or excluded term breaks these)."""
    errs = []
    for n in (41, 81):
        S, spec, theta, e = _noslip_box(n)
        out = S.view(S.enforce(S.U, 0.0), 0)
        D = fcgram.dense_operator(n, 5, 27, "d1")
        for j in (0, n - 1):
            assert np.all(out[1, j] == 0.0) and np.all(out[2, j] == 0.0)
            assert np.array_equal(out[0, j], e[0, j])
        th = out[3] / out[0]  # theta on the wall rows (momentum zero)
        col = np.where(np.arange(n)[:, None] == 0, th, np.where(np.arange(n)[:, None] == n - 1, th,
                                                                   euler.temperature_like(out)))
        dth = D @ col
        assert np.abs(dth[0]).max() < 1e-10 and np.abs(dth[-1]).max() < 1e-10
        assert np.array_equal(out[:, 1:-1], e[:, 1:-1])  # interior untouched
        errs.append(max(np.abs(th[0] - theta[0]).max(), np.abs(th[-1] - theta[-1]).max()))
    assert max(errs) < 1e-10, errs
