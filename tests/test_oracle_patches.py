"""Pins of the oracle's patch geometry, communication and viscosity (CPU)."""
import numpy as np
import pytest

import workloads as W
from oracle import overlap, patches, sdnn, solver, viscosity


def test_l_grid_bookkeeping():
    """Relations of the L parameter-space discretization (Sec. 3.2.2): with
    r preliminary squares per arm of n1 points, N = r (n1 + 1) - 1, each
    arm has N + 2 n_v points, there are 3 r^2 / 4 preliminary squares and
    3 r^2 / 4 - 2 overlapping subpatches (three squares merge into the
    L-shaped corner subpatch); the figure's example r = 4 gives 12 and 10."""
    for r, n1, nv in ((4, 9, 3), (2, 43, 9), (6, 43, 9)):
        N = r * (n1 + 1) - 1
        h = 1.0 / (N + 2 * nv - 1)
        a0 = (nv - 1) * h
        edges = a0 + np.arange(r + 1) * (n1 + 1) * h
        assert abs(edges[-1] - (1 - (nv - 1) * h)) < 1e-12  # arm fits [0, 1]
        squares = [(i, j) for i in range(r) for j in range(r) if not (i < r // 2 and j < r // 2)]
        assert len(squares) == 3 * r * r // 4
        assert len(squares) - 3 + 1 == 3 * r * r // 4 - 2
        # overlapping square side: n1 + 2 n_v points; L subpatch: two line
        # lengths n1 + 2 n_v and 2 n1 + 2 n_v + 1
        side = round(((n1 + 1) * h + 2 * (nv - 1) * h) / h) + 1
        assert side == n1 + 2 * nv
        long = round((2 * (n1 + 1) * h + 2 * (nv - 1) * h) / h) + 1
        assert long == 2 * n1 + 2 * nv + 1
    assert (43 + 2 * 9, 2 * 43 + 2 * 9 + 1) == (61, 105)


def test_l_patch_runs_and_boundary():
    h = 0.01
    spec = W.lattice_patch(h, 0, 40, 0, 40, {k: W.INTERNAL for k in "WESN"}, "C1", notch_box=(21, 40, 0, 19))
    p = solver.patches_from_specs([spec])[0]
    g = patches.Grid(p, 2, 27, 5)
    lens = sorted(set(n for _, n in g.row_runs))
    assert lens == [21, 41]
    assert sorted(set(n for _, n in g.col_runs)) == [21, 41]
    # notch sides are slip boundary points; the corner node ends no line
    bset = {(j, i) for (j, i, k, _) in g.boundary}
    assert (10, 20) in bset and (20, 30) in bset and (20, 20) not in bset
    assert g.affine
    assert np.allclose(g.t1x[p.mask], 1 / h) and np.allclose(g.t2y[p.mask], 1 / h)


def test_metrics_annulus():
    spec = W.annular_sector(64, 48)[0]
    g = patches.Grid(solver.patches_from_specs([spec])[0], 5, 27, 5)
    r = np.hypot(spec.x, spec.y)
    th = np.arctan2(spec.y, spec.x)
    # t1 = theta / dtheta ; t2 = (r - r0) / dr  with dtheta = (pi/3)/63, dr = 1/47
    dth, dr = (np.pi / 3) / 63, 1.0 / 47
    t1x = -np.sin(th) / r / dth
    t2x = np.cos(th) / dr
    assert np.abs(g.t1x - t1x).max() < 1e-7 * np.abs(t1x).max()
    assert np.abs(g.t2x - t2x).max() < 1e-7 * np.abs(t2x).max()
    # Laplacian of t2 = (r - r0)/dr is 1 / (r dr)
    assert np.abs(g.lap2 - 1 / (r * dr)).max() < 1e-5 * np.abs(1 / (r * dr)).max()


def test_lagrange_reproduces_quintics():
    rng = np.random.default_rng(3)
    u = rng.uniform(0, 5, 200)
    w = overlap.lagrange_weights(u)
    for k in range(6):
        assert np.abs(w @ (np.arange(6.0) ** k) - u ** k).max() < 1e-11 * max(1, 5 ** k)
    dw = overlap.lagrange_dweights(u)
    for k in range(1, 6):
        assert np.abs(dw @ (np.arange(6.0) ** k) - k * u ** (k - 1)).max() < 1e-9 * 5 ** k


def test_shifted_stencil_beside_the_notch_reproduces_polynomials():
    """Interpolation inside a skewed corner subpatch (the wedge tip's C1
    patch, affine, obstacle quadrant masked): where the centred 6 x 6
    stencil would take masked nodes next to the notch, the stencil moves
    (one-sided interpolation) and still reproduces a polynomial of degree 5
    exactly; away from the notch the centred stencil is kept."""
    geo = W.wedge_geometry(400)
    m = 20
    spec = W._c1_patch(1.0 / 400, geo["T"], -geo["l"], -geo["u"], m, W.WEDGE_INFLOW)
    g = patches.Grid(solver.patches_from_specs([spec])[0], 2, 27, 5)
    mask = g.p.mask
    f = lambda x, y: 1e6 * x ** 3 * y ** 2 - 3e4 * y ** 4 + 7e2 * x * y + x - 2 * y
    shifted = 0
    for xi, eta in ((m + 0.4, m - 3.7), (m + 1.3, m - 7.2), (m + 2.6, m - 1.5), (m - 4.3, m + 0.7),
                    (m + 0.5, m + 0.5), (m + 10.25, m + 8.75)):
        ent = overlap.stencil(g, xi, eta, lambda j, i: mask[j, i])
        assert ent is not None and all(mask[j, i] for j, i, _ in ent)
        c = overlap.stencil(g, xi, eta)
        shifted += [(j, i) for j, i, _ in ent] != [(j, i) for j, i, _ in c]
        # the map is affine: the point's coordinates are the same affine
        # combination of node coordinates under either stencil
        px = sum(w * g.p.x[j, i] for j, i, w in ent)
        py = sum(w * g.p.y[j, i] for j, i, w in ent)
        assert abs(px - sum(w * g.p.x[j, i] for j, i, w in c)) < 1e-14
        assert abs(py - sum(w * g.p.y[j, i] for j, i, w in c)) < 1e-14
        v = sum(w * f(g.p.x[j, i], g.p.y[j, i]) for j, i, w in ent)
        assert abs(v - f(px, py)) < 1e-9 * max(1.0, abs(f(px, py)))
    assert shifted >= 4
    # far from the notch and inside the box: the centred stencil
    ent = overlap.stencil(g, m + 10.25, m + 8.75, lambda j, i: mask[j, i])
    assert ent == overlap.stencil(g, m + 10.25, m + 8.75)
    assert min(i for _, i, _ in ent) == m + 8 and min(j for j, _, _ in ent) == m + 6
    # no position exists when the point is inside the notch
    assert overlap.stencil(g, m - 3.5, m - 3.5, lambda j, i: mask[j, i]) is None


def test_newton_inversion_curved():
    spec = W.annular_sector(40, 30)[0]
    g = patches.Grid(solver.patches_from_specs([spec])[0], 5, 27, 5)
    rng = np.random.default_rng(4)
    th = rng.uniform(0.1, np.pi / 3 - 0.1, 50)
    r = rng.uniform(1.1, 1.9, 50)
    xi, eta, ok = overlap.invert_map(g, r * np.cos(th), r * np.sin(th))
    assert ok.all()
    assert np.abs(xi - th / (np.pi / 3) * 39).max() < 1e-5  # map is interpolated (degree 5)
    assert np.abs(eta - (r - 1) * 29).max() < 1e-8


def test_step_channel_exchange_is_copy_and_donors_not_recipients():
    specs = W.step_channel()
    grids = [patches.Grid(p, 2, 27, 5) for p in solver.patches_from_specs(specs)]
    rows = overlap.fringe_rows(grids)
    n = 0
    for p, r in enumerate(rows):
        for (j, i, s, ent) in r:
            assert s != p and len(ent) == 1 and ent[0][2] == 1.0
            jd, id_, _ = ent[0]
            assert not grids[s].fringe[jd, id_]
            assert np.isclose(grids[s].p.x[jd, id_], grids[p].p.x[j, i])
            assert np.isclose(grids[s].p.y[jd, id_], grids[p].p.y[j, i])
            n += 1
    assert n == sum(int(g.fringe.sum()) for g in grids)
    assert {s.kind for s in specs} >= {"C1", "C2", "S", "I"}


def test_interpolation_reproduces_polynomials_multipatch():
    specs = W.vortex_multipatch(41)
    grids = [patches.Grid(p, 5, 27, 5) for p in solver.patches_from_specs(specs)]
    rows = overlap.fringe_rows(grids)
    # a field that is a polynomial of degree <= 5 in each index coordinate of
    # every donor (these grids are affine): x^2 y^3 + y^5 - x
    f = lambda x, y: 1e-3 * (x ** 2 * y ** 3) + 1e-4 * y ** 5 - x
    ninterp = 0
    for p, r in enumerate(rows):
        for (j, i, s, ent) in r:
            gs = grids[s].p
            v = sum(w * f(gs.x[jd, id_], gs.y[jd, id_]) for jd, id_, w in ent)
            assert abs(v - f(grids[p].p.x[j, i], grids[p].p.y[j, i])) < 1e-10
            ninterp += len(ent) > 1
    assert ninterp > 100


def test_smoothing_fast_equals_direct():
    rng = np.random.default_rng(5)
    m = np.where(rng.random((30, 40)) < 0.05, rng.random((30, 40)), 0.0)
    assert np.array_equal(viscosity.smooth(m, 9), viscosity.smooth_fast(m, 9))


def test_blend_rows_partition_of_unity():
    specs = W.step_channel()
    grids = [patches.Grid(p, 2, 27, 5) for p in solver.patches_from_specs(specs)]
    rows = overlap.blend_rows(grids[:9], 9)
    count = 0
    for r in rows:
        for key, ent in r.items():
            assert abs(sum(w for _, w in ent) - 1.0) < 1e-13
            assert all(w >= 0 for _, w in ent)
            count += 1
    assert count > 1000


def test_gradient_check_fd():
    rng = np.random.default_rng(6)
    prm = sdnn.init_params(rng)
    x = rng.random((32, 16))
    lab = rng.integers(0, 3, 32)
    loss, g = sdnn.loss_and_grads(prm, x, lab)
    for k in ("W1", "b1", "W2", "W3", "b3"):
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in prm[k].shape)
            eps = 1e-6
            p1 = {kk: v.copy() for kk, v in prm.items()}
            p1[k][idx] += eps
            p2 = {kk: v.copy() for kk, v in prm.items()}
            p2[k][idx] -= eps
            fd = (sdnn.loss_and_grads(p1, x, lab)[0] - sdnn.loss_and_grads(p2, x, lab)[0]) / (2 * eps)
            assert abs(fd - g[k][idx]) < 1e-7 * max(1, abs(fd)), (k, idx, fd, g[k][idx])


def test_modal_indicator_flags_jumps_not_smooth():
    x = np.linspace(0, 1, 16)
    smooth = np.exp(np.sin(3 * x))[None, :]
    jump = (x > 0.5).astype(float)[None, :] + 0.1 * x[None, :]
    assert sdnn.modal_classify(smooth)[0] == 0
    assert sdnn.modal_classify(jump)[0] == 2
    assert sdnn.modal_classify(np.full((1, 16), 3.0))[0] == 0


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 1e-3])
    r = sdnn.round_bf16(v)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -6 and r[3] == -2.5
    assert abs(r[4] - 1e-3) < 1e-3 * 2 ** -8
