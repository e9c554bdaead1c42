"""The Mach-10 wedge tunnel (host only): its decomposition into C1 corner
subpatches (non-right angles), skewed-affine S subpatches on the faces,
rear-face S subpatches and seeded lattice subpatches; every node outside
the obstacle, every wall node on it, the corner subpatches' masked quadrant
inside it; and the library accepts the small and the full-size set (every
fringe point has an eligible donor, checked by fcs_create)."""
import ctypes
import os

import numpy as np
import pytest

import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden", "sdnn_oracle_weights.npz")


def _create(specs):
    import paper_2506_19370_amd as F
    from paper_2506_19370_amd import _lib as L
    blob = np.load(GOLD)["params"]
    h = F.api.create_context(specs, F.SolverParams(fc_d=2, fc_C=27, cfl=0.5, av="sdnn", sdnn_weights=blob,
                                                   filter=True))
    try:
        n = ctypes.c_size_t()
        assert L.fcs_workspace_size(h, ctypes.byref(n)) == 0 and n.value > 0
        return n.value
    finally:
        L.fcs_destroy(h)


def _inside_obstacle(geo, x, y, tol):
    """Signed test: > tol inside the triangle T, R+, R- (index units)."""
    T, Rp, Rm = geo["T"], geo["Rp"], geo["Rm"]
    def side(a, b):  # distance to the left of a -> b
        d = b - a
        return ((x - a[0]) * d[1] - (y - a[1]) * d[0]) / np.hypot(*d)
    # the triangle is T -> R- -> R+ counter-clockwise: inside = all negative
    s = np.maximum.reduce([side(T, Rm), side(Rm, Rp), side(Rp, T)])
    return -s > tol


@pytest.mark.parametrize("N,smin,smax", [(600, 48, 96), (4400, 150, 300)])
def test_wedge_nodes_walls_and_notches(N, smin, smax):
    specs = W.wedge_tunnel(N, smin, smax)
    geo = W.wedge_geometry(N)
    tol = 1e-9 * N
    nwall = 0
    for s in specs:
        X, Y = s.x * N, s.y * N
        act = np.ones(s.shape, bool) if s.mask is None else s.mask
        assert not _inside_obstacle(geo, X[act], Y[act], tol).any()
        assert (X[act] >= -tol).all() and (X[act] <= N + tol).all()
        assert (Y[act] >= -tol).all() and (Y[act] <= N / 2 + tol).all()
        if s.kind == "C1":
            # the masked quadrant is the obstacle; its boundary rows are the walls
            assert _inside_obstacle(geo, X[~act], Y[~act], -tol).all()
            # walls: the active nodes next to a masked one
            pad = np.pad(~act, 1)
            nb = pad[:-2, 1:-1] | pad[2:, 1:-1] | pad[1:-1, :-2] | pad[1:-1, 2:]
            w = act & nb
            wall = np.column_stack([X[w], Y[w]])
        elif s.sides["S"] == W.SLIP and s.kind == "S" and not np.allclose(Y[0], Y[0, 0]):
            wall = np.column_stack([X[0], Y[0]])          # upper face
        elif s.sides["N"] == W.SLIP and s.kind == "S" and not np.allclose(Y[-1], Y[-1, 0]):
            wall = np.column_stack([X[-1], Y[-1]])        # lower face (mirror)
        elif s.sides["W"] == W.SLIP and s.kind == "S" and abs(X[0, 0] - geo["Xr"]) < tol:
            wall = np.column_stack([X[:, 0], Y[:, 0]])    # rear face
        else:
            continue
        nwall += 1
        # wall nodes lie on the obstacle's boundary (not inside, not off it)
        on = ~_inside_obstacle(geo, wall[:, 0], wall[:, 1], 1e-9 * N) & \
            _inside_obstacle(geo, wall[:, 0], wall[:, 1], -1e-9 * N)
        assert on.all()
    kinds = [s.kind for s in specs]
    assert kinds.count("C1") == 3 and nwall >= 3 + 4
    # the faces' S subpatches are skewed: one axis along the face, one vertical
    face = [s for s in specs if s.kind == "S" and not np.allclose(s.y[0], s.y[0, 0])
            and not np.allclose(s.x[:, 0], s.x[0, 0])]
    for s in face:
        e1 = np.array([s.x[0, 1] - s.x[0, 0], s.y[0, 1] - s.y[0, 0]])
        e2 = np.array([s.x[1, 0] - s.x[0, 0], s.y[1, 0] - s.y[0, 0]])
        cosang = abs(e1 @ e2) / np.hypot(*e1) / np.hypot(*e2)
        assert abs(cosang - np.sin(geo["theta"])) < 1e-9


def test_wedge_shape_full_size():
    specs = W.wedge_tunnel()
    sides = np.array([s.shape for s in specs])
    npts = sum(s.npoints() for s in specs)
    assert 230 <= len(specs) <= 260 and 1.1e7 < npts < 1.25e7
    # seeded sides in [150, 300]; pieces rescaled to fill a span and the
    # wall-side subpatches without an overlap reach a little beyond
    assert sides.min() >= 130 and sides.max() <= 335
    assert np.median(sides) > 170
    again = W.wedge_tunnel()
    assert all(np.array_equal(a.x, b.x) and np.array_equal(a.y, b.y) for a, b in zip(specs, again))


def test_wedge_accepted_small():
    specs = W.wedge_tunnel(600, 48, 96)
    assert _create(specs) > 0


def test_wedge_accepted_full_size():
    # about 8 GB of device workspace for 1.16e7 points (FP64)
    assert 6e9 < _create(W.wedge_tunnel()) < 1.1e10
