"""Inter-patch communication: donor search, interpolation weights, blends.

Follows Sec. 3.3: every point of the n_f-point fringe of a subpatch receives,
at every stage, the solution value at the same physical location taken from
another subpatch, by exchange (when the grids coincide) or by polynomial
interpolation; donors are never themselves fringe points (the minimum
overlap condition of Sec. 3.2.3).  The interpolation degree, the donor
choice and the inversion of the donor mapping are not given in the paper;
the reading here is

* the donor mapping is the degree-5 tensor-product Lagrange interpolant of
  its node coordinates, inverted by Newton's method from the nearest node;
* values are interpolated with the same 6 x 6 tensor Lagrange stencil,
  centred on the donor cell and clamped into the index box; a coordinate
  within 1e-9 of a grid line is snapped to it (exchange then reduces to a
  copy); where the centred stencil would take a node the donor cannot give
  (masked, or a fringe node), the stencil moves by up to two nodes per
  direction, keeping the point inside its span, to the nearest position
  whose nodes are all eligible (near the obstacle quadrant of a corner
  subpatch the interpolation is then one-sided);
* the donor is the eligible subpatch in which the point lies deepest (index
  distance to its internal sides), ties to the lowest subpatch index.

The same machinery gives the rows of the multi-patch viscosity blend
(Sec. 4; reading of the windowing functions of Part I).
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree

SNAP = 1e-9
ORDER = 6  # points per direction of the interpolation stencil


def lagrange_weights(u: np.ndarray) -> np.ndarray:
    """Weights of the 6-point Lagrange interpolant at offsets 0..5 for
    positions u (shape (m,)); returns (m, 6)."""
    u = np.asarray(u, dtype=np.float64)
    w = np.ones(u.shape + (ORDER,))
    for k in range(ORDER):
        for m in range(ORDER):
            if m != k:
                w[..., k] *= (u - m) / (k - m)
    return w


def lagrange_dweights(u: np.ndarray) -> np.ndarray:
    """Derivatives of :func:`lagrange_weights` with respect to u."""
    u = np.asarray(u, dtype=np.float64)
    dw = np.zeros(u.shape + (ORDER,))
    for k in range(ORDER):
        for m in range(ORDER):
            if m == k:
                continue
            term = np.full(u.shape, 1.0 / (k - m))
            for l in range(ORDER):
                if l != k and l != m:
                    term = term * (u - l) / (k - l)
            dw[..., k] += term
    return dw


def stencil_start(xi: np.ndarray, n: int) -> np.ndarray:
    return np.clip(np.floor(xi).astype(np.int64) - 2, 0, n - ORDER)


def invert_map(grid, px: np.ndarray, py: np.ndarray):
    """Newton inversion of the donor mapping of ``grid`` at physical points
    (px, py).  Returns (xi, eta, ok)."""
    p = grid.p
    n2, n1 = p.x.shape
    tree = cKDTree(np.column_stack([p.x.ravel(), p.y.ravel()]))
    _, idx = tree.query(np.column_stack([px, py]))
    xi = (idx % n1).astype(np.float64)
    eta = (idx // n1).astype(np.float64)
    scale = max(np.ptp(p.x), np.ptp(p.y), 1e-300)
    ok = np.zeros(px.shape, dtype=bool)
    for _ in range(40):
        i0 = stencil_start(xi, n1)
        j0 = stencil_start(eta, n2)
        u, v = xi - i0, eta - j0
        wu, wv = lagrange_weights(u), lagrange_weights(v)
        du, dv = lagrange_dweights(u), lagrange_dweights(v)
        jj = j0[:, None] + np.arange(ORDER)[None, :]
        ii = i0[:, None] + np.arange(ORDER)[None, :]
        X = p.x[jj[:, :, None], ii[:, None, :]]  # (m, 6[j], 6[i])
        Y = p.y[jj[:, :, None], ii[:, None, :]]
        fx = np.einsum("mb,ma,mba->m", wv, wu, X) - px
        fy = np.einsum("mb,ma,mba->m", wv, wu, Y) - py
        xa = np.einsum("mb,ma,mba->m", wv, du, X)
        xb = np.einsum("mb,ma,mba->m", dv, wu, X)
        ya = np.einsum("mb,ma,mba->m", wv, du, Y)
        yb = np.einsum("mb,ma,mba->m", dv, wu, Y)
        det = xa * yb - xb * ya
        dxi = (yb * fx - xb * fy) / det
        deta = (-ya * fx + xa * fy) / det
        xi = xi - dxi
        eta = eta - deta
        # keep the iterate inside a slightly enlarged box
        xi = np.clip(xi, -3.0, n1 + 2.0)
        eta = np.clip(eta, -3.0, n2 + 2.0)
        # converged once the step is below the rounding floor of fine grids
        # with O(1) coordinates (a few 1e-12 index units), well under SNAP
        ok = (np.abs(dxi) < 1e-10) & (np.abs(deta) < 1e-10) | (np.hypot(fx, fy) < 1e-15 * scale)
        if ok.all():
            break
    # snap to grid lines
    rx, ry = np.rint(xi), np.rint(eta)
    xi = np.where(np.abs(xi - rx) < SNAP, rx, xi)
    eta = np.where(np.abs(eta - ry) < SNAP, ry, eta)
    return xi, eta, ok


def inside(grid, xi: float, eta: float) -> bool:
    """Whether a parameter position lies in the active part of the grid."""
    n2, n1 = grid.p.x.shape
    if not (-SNAP <= xi <= n1 - 1 + SNAP and -SNAP <= eta <= n2 - 1 + SNAP):
        return False
    j = int(np.clip(np.rint(eta), 0, n2 - 1))
    i = int(np.clip(np.rint(xi), 0, n1 - 1))
    s, n = grid.row_runs[j]
    if n == 0 or not (s - SNAP <= xi <= s + n - 1 + SNAP):
        return False
    s, n = grid.col_runs[i]
    if n == 0 or not (s - SNAP <= eta <= s + n - 1 + SNAP):
        return False
    return True


def _starts(xi: float, n: int):
    """Candidate first nodes of the 6-point stencil along one direction, in
    order of preference: the centred (clamped) start, then shifted by +1,
    -1, +2, -2, keeping 0 <= start <= n - 6 and the point inside the span.
    A coordinate on a grid line has the single node itself."""
    if xi == np.rint(xi):
        return [None]
    c = int(stencil_start(np.array([xi]), n)[0])
    out = []
    for s in (c, c + 1, c - 1, c + 2, c - 2):
        if 0 <= s <= n - ORDER and s <= xi <= s + ORDER - 1:
            out.append(s)
    return out


def stencil(grid, xi: float, eta: float, eligible=None):
    """Interpolation entries [(j, i, weight)] at (xi, eta); coordinates that
    sit on a grid line contribute a single node along that direction.  With
    ``eligible(j, i)``, the first stencil position (in the order of _starts,
    by the sum of the two ranks, then the rank along q^1) whose nodes are
    all eligible; None when there is none."""
    n2, n1 = grid.p.x.shape
    si, sj = _starts(xi, n1), _starts(eta, n2)
    for total in range(len(si) + len(sj) - 1):
        for ri in range(total + 1):
            rj = total - ri
            if ri >= len(si) or rj >= len(sj):
                continue
            i0, j0 = si[ri], sj[rj]
            ii = [int(xi)] if i0 is None else list(range(i0, i0 + ORDER))
            jj = [int(eta)] if j0 is None else list(range(j0, j0 + ORDER))
            if eligible is not None and not all(eligible(j, i) for j in jj for i in ii):
                continue
            wi = [1.0] if i0 is None else _lagrange_scalar(xi - i0)
            wj = [1.0] if j0 is None else _lagrange_scalar(eta - j0)
            return [(j, i, wj[b] * wi[a]) for b, j in enumerate(jj) for a, i in enumerate(ii)]
    return None


def _lagrange_scalar(u: float):
    """lagrange_weights for one position, as plain floats."""
    w = []
    for k in range(ORDER):
        v = 1.0
        for m in range(ORDER):
            if m != k:
                v *= (u - m) / (k - m)
        w.append(v)
    return w


def _bbox_candidates(g_p, g_s, pts):
    ms = g_s.p.mask
    xs, ys = g_s.p.x[ms], g_s.p.y[ms]
    tol = 1e-9 * max(np.ptp(xs), np.ptp(ys), 1.0)
    px, py = g_p.p.x[pts], g_p.p.y[pts]
    return (px >= xs.min() - tol) & (px <= xs.max() + tol) & (py >= ys.min() - tol) & (py <= ys.max() + tol)


def fringe_rows(grids):
    """Interpolation rows for every fringe point of every subpatch.

    Returns a list over subpatches of lists of (j, i, donor, entries), with
    entries [(jd, id, w)] of the donor subpatch.  Raises ValueError when a
    fringe point has no eligible donor (minimum overlap violated)."""
    out = []
    for p, gp in enumerate(grids):
        pts = np.nonzero(gp.fringe)
        best = [(-np.inf, None, None)] * len(pts[0])
        for s, gs in enumerate(grids):
            if s == p:
                continue
            cand = np.flatnonzero(_bbox_candidates(gp, gs, pts))
            if cand.size == 0:
                continue
            xi, eta, ok = invert_map(gs, gp.p.x[pts][cand], gp.p.y[pts][cand])
            for k, c in enumerate(cand):
                if not ok[k] or not inside(gs, xi[k], eta[k]):
                    continue
                ent = stencil(gs, xi[k], eta[k], lambda j, i: gs.p.mask[j, i] and not gs.fringe[j, i])
                if ent is None:
                    continue
                dep = gs.depth_at(xi[k], eta[k])
                if dep > best[c][0] + 1e-9:
                    best[c] = (dep, s, ent)
        rows = []
        for c, (dep, s, ent) in enumerate(best):
            if s is None:
                raise ValueError(f"fringe point {(int(pts[0][c]), int(pts[1][c]))} of subpatch {p} has no donor")
            rows.append((int(pts[0][c]), int(pts[1][c]), s, ent))
        out.append(rows)
    return out


def smooth_step(t: np.ndarray) -> np.ndarray:
    """C-infinity step: 0 for t <= 0, 1 for t >= 1."""
    t = np.asarray(t, dtype=np.float64)
    out = np.where(t >= 1.0, 1.0, 0.0)
    mid = (t > 0.0) & (t < 1.0)
    tm = t[mid]
    a = np.exp(-1.0 / tm)
    b = np.exp(-1.0 / (1.0 - tm))
    out[mid] = a / (a + b)
    return out


def blend_weight(depth, n_v: int):
    """Window value of a subpatch at a point at the given depth (index
    distance to its internal sides): rises from 0 at the side to 1 at depth
    2 n_v (reading of the windowing functions I-(42))."""
    return smooth_step(np.asarray(depth, dtype=np.float64) / (2.0 * n_v))


def blend_rows(grids, n_v: int):
    """Rows of the viscosity blend mu = sum_s W_s mu_s / sum_s W_s over the
    subpatches s covering each point (reading of I-(44)): for every point of
    subpatch p covered by another subpatch with positive window value,
    a list of ((subpatch, j, i), weight) entries that sum to one.
    Returns a list over subpatches of dicts {(j, i): entries}.
    parity unpinned: the windowing functions of Part I are not available."""
    out = []
    for p, gp in enumerate(grids):
        pts = np.nonzero(gp.p.mask)
        contrib = [[] for _ in range(len(pts[0]))]
        for s, gs in enumerate(grids):
            if s == p:
                continue
            cand = np.flatnonzero(_bbox_candidates(gp, gs, pts))
            if cand.size == 0:
                continue
            xi, eta, ok = invert_map(gs, gp.p.x[pts][cand], gp.p.y[pts][cand])
            for k, c in enumerate(cand):
                if not ok[k] or not inside(gs, xi[k], eta[k]):
                    continue
                w = float(blend_weight(gs.depth_at(xi[k], eta[k]), n_v))
                if w <= 0.0:
                    continue
                ent = stencil(gs, xi[k], eta[k], lambda j, i: gs.p.mask[j, i])
                if ent is None:
                    continue
                contrib[c].append((s, w, ent))
        rows = {}
        for c, lst in enumerate(contrib):
            if not lst:
                continue
            j, i = int(pts[0][c]), int(pts[1][c])
            wp = float(blend_weight(gp.depth[j, i], n_v))
            total = wp + sum(w for _, w, _ in lst)
            ent = [((p, j, i), wp / total)] if wp > 0 else []
            for s, w, e in lst:
                ent += [((s, jd, id_), w * wl / total) for jd, id_, wl in e]
            rows[(j, i)] = ent
        out.append(rows)
    return out
