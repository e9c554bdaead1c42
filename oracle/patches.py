"""Subpatch grids: line runs, metrics, fringe and boundary points.

Follows Sec. 3 (patches S, I, C1, C2 with parameter spaces Q and L, the
subpatch grids of equation "c1_grid" and the index sets "D_C1"), the fringe
definition of Sec. 3.3 (points within n_f points of an internal side along
one of the two parameter directions) and item 1 of Sec. 5 (the Jacobian of
the inverse mapping, used to write the equations in parameter space).

A subpatch is given by its node coordinates x, y of shape (n2, n1) (q^1 is
the fast index i, q^2 the slow index j), an activity mask (the L-shaped C1
corner subpatch masks one quadrant, the obstacle), the kind of each of the
four sides of its index box and the kind of the mask boundary (the "notch",
the arcs AC and BC of a C1 patch, always external).

Every row and column of active points must be one contiguous run; all
derivatives are taken run by run with the FC operator of the run's length.
Derivatives are in index units (with respect to i and j); the metric terms
carry the grid spacing.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import fcgram

INTERNAL, INFLOW, OUTFLOW, SLIP, EXACT, NOSLIP = 0, 1, 2, 3, 4, 5
SIDES = ("W", "E", "S", "N")


@dataclass
class Patch:
    x: np.ndarray
    y: np.ndarray
    mask: np.ndarray | None = None
    sides: dict = field(default_factory=lambda: {s: INTERNAL for s in SIDES})
    notch: int = SLIP
    inflow: np.ndarray | None = None  # primitive state for INFLOW sides
    kind: str = "I"

    def __post_init__(self):
        self.x = np.ascontiguousarray(self.x, dtype=np.float64)
        self.y = np.ascontiguousarray(self.y, dtype=np.float64)
        if self.mask is None:
            self.mask = np.ones(self.x.shape, dtype=bool)
        self.mask = np.asarray(self.mask, dtype=bool)

    @property
    def n1(self):
        return self.x.shape[1]

    @property
    def n2(self):
        return self.x.shape[0]


def runs_of(mask_lines: np.ndarray):
    """(start, length) of the single run of True values in each line."""
    out = []
    for line in mask_lines:
        idx = np.flatnonzero(line)
        if idx.size == 0:
            out.append((0, 0))
            continue
        if idx[-1] - idx[0] + 1 != idx.size:
            raise ValueError("a grid line holds more than one run of active points")
        out.append((int(idx[0]), int(idx.size)))
    return out


class Grid:
    """Per-subpatch discretization data derived from a :class:`Patch`."""

    def __init__(self, patch: Patch, d: int, C: int, n_f: int):
        self.p = patch
        self.d, self.C, self.n_f = d, C, n_f
        m = patch.mask
        self.row_runs = runs_of(m)          # per j: along q^1
        self.col_runs = runs_of(m.T)        # per i: along q^2
        self._end_kinds()
        self._metrics()
        self._fringe_and_boundary()

    # --- FC along lines -------------------------------------------------
    def deriv(self, f: np.ndarray, direction: int, kind: str = "d1") -> np.ndarray:
        """Apply the FC map ``kind`` along q^1 (direction 0) or q^2 (1) of a
        field of shape (..., n2, n1); masked points are returned as 0."""
        out = np.zeros_like(f, dtype=np.float64)
        if direction == 0:
            groups = {}
            for j, (s, n) in enumerate(self.row_runs):
                if n:
                    groups.setdefault((s, n), []).append(j)
            for (s, n), js in groups.items():
                out[..., js, s:s + n] = fcgram.fc_apply(f[..., js, s:s + n], self.d, self.C, kind)
        else:
            ft = np.swapaxes(f, -1, -2)
            ot = np.swapaxes(out, -1, -2)
            groups = {}
            for i, (s, n) in enumerate(self.col_runs):
                if n:
                    groups.setdefault((s, n), []).append(i)
            for (s, n), is_ in groups.items():
                ot[..., is_, s:s + n] = fcgram.fc_apply(ft[..., is_, s:s + n], self.d, self.C, kind)
        return out

    # --- sides ----------------------------------------------------------
    def _end_kinds(self):
        p = self.p
        self.row_end = []
        for (s, n) in self.row_runs:
            if n == 0:
                self.row_end.append((None, None))
                continue
            lo = p.sides["W"] if s == 0 else p.notch
            hi = p.sides["E"] if s + n == p.n1 else p.notch
            self.row_end.append((lo, hi))
        self.col_end = []
        for (s, n) in self.col_runs:
            if n == 0:
                self.col_end.append((None, None))
                continue
            lo = p.sides["S"] if s == 0 else p.notch
            hi = p.sides["N"] if s + n == p.n2 else p.notch
            self.col_end.append((lo, hi))

    # --- metrics (Sec. 5 item 1) ---------------------------------------
    def _metrics(self):
        p = self.p
        m = p.mask
        x1 = self.deriv(p.x, 0)
        x2 = self.deriv(p.x, 1)
        y1 = self.deriv(p.y, 0)
        y2 = self.deriv(p.y, 1)
        det = x1 * y2 - x2 * y1
        det = np.where(m, det, 1.0)
        t1x, t1y = y2 / det, -x2 / det
        t2x, t2y = -y1 / det, x1 / det
        met = np.stack([t1x, t1y, t2x, t2y])
        scale = np.abs(met[:, m]).max()
        mean = met[:, m].mean(axis=1)
        # Reading: an affine subpatch (constant metrics up to the FC fit
        # error) uses the exact constant metrics.
        self.affine = bool(np.abs(met[:, m] - mean[:, None]).max() <= 1e-6 * scale)
        if self.affine:
            # components below 1e-6 of the largest are zero (axis-aligned
            # grids are then exactly Cartesian)
            mean = np.where(np.abs(mean) <= 1e-6 * scale, 0.0, mean)
            met = np.where(m, mean[:, None, None], 0.0) * np.ones_like(met)
        else:
            met = np.where(m, met, 0.0)
        self.t1x, self.t1y, self.t2x, self.t2y = met
        # contravariant metric tensor g^{kl} = grad t^k . grad t^l
        self.g11 = self.t1x ** 2 + self.t1y ** 2
        self.g12 = self.t1x * self.t2x + self.t1y * self.t2y
        self.g22 = self.t2x ** 2 + self.t2y ** 2
        # Laplacian of the index coordinates, Delta t^k (zero when affine)
        if self.affine:
            self.lap1 = np.zeros_like(self.g11)
            self.lap2 = np.zeros_like(self.g11)
        else:
            def dx(f):
                return self.t1x * self.deriv(f, 0) + self.t2x * self.deriv(f, 1)

            def dy(f):
                return self.t1y * self.deriv(f, 0) + self.t2y * self.deriv(f, 1)
            self.lap1 = np.where(m, dx(self.t1x) + dy(self.t1y), 0.0)
            self.lap2 = np.where(m, dx(self.t2x) + dy(self.t2y), 0.0)
        # local mesh size at each point: 1 / sqrt of the largest eigenvalue
        # of the metric tensor g^{kl} (index units), i.e. the distance
        # between neighbouring grid lines along the most compressed
        # direction; on an orthogonal grid the smaller spacing, on a skewed
        # one (cells of angle a) smaller by up to sin(a/2) ... sin(a)
        half = 0.5 * (self.g11 + self.g22)
        lam = half + np.sqrt(0.25 * (self.g11 - self.g22) ** 2 + self.g12 ** 2)
        hx = 1.0 / np.sqrt(np.where(m, lam, 1.0))
        self.hx = np.where(m, hx, 0.0)

    # --- fringe, boundary, depth (Sec. 3.3) ----------------------------
    def _fringe_and_boundary(self):
        """Fringe (interpolation recipients), exact-data fringe (points within
        n_f of an EXACT side) and the physical boundary points (run ends on
        SLIP, INFLOW or OUTFLOW sides)."""
        p, n_f = self.p, self.n_f
        n2, n1 = p.x.shape
        fringe = np.zeros((n2, n1), dtype=bool)
        xfringe = np.zeros((n2, n1), dtype=bool)
        depth = np.full((n2, n1), np.inf)
        bnd = []  # (j, i, kind, direction of the line that ends there)

        def end(kind, dist, sl, j_or_i, direction):
            if kind == INTERNAL:
                fringe[sl] |= dist < n_f
                depth[sl] = np.minimum(depth[sl], dist)
            elif kind == EXACT:
                xfringe[sl] |= dist < n_f
            else:
                bnd.append(j_or_i + (kind, direction))

        for j, ((s, n), (lo, hi)) in enumerate(zip(self.row_runs, self.row_end)):
            if n == 0:
                continue
            i = np.arange(s, s + n)
            sl = (j, slice(s, s + n))
            end(lo, i - s, sl, (j, s), 0)
            end(hi, s + n - 1 - i, sl, (j, s + n - 1), 0)
        for i, ((s, n), (lo, hi)) in enumerate(zip(self.col_runs, self.col_end)):
            if n == 0:
                continue
            j = np.arange(s, s + n)
            sl = (slice(s, s + n), i)
            end(lo, j - s, sl, (s, i), 1)
            end(hi, s + n - 1 - j, sl, (s + n - 1, i), 1)
        self.fringe = fringe & p.mask
        self.xfringe = xfringe & p.mask & ~self.fringe
        self.depth = np.where(p.mask, depth, 0.0)
        self.boundary = bnd

    def depth_at(self, xi: float, eta: float) -> float:
        """Index distance from a (fractional) parameter position to the
        nearest internal side, along the row and the column of the nearest
        node; infinite when no internal side bounds those lines."""
        j = int(np.clip(np.rint(eta), 0, self.p.n2 - 1))
        i = int(np.clip(np.rint(xi), 0, self.p.n1 - 1))
        best = np.inf
        s, n = self.row_runs[j]
        lo, hi = self.row_end[j]
        if n:
            if lo == INTERNAL:
                best = min(best, xi - s)
            if hi == INTERNAL:
                best = min(best, s + n - 1 - xi)
        s, n = self.col_runs[i]
        lo, hi = self.col_end[i]
        if n:
            if lo == INTERNAL:
                best = min(best, eta - s)
            if hi == INTERNAL:
                best = min(best, s + n - 1 - eta)
        return best
