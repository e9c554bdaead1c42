"""The multi-patch FC-SDNN time loop, step by step (Alg. 1, 3, 4, 5).

One step: preliminary viscosity on every subpatch (Alg. 3) and its blend
across subpatches, filtering of the solution for t > 0 (Alg. 4), the
adaptive time step, and the five SSPRK stages (Alg. 5), each followed by the
boundary conditions and the fringe communication (Alg. 1).

The spatial operator follows item 1 and the stage algorithm of Sec. 5: the
Euler equations written in index coordinates with the Jacobian of the
inverse mapping (chain rule: d/dx = t1_x d/dt1 + t2_x d/dt2), FC derivatives
along grid lines, and the artificial-viscosity term built from the gradient
of mu and first and second derivatives by the product rule.  Reading of the
viscous term (Part I not available): mu Laplacian(w) + grad(mu) . grad(w)
for each conserved variable w.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import euler, fcgram, overlap, patches, sdnn, ssprk, viscosity


@dataclass
class Params:
    gamma: float = euler.GAMMA
    cfl: float = 0.5
    fc_d: int = 5
    fc_C: int = 27
    n_f: int = 5
    n_v: int = 9
    av: str = "off"          # "off", "modal", "sdnn"
    c_mu: float = 1.0
    filter: bool = False
    smear: bool = False      # localized smearing of the initial data (Alg. 4, t = 0)
    dt_fixed: float | None = None  # bypass the adaptive step (tests)


class Solver:
    def __init__(self, patch_list, prm: Params, sdnn_params=None, exact=None):
        self.prm = prm
        self.grids = [patches.Grid(p, prm.fc_d, prm.fc_C, prm.n_f) for p in patch_list]
        self.sizes = [g.p.x.size for g in self.grids]
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)])
        self.mask = np.concatenate([g.p.mask.ravel() for g in self.grids])
        self.fringe_rows = overlap.fringe_rows(self.grids) if len(self.grids) > 1 else [[] for _ in self.grids]
        self.blend = overlap.blend_rows(self.grids, prm.n_v) if (prm.av != "off" and len(self.grids) > 1) else None
        self.sdnn_params = sdnn_params
        self.exact = exact  # exact(x, y, t) -> primitive, for EXACT sides
        self.t = 0.0
        self.nstep = 0
        self.U = np.zeros((4, self.offsets[-1]))
        self.mu = None
        self.tau_override = None
        self.last_tau = None
        self.last_dt = None

    # ----------------------------------------------------------- views
    def view(self, U, p):
        g = self.grids[p]
        return U[:, self.offsets[p]:self.offsets[p + 1]].reshape(4, g.p.n2, g.p.n1)

    def field(self, arr, p):
        g = self.grids[p]
        return arr[self.offsets[p]:self.offsets[p + 1]].reshape(g.p.n2, g.p.n1)

    def set_prim(self, prim_list):
        for p, w in enumerate(prim_list):
            self.view(self.U, p)[...] = np.where(self.grids[p].p.mask, euler.prim_to_cons(w, self.prm.gamma), 0.0)

    # ----------------------------------------------------------- operator
    def rhs_patch(self, e, p, mu=None):
        """L(e) on subpatch p (stage algorithm, Sec. 5)."""
        g, gam = self.grids[p], self.prm.gamma
        m = g.p.mask
        ee = np.where(m, e, np.array([1.0, 0.0, 0.0, 1.0])[:, None, None])
        fx, fy = euler.fluxes(ee, gam)
        fx = np.where(m, fx, 0.0)
        fy = np.where(m, fy, 0.0)
        L = -(g.t1x * g.deriv(fx, 0) + g.t1y * g.deriv(fy, 0)
              + g.t2x * g.deriv(fx, 1) + g.t2y * g.deriv(fy, 1))
        if mu is not None:
            mu_p, mu1, mu2 = mu
            w = np.where(m, e, 0.0)
            w1, w2 = g.deriv(w, 0), g.deriv(w, 1)
            w11, w22 = g.deriv(w, 0, "d2"), g.deriv(w, 1, "d2")
            w12 = g.deriv(w1, 1)
            lap = g.g11 * w11 + 2.0 * g.g12 * w12 + g.g22 * w22 + g.lap1 * w1 + g.lap2 * w2
            grad = g.g11 * mu1 * w1 + g.g12 * (mu1 * w2 + mu2 * w1) + g.g22 * mu2 * w2
            L = L + mu_p * lap + grad
        return np.where(m, L, 0.0)

    def rhs(self, U):
        out = np.zeros_like(U)
        for p in range(len(self.grids)):
            mu = None
            if self.mu is not None:
                mu = tuple(self.field(a, p) for a in self.mu)
            out[:, self.offsets[p]:self.offsets[p + 1]] = self.rhs_patch(self.view(U, p), p, mu).reshape(4, -1)
        return out

    # ----------------------------------------------------------- BCs + fringe
    def enforce(self, U, t_stage, fringe=True):
        """Boundary conditions, then (unless fringe is False) the fringe
        communication (Alg. 1)."""
        gam = self.prm.gamma
        U = U.copy()
        for p, g in enumerate(self.grids):
            e = self.view(U, p)
            # slip walls: remove the normal momentum, keep the pressure
            normals = {}
            for (j, i, kind, direction) in g.boundary:
                if kind == patches.SLIP:
                    if direction == 0:
                        n = np.array([g.t1x[j, i], g.t1y[j, i]])
                    else:
                        n = np.array([g.t2x[j, i], g.t2y[j, i]])
                    normals.setdefault((j, i), []).append(n / np.hypot(*n))
            for (j, i), ns in normals.items():
                rho, mx, my, E = e[:, j, i]
                pr = (gam - 1.0) * (E - 0.5 * (mx * mx + my * my) / rho)
                if len(ns) == 1:
                    n = ns[0]
                    mn = mx * n[0] + my * n[1]
                    mx, my = mx - mn * n[0], my - mn * n[1]
                else:
                    mx, my = 0.0, 0.0
                e[1, j, i], e[2, j, i] = mx, my
                e[3, j, i] = pr / (gam - 1.0) + 0.5 * (mx * mx + my * my) / rho
            # no-slip adiabatic walls (reading of the obstacle conditions of
            # Sec. 7 and of Alg. 5's boundary treatment): zero momentum, rho
            # kept, and theta = p / ((gamma - 1) rho) at the wall set so that
            # the FC first derivative along the grid line ending at the wall
            # vanishes there (FC-Neumann).  A node where two such lines end
            # uses the line along q^2; a line with such walls at both ends
            # takes both wall values from the two conditions together.
            walls = {}
            for (j, i, kind, direction) in g.boundary:
                if kind == patches.NOSLIP:
                    walls[(j, i)] = max(walls.get((j, i), 0), direction)
            lines = {}
            for (j, i), direction in walls.items():
                key = (direction, j if direction == 0 else i)
                lines.setdefault(key, []).append((j, i))
            ee = np.where(g.p.mask, e, np.array([1.0, 0.0, 0.0, 1.0])[:, None, None])
            theta = euler.temperature_like(ee, gam)
            fixed = {}
            for (direction, l), nodes in lines.items():
                if direction == 0:
                    s0, n = g.row_runs[l]
                    line = theta[l, s0:s0 + n]
                    pos = [i - s0 for (j, i) in nodes]
                else:
                    s0, n = g.col_runs[l]
                    line = theta[s0:s0 + n, l]
                    pos = [j - s0 for (j, i) in nodes]
                D = fcgram.dense_operator(n, self.prm.fc_d, self.prm.fc_C, "d1")
                rest = np.ones(n, dtype=bool)
                rest[pos] = False
                A = D[np.ix_(pos, pos)]
                rhs = -(D[np.ix_(pos, np.flatnonzero(rest))] @ line[rest])
                for node, th in zip(nodes, np.linalg.solve(A, rhs)):
                    fixed[node] = th
            for (j, i), th in fixed.items():
                rho = e[0, j, i]
                e[1, j, i] = e[2, j, i] = 0.0
                e[3, j, i] = rho * th
            # Dirichlet data: inflow sides, exact-data fringe
            for (j, i, kind, direction) in g.boundary:
                if kind == patches.INFLOW:
                    e[:, j, i] = euler.prim_to_cons(np.asarray(g.p.inflow, dtype=float), gam)
            if g.xfringe.any():
                jj, ii = np.nonzero(g.xfringe)
                w = self.exact(g.p.x[jj, ii], g.p.y[jj, ii], t_stage)
                e[:, jj, ii] = euler.prim_to_cons(w, gam)
        if not fringe:
            return U
        src = U.copy()
        for p, rows in enumerate(self.fringe_rows):
            e = self.view(U, p)
            for (j, i, s, ent) in rows:
                d = self.view(src, s)
                e[:, j, i] = sum(w * d[:, jd, id_] for jd, id_, w in ent)
        return U

    # ----------------------------------------------------------- per step
    def classifier(self):
        if self.prm.av == "sdnn":
            return lambda wins: sdnn.classify(self.sdnn_params, wins)
        return sdnn.modal_classify

    def compute_viscosity(self, U):
        """Alg. 3 on every subpatch, then the blend (Alg. 1, viscosity line)."""
        prm = self.prm
        mu_t = []
        taus = []
        for p, g in enumerate(self.grids):
            e = self.view(U, p)
            if self.tau_override is not None:
                tau = self.tau_override[p]
            else:
                tau = viscosity.classify_patch(e, g, self.classifier(), prm.gamma)
            taus.append(tau)
            mh = viscosity.preliminary(e, g, tau, prm.c_mu, prm.gamma)
            mu_t.append(np.where(g.p.mask, viscosity.smooth_fast(mh, prm.n_v), 0.0))
        self.last_tau = taus
        mu = np.zeros(self.offsets[-1])
        for p, g in enumerate(self.grids):
            out = mu_t[p].copy()
            if self.blend is not None:
                for (j, i), ent in self.blend[p].items():
                    out[j, i] = sum(w * mu_t[s][jd, id_] for (s, jd, id_), w in ent)
            out = np.maximum(out, 0.0)
            mu[self.offsets[p]:self.offsets[p + 1]] = out.ravel()
        mu1 = np.zeros_like(mu)
        mu2 = np.zeros_like(mu)
        for p, g in enumerate(self.grids):
            f = self.field(mu, p)
            mu1[self.offsets[p]:self.offsets[p + 1]] = g.deriv(f, 0).ravel()
            mu2[self.offsets[p]:self.offsets[p + 1]] = g.deriv(f, 1).ravel()
        return mu, mu1, mu2

    def apply_filter(self, U):
        """Alg. 4 (t > 0): filter rho, rho u, rho v and theta along both
        directions, then rebuild E from the filtered values."""
        gam = self.prm.gamma
        out = U.copy()
        for p, g in enumerate(self.grids):
            e = self.view(U, p)
            m = g.p.mask
            ee = np.where(m, e, np.array([1.0, 0.0, 0.0, 1.0])[:, None, None])
            theta = np.where(m, euler.temperature_like(ee, gam), 0.0)
            q = np.stack([e[0], e[1], e[2], theta])
            q = g.deriv(g.deriv(q, 0, "filter"), 1, "filter")
            rho, mx, my, th = q
            rr = np.where(m, rho, 1.0)
            E = rho * th + 0.5 * (mx * mx + my * my) / rr
            v = self.view(out, p)
            v[...] = np.where(m, np.stack([rho, mx, my, E]), 0.0)
        return out

    def smear_initial_data(self, U):
        """Alg. 4 at t = 0 (reading of Part I's localized smearing, which is
        not available): near discontinuities the initial data are replaced
        by a more strongly filtered version, blended in smoothly.

        1. indicator: 1 at the non-fringe points whose class (either
           direction) flags a discontinuity in the window, from the first
           step's classification (Alg. 3 on the same data);
        2. window w in [0, 1]: the indicator localized exactly as the
           preliminary viscosity (windowed max over n_v, then the
           multi-patch blend), clipped to [0, 1];
        3. the strong filter (order SMEAR_ORDER) along q^1 then q^2 of rho,
           rho u, rho v and theta, as the filter of t > 0 does with its own
           order;
        4. (rho, rho u, rho v, theta) <- w * filtered + (1 - w) * given, and E
           rebuilt from them."""
        gam, n_v = self.prm.gamma, self.prm.n_v
        w_t = []
        for p, g in enumerate(self.grids):
            tau = self.last_tau[p]
            ind = (np.maximum(tau[0], tau[1]) >= 1) & g.p.mask & ~g.fringe & ~g.xfringe
            w_t.append(np.where(g.p.mask, viscosity.smooth_fast(ind.astype(np.float64), n_v), 0.0))
        out = U.copy()
        for p, g in enumerate(self.grids):
            w = w_t[p].copy()
            if self.blend is not None:
                for (j, i), ent in self.blend[p].items():
                    w[j, i] = sum(c * w_t[s][jd, id_] for (s, jd, id_), c in ent)
            w = np.clip(w, 0.0, 1.0)
            e = self.view(U, p)
            m = g.p.mask
            ee = np.where(m, e, np.array([1.0, 0.0, 0.0, 1.0])[:, None, None])
            theta = np.where(m, euler.temperature_like(ee, gam), 0.0)
            q = np.stack([e[0], e[1], e[2], theta])
            qs = g.deriv(g.deriv(q, 0, "smear"), 1, "smear")
            rho, mx, my, th = w * qs + (1.0 - w) * q
            rr = np.where(m, rho, 1.0)
            E = rho * th + 0.5 * (mx * mx + my * my) / rr
            self.view(out, p)[...] = np.where(m, np.stack([rho, mx, my, E]), 0.0)
        return out

    def timestep(self, U, mu):
        """Adaptive step (reading of I-(31)): CFL times the minimum over all
        points of h_x / (|u| + a) and h_x^2 / (4 mu).  The factor 4 keeps the
        viscous eigenvalues (two directions, Fourier second derivative up to
        pi^2 / h^2 each) inside the real-axis stability interval of SSPRK(5,4)
        (|z| <= 5.33) for CFL <= 1."""
        if self.prm.dt_fixed is not None:
            return self.prm.dt_fixed
        best = np.inf
        for p, g in enumerate(self.grids):
            m = g.p.mask
            e = self.view(U, p)[:, m]
            s = np.sqrt(e[1] ** 2 + e[2] ** 2) / e[0] + euler.sound_speed(e, self.prm.gamma)
            h = g.hx[m]
            best = min(best, np.min(h / s))
            if mu is not None:
                mp_ = self.field(mu[0], p)[m]
                pos = mp_ > 0
                if pos.any():
                    best = min(best, np.min(h[pos] ** 2 / (4.0 * mp_[pos])))
        return self.prm.cfl * best

    def step(self):
        prm = self.prm
        if self.nstep == 0:
            # the initial data are made to satisfy the boundary conditions
            # (walls, inflow, exact data), as the solution does after every
            # stage; the first step's viscosity then sees the jumps the walls
            # impose.  The fringe points keep the data's own values (given
            # pointwise): interpolating discontinuous initial data would
            # overshoot, and the first stage's fringe fill follows the
            # smearing.
            self.U = self.enforce(self.U, self.t, fringe=False)
        self.mu = self.compute_viscosity(self.U) if prm.av != "off" else None
        if prm.filter and self.nstep > 0:
            self.U = self.apply_filter(self.U)
        elif prm.smear and self.nstep == 0:
            self.U = self.smear_initial_data(self.U)
        dt = self.timestep(self.U, self.mu)
        self.last_dt = dt
        ct = ssprk.stage_times()
        t0 = self.t
        self.U = ssprk.step(self.U, dt, lambda u, k: self.rhs(u),
                            lambda u, k: self.enforce(u, t0 + ct[k] * dt))
        self.t = t0 + dt
        self.nstep += 1
        return dt

    def prim(self, p):
        return euler.cons_to_prim(np.where(self.grids[p].p.mask, self.view(self.U, p), np.array([1.0, 0, 0, 1.0])[:, None, None]), self.prm.gamma)


def patches_from_specs(specs):
    """Oracle patches from plain subpatch descriptions (objects with x, y,
    mask, sides, notch, inflow and kind attributes)."""
    return [patches.Patch(s.x, s.y, s.mask, dict(s.sides), s.notch,
                          None if s.inflow is None else np.asarray(s.inflow, dtype=float), s.kind)
            for s in specs]
