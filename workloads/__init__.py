"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the method: it only lays out subpatch
node coordinates, activity masks and side kinds, initial primitive states and
random test data.  Geometry follows the shapes of the paper's workloads
(Sec. 3 patch types, Sec. 7 test configurations); all inputs are synthetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

INTERNAL, INFLOW, OUTFLOW, SLIP, EXACT, NOSLIP = 0, 1, 2, 3, 4, 5
GAMMA = 1.4
SEED_BASE = 25061937


def rng(config_index: int, salt: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + config_index + 7919 * salt))


@dataclass
class PatchSpec:
    """One subpatch: node coordinates (n2, n1), optional activity mask,
    side kinds W, E, S, N, kind of the mask boundary, inflow state."""
    x: np.ndarray
    y: np.ndarray
    mask: np.ndarray | None = None
    sides: dict = field(default_factory=lambda: {"W": INTERNAL, "E": INTERNAL, "S": INTERNAL, "N": INTERNAL})
    notch: int = SLIP
    inflow: tuple | None = None
    kind: str = "I"

    @property
    def shape(self):
        return self.x.shape

    def npoints(self):
        return int(self.x.size if self.mask is None else self.mask.sum())


def box_patch(x0, x1, y0, y1, n1, n2, sides, kind="I", inflow=None):
    """Cartesian subpatch on [x0, x1] x [y0, y1] with n1 x n2 nodes."""
    xs = np.linspace(x0, x1, n1)
    ys = np.linspace(y0, y1, n2)
    X, Y = np.meshgrid(xs, ys)
    return PatchSpec(X, Y, None, dict(sides), SLIP, inflow, kind)


def lattice_patch(h, X0, X1, Y0, Y1, sides, kind="I", inflow=None, notch_box=None):
    """Subpatch whose nodes are the lattice points (X h, Y h) for integer X in
    [X0, X1], Y in [Y0, Y1]; ``notch_box`` = (Xa, Xb, Ya, Yb) masks the lattice
    points with Xa <= X <= Xb and Ya <= Y <= Yb (the obstacle quadrant of an
    L-shaped C1 corner subpatch)."""
    Xi = np.arange(X0, X1 + 1)
    Yi = np.arange(Y0, Y1 + 1)
    XX, YY = np.meshgrid(Xi, Yi)
    mask = None
    if notch_box is not None:
        Xa, Xb, Ya, Yb = notch_box
        mask = ~((XX >= Xa) & (XX <= Xb) & (YY >= Ya) & (YY <= Yb))
    return PatchSpec(XX * h, YY * h, mask, dict(sides), SLIP, inflow, kind)


# ---------------------------------------------------------------- single-patch vortex
def vortex_box(n=101, L=10.0):
    """One Cartesian patch n x n over [0, L]^2 with exact-data sides (the
    single-patch FP64 configuration)."""
    s = {k: EXACT for k in "WESN"}
    return [box_patch(0.0, L, 0.0, L, n, n, s, kind="I")]


def vortex_multipatch(n=41):
    """Four overlapping patches over [0, 10]^2 whose grids do not coincide:
    the communication is a true interpolation."""
    s = {k: EXACT for k in "WESN"}
    out = []
    h = 10.0 / (2 * n - 20)
    # left column: spacing h; right column: spacing 0.93 h, shifted
    for (xa, xb, nx) in ((0.0, (n - 1) * h, n), (10.0 - (n + 3) * 0.93 * h, 10.0, n + 4)):
        for (ya, yb, ny) in ((0.0, (n - 1) * h, n), (10.0 - (n + 1) * 0.97 * h, 10.0, n + 2)):
            sides = dict(s)
            sides["E" if xa == 0.0 else "W"] = INTERNAL
            sides["N" if ya == 0.0 else "S"] = INTERNAL
            out.append(box_patch(xa, xb, ya, yb, nx, ny, sides))
    return out


def vortex_curved_pair(n=61):
    """Two overlapping curvilinear patches covering [0, 10]^2 for the vortex:
    A maps q in [0, 6] x [0, 10], B maps q in [4, 10] x [0, 10] (spacing
    0.93 of A's), each perturbed by a different smooth bump that vanishes on
    the outer box edges, so the overlap's grid lines are curved and do not
    coincide: the fringe is filled by interpolation with donors found by
    Newton inversion of a curved mapping.  Outer sides carry exact vortex
    data, the curved inner sides are internal."""
    h = 10.0 / (n - 1)
    out = []
    for (qa, qb, hh, ax, ay, sx) in ((0.0, 6.0, h, 0.3, 0.2, 1.0), (4.0, 10.0, 0.93 * h, -0.25, -0.15, -1.0)):
        n1 = int(round((qb - qa) / hh)) + 1
        n2 = int(round(10.0 / hh)) + 1
        q1 = np.linspace(qa, qb, n1)[None, :]
        q2 = np.linspace(0.0, 10.0, n2)[:, None]
        # bump: zero on the outer edge of the patch (x = 0 or x = 10) and on y = 0, 10
        r = (q1 - qa) / (qb - qa) if sx > 0 else (qb - q1) / (qb - qa)
        X = q1 + ax * np.sin(np.pi * q2 / 10.0) * r * r
        Y = q2 + ay * np.sin(np.pi * (q1 - qa) / (qb - qa)) * np.sin(np.pi * q2 / 10.0) * r
        sides = {k: EXACT for k in "WESN"}
        sides["E" if sx > 0 else "W"] = INTERNAL
        out.append(PatchSpec(X, Y, None, sides, SLIP, None, "I"))
    return out


def curved_patch(n1=48, n2=40, amp=0.05):
    """A curvilinear patch (sinusoidally perturbed unit square), for
    freestream-preservation checks."""
    q1 = np.linspace(0, 1, n1)
    q2 = np.linspace(0, 1, n2)
    Q1, Q2 = np.meshgrid(q1, q2)
    X = Q1 + amp * np.sin(2 * np.pi * Q2)
    Y = Q2 + amp * np.sin(2 * np.pi * Q1) * 0.5 + 0.1 * Q1 * Q2
    return [PatchSpec(X, Y, None, {k: EXACT for k in "WESN"}, SLIP, None, "I")]


def annular_sector(n1=48, n2=32, r0=1.0, r1=2.0, th0=0.0, th1=np.pi / 3):
    q1 = np.linspace(0, 1, n1)
    q2 = np.linspace(0, 1, n2)
    Q1, Q2 = np.meshgrid(q1, q2)
    th = th0 + (th1 - th0) * Q1
    r = r0 + (r1 - r0) * Q2
    return [PatchSpec(r * np.cos(th), r * np.sin(th), None, {k: EXACT for k in "WESN"}, SLIP, None, "S")]


# ---------------------------------------------------------------- reflecting Sod box
SOD_LEFT = (1.0, 0.0, 0.0, 1.0)
SOD_RIGHT = (0.125, 0.0, 0.0, 0.1)


def sod_reflect(h_index=200, nsub=4):
    """2-D Sod problem on [0, 1] x [0, 0.25] (lattice spacing 1 / h_index):
    one patch split along x into nsub overlapping subpatches (neighbouring
    cores share 17 points), reflecting (slip) walls on all four sides."""
    h = 1.0 / h_index
    XE, YT = h_index, h_index // 4
    e = 8
    cuts = [int(round(XE * k / nsub)) for k in range(nsub + 1)]
    out = []
    for k in range(nsub):
        X0 = cuts[k] - (e if k > 0 else 0)
        X1 = cuts[k + 1] + (e if k < nsub - 1 else 0)
        sides = {"W": SLIP if k == 0 else INTERNAL, "E": SLIP if k == nsub - 1 else INTERNAL, "S": SLIP, "N": SLIP}
        out.append(lattice_patch(h, X0, X1, 0, YT, sides, "I"))
    return out


def sod_reflect_cores(h_index=200, nsub=4):
    """Global lattice column ranges [c0, c1) owned by each subpatch of
    sod_reflect (its core; the last one includes x = 1), for integrals over
    the union without counting overlaps twice."""
    XE = h_index
    cuts = [int(round(XE * k / nsub)) for k in range(nsub + 1)]
    return [(cuts[k], cuts[k + 1] + (1 if k == nsub - 1 else 0)) for k in range(nsub)]


def sod_state(patch_list):
    """Primitive Sod data: left state for x < 0.5, right state for x >= 0.5."""
    out = []
    for s in patch_list:
        left = (s.x < 0.5)[None]
        out.append(np.where(left, np.asarray(SOD_LEFT, float)[:, None, None],
                            np.asarray(SOD_RIGHT, float)[:, None, None]))
    return out


# ---------------------------------------------------------------- Mach-M shock tube
def mach_shock_states(M, gamma=1.4):
    """Primitive states behind and ahead of a shock travelling at speed M into
    gas at rest with (rho, p) = (1.4, 1) (sound speed 1): the
    Rankine-Hugoniot jump of pressure zeta, velocity (zeta - 1) / (gamma M)
    and density ratio (gamma + 1) M^2 / ((gamma - 1) M^2 + 2)."""
    zeta = (2 * gamma * M * M - gamma + 1) / (gamma + 1)
    ratio = (gamma + 1) * M * M / ((gamma - 1) * M * M + 2)
    ahead = (1.4, 0.0, 0.0, 1.0)
    behind = (1.4 * ratio, (zeta - 1) / (gamma * M), 0.0, zeta)
    return behind, ahead


def mach_shock_tube(M, h_index=200, nsub=4):
    """Channel [0, 1] x [0, 0.25] split along x into nsub overlapping
    subpatches (neighbouring cores share 17 points): inflow of the post-shock
    state at x = 0, outflow at x = 1, slip walls at y = 0 and y = 0.25."""
    behind, _ = mach_shock_states(M)
    h = 1.0 / h_index
    XE, YT = h_index, h_index // 4
    e = 8
    cuts = [int(round(XE * k / nsub)) for k in range(nsub + 1)]
    out = []
    for k in range(nsub):
        X0 = cuts[k] - (e if k > 0 else 0)
        X1 = cuts[k + 1] + (e if k < nsub - 1 else 0)
        sides = {"W": INFLOW if k == 0 else INTERNAL, "E": OUTFLOW if k == nsub - 1 else INTERNAL,
                 "S": SLIP, "N": SLIP}
        out.append(lattice_patch(h, X0, X1, 0, YT, sides, "I", behind))
    return out


def mach_shock_state(patch_list, M, x_s):
    """The Mach-M shock data: post-shock state for x < x_s, gas at rest ahead."""
    behind, ahead = mach_shock_states(M)
    return [np.where((s.x < x_s)[None], np.asarray(behind, float)[:, None, None],
                     np.asarray(ahead, float)[:, None, None]) for s in patch_list]


# ---------------------------------------------------------------- Mach 3 step channel
STEP_INFLOW = (1.4, 3.0, 0.0, 1.0)


def step_channel(h_index=250):
    """Mach 3 channel [0, 3] x [0, 1] with a step occupying [0.6, 3] x [0, 0.2]
    (lattice spacing h = 1 / h_index).  Subpatches: an S/inflow column, a C2
    corner patch at the foot of the step face, an L-shaped C1 corner patch at
    the step corner, patches above it and two rows of patches over the step;
    all share one lattice, so overlaps are exchanges."""
    h = 1.0 / h_index
    s = h_index / 250.0
    I = lambda v: int(round(v * s))
    XW, XS, YS, XE, YT = 0, I(150), I(50), I(750), I(250)  # x = 0, 0.6 ; y = 0.2 ; x = 3 ; y = 1
    e = 8  # half overlap: neighbouring cores overlap by 2 e + 1 points
    pts = []

    def add(X0, X1, Y0, Y1, W, E, S, N, kind="I", notch=None):
        pts.append(lattice_patch(h, X0, X1, Y0, Y1, {"W": W, "E": E, "S": S, "N": N}, kind,
                                 STEP_INFLOW, notch))

    A1 = I(110)
    ylev = [0, YS, I(150), YT]
    # inflow column x in [0, A1]: two columns of cores, three rows
    xa = [XW, I(55), A1]
    for c in range(2):
        for r in range(3):
            X0 = xa[c] - (e if c > 0 else 0)
            X1 = xa[c + 1] + e
            Y0 = ylev[r] - (e if r > 0 else 0)
            Y1 = ylev[r + 1] + (e if r < 2 else 0)
            add(X0, X1, Y0, Y1, INFLOW if c == 0 else INTERNAL, INTERNAL,
                SLIP if r == 0 else INTERNAL, SLIP if r == 2 else INTERNAL,
                "S" if (c == 0 or r in (0, 2)) else "I")
    B0, B1 = A1 - e, I(190) + e
    # C2 corner patch: step face (east) and bottom wall (south)
    add(B0, XS, 0, YS, INTERNAL, SLIP, SLIP, INTERNAL, "C2")
    # C1 L-shaped corner patch around (0.6, 0.2); the quadrant x > 0.6, y < 0.2 is the obstacle
    Ly0, Ly1 = I(10), I(90) + e
    add(B0, B1, Ly0, Ly1, INTERNAL, INTERNAL, INTERNAL, INTERNAL, "C1", notch=(XS + 1, B1, Ly0, YS - 1))
    # above the L patch
    add(B0, B1, I(90) - e, I(165) + e, INTERNAL, INTERNAL, INTERNAL, INTERNAL, "I")
    add(B0, B1, I(165) - e, YT, INTERNAL, INTERNAL, INTERNAL, SLIP, "S")
    # over the step: columns of cores between x = 0.76 and x = 3
    xr = [I(190), I(285), I(380), I(475), I(570), I(660), XE]
    yr = [YS, I(150), YT]
    for c in range(len(xr) - 1):
        last = c == len(xr) - 2
        X0 = xr[c] - e
        X1 = xr[c + 1] + (0 if last else e)
        for r in range(2):
            Y0 = yr[r] - (e if r > 0 else 0)
            Y1 = yr[r + 1] + (e if r == 0 else 0)
            add(X0, X1, Y0, Y1, INTERNAL, OUTFLOW if last else INTERNAL,
                SLIP if r == 0 else INTERNAL, SLIP if r == 1 else INTERNAL, "S")
    return pts


def _split(lo, hi, cmin, cmax, g):
    """Cut points lo = c_0 < ... < c_k = hi: k pieces of lengths drawn
    uniformly in [cmin, cmax], rescaled to fill [lo, hi] exactly."""
    span = hi - lo
    k = max(1, int(round(span / (0.5 * (cmin + cmax)))))
    w = g.uniform(cmin, cmax, k)
    c = lo + np.rint(np.cumsum(w) / w.sum() * span).astype(int)
    return [lo] + [int(v) for v in c]


def step_channel_tiled(h_index=2000, smin=150, smax=300, corner=140, config_index=5, seed_salt=0):
    """The Mach-3 step channel ([0, 3] x [0, 1], step [0.6, 3] x [0, 0.2]) on
    one lattice of spacing 1 / h_index, tiled by subpatches of uneven sizes:
    core extents are drawn (seeded) so that a subpatch side, with the
    17-point overlaps on its internal sides, lies in [smin, smax].  Columns of
    cores in front of the step; a corner column of width 2 corner around
    x = 0.6 with a C2 patch at the foot of the step face, an L-shaped C1
    patch around the step corner and cores above it; columns of cores over
    the step.  Side kinds: inflow at x = 0, outflow at x = 3, slip walls on
    y = 0, y = 1, the step face and the step top."""
    assert h_index % 5 == 0
    g = rng(config_index, seed_salt)
    h = 1.0 / h_index
    XS, YS, XE, YT = 3 * h_index // 5, h_index // 5, 3 * h_index, h_index
    a, e = corner, 8
    assert 2 * e < YS - a and a + 2 * e < YS
    cmin, cmax = smin - 2 * e - 1, smax - 2 * e - 1
    pts = []

    def add(x0, x1, y0, y1, W, E, S, N, kind=None, notch=None):
        X0, X1 = x0 - (e if W == INTERNAL else 0), x1 + (e if E == INTERNAL else 0)
        Y0, Y1 = y0 - (e if S == INTERNAL else 0), y1 + (e if N == INTERNAL else 0)
        if kind is None:
            kind = "I" if (W, E, S, N) == (INTERNAL,) * 4 else "S"
        pts.append(lattice_patch(h, X0, X1, Y0, Y1, {"W": W, "E": E, "S": S, "N": N}, kind, STEP_INFLOW, notch))

    def column(x0, x1, ylo, yhi, wall_below):
        ys = _split(ylo, yhi, cmin, cmax, g)
        for r in range(len(ys) - 1):
            add(x0, x1, ys[r], ys[r + 1], INFLOW if x0 == 0 else INTERNAL, OUTFLOW if x1 == XE else INTERNAL,
                SLIP if (r == 0 and wall_below) else INTERNAL, SLIP if ys[r + 1] == YT else INTERNAL)

    # in front of the step
    xs = _split(0, XS - a, cmin, cmax, g)
    for c in range(len(xs) - 1):
        column(xs[c], xs[c + 1], 0, YT, True)
    # corner column: C2 at the foot of the step face, C1 around the step corner, cores above
    add(XS - a, XS, 0, YS - a, INTERNAL, SLIP, SLIP, INTERNAL, "C2")
    add(XS - a, XS + a, YS - a, YS + a, INTERNAL, INTERNAL, INTERNAL, INTERNAL, "C1",
        notch=(XS + 1, XS + a + e, YS - a - e, YS - 1))
    column(XS - a, XS + a, YS + a, YT, False)
    # over the step
    xs = _split(XS + a, XE, cmin, cmax, g)
    for c in range(len(xs) - 1):
        column(xs[c], xs[c + 1], YS, YT, True)
    return pts


def uniform_state(patch_list, prim):
    return [np.broadcast_to(np.asarray(prim, dtype=float)[:, None, None], (4,) + p.shape).copy()
            for p in patch_list]


# ---------------------------------------------------------------- derivative sweep
FIELD_OFFSET_SCALE = ((1.4, 0.14), (4.2, 0.42), (0.0, 0.42), (8.8, 0.88))


def deriv_sweep(npatch=2000, nmin=64, nmax=256, config_index=3, seed_salt=0):
    """Patches with sides drawn uniformly from [nmin, nmax] and four fields of
    smooth random trigonometric sums (Mach-3 freestream magnitudes), with a
    jump added along 5 % of the q^1 lines and 5 % of the q^2 lines.
    Returns (sizes (npatch, 2) as (n1, n2), list of fields (4, n2, n1))."""
    g = rng(config_index, seed_salt)
    sizes = g.integers(nmin, nmax + 1, size=(npatch, 2))
    return sizes, sweep_fields(sizes, g)


def sweep_fields(sizes, g):
    """The four fields of deriv_sweep on patches of the given (n1, n2) sizes,
    drawn from the generator g."""
    fields = []
    for (n1, n2) in sizes:
        q1 = np.linspace(0, 1, n1)[None, :]
        q2 = np.linspace(0, 1, n2)[:, None]
        f = np.empty((4, n2, n1))
        for c, (off, sc) in enumerate(FIELD_OFFSET_SCALE):
            a = g.standard_normal(8) / np.sqrt(8)
            k1 = g.uniform(-6, 6, 8)
            k2 = g.uniform(-6, 6, 8)
            ph = g.uniform(0, 2 * np.pi, 8)
            v = np.zeros((n2, n1))
            for k in range(8):
                v += a[k] * np.cos(2 * np.pi * (k1[k] * q1 + k2[k] * q2) + ph[k])
            rows = np.flatnonzero(g.random(n2) < 0.05)
            for j in rows:
                qj = g.uniform(0.1, 0.9)
                v[j] += g.uniform(0.1, 1.0) * (q1[0] >= qj)
            cols = np.flatnonzero(g.random(n1) < 0.05)
            for i in cols:
                qj = g.uniform(0.1, 0.9)
                v[:, i] += g.uniform(0.1, 1.0) * (q2[:, 0] >= qj)
            f[c] = off + sc * v
        fields.append(f)
    return fields


# ---------------------------------------------------------------- classifier weights
SDNN_SHAPES = (("W1", (64, 16)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (3, 64)), ("b3", (3,)))


def sdnn_init(g: np.random.Generator):
    """Seeded He-normal initial parameters of the 16-64-64-3 classifier,
    FP32 values; biases zero."""
    out = {}
    for name, shape in SDNN_SHAPES:
        if name.startswith("b"):
            out[name] = np.zeros(shape, dtype=np.float32)
        else:
            out[name] = (g.standard_normal(shape) * np.sqrt(2.0 / shape[1])).astype(np.float32)
    return out


def sdnn_blob(params) -> np.ndarray:
    return np.concatenate([np.asarray(params[k], dtype=np.float32).ravel() for k, _ in SDNN_SHAPES])


def sdnn_unblob(blob) -> dict:
    out, o = {}, 0
    for k, shape in SDNN_SHAPES:
        n = int(np.prod(shape))
        out[k] = np.asarray(blob[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


# ---------------------------------------------------------------- classifier lines
def classifier_lines(nlines, n=101, config_index=4, seed_salt=0):
    """Raw synthetic lines for the smoothness classifier: smooth random
    Fourier sums plus 0-2 jumps at uniform positions with log-uniform
    amplitudes in [1e-3, 1] and random sign.  Returns (lines (nlines, n),
    jump positions (nlines, 2) in index units, NaN when absent, jump
    amplitudes (nlines, 2))."""
    g = rng(config_index, seed_salt)
    x = np.linspace(0, 1, n)
    lines = np.zeros((nlines, n))
    K = g.integers(1, 13, size=nlines)
    for r in range(nlines):
        b = g.standard_normal(K[r]) / np.arange(1, K[r] + 1)
        ph = g.uniform(0, 2 * np.pi, K[r])
        lines[r] = (b[:, None] * np.sin(2 * np.pi * np.arange(1, K[r] + 1)[:, None] * x[None, :] + ph[:, None])).sum(0)
    nj = g.integers(0, 3, size=nlines)
    pos = np.full((nlines, 2), np.nan)
    amp = np.zeros((nlines, 2))
    for r in range(nlines):
        for k in range(nj[r]):
            q = g.uniform(0.02, 0.98)
            a = 10.0 ** g.uniform(-3, 0) * (1 if g.random() < 0.5 else -1)
            pos[r, k] = q * (n - 1)
            amp[r, k] = a
            lines[r] += a * (x >= q)
    return lines, pos, amp


def window_labels(pos, amp, lines, n=101, rel_tol=1e-2):
    """Class of the 16-point window of every point of every line: 2 when a
    significant jump lies within 2 points of the point, 1 when one lies
    elsewhere in the window, else 0 (a jump is significant when its amplitude
    is at least rel_tol times the line's range)."""
    nl = lines.shape[0]
    start = np.clip(np.arange(n) - 8, 0, n - 16)
    lab = np.zeros((nl, n), dtype=np.int64)
    rngv = lines.max(axis=1) - lines.min(axis=1)
    for k in range(pos.shape[1]):
        p = pos[:, k]
        sig = np.isfinite(p) & (np.abs(amp[:, k]) >= rel_tol * np.maximum(rngv, 1e-300))
        pp = np.where(np.isfinite(p), p, -1e9)[:, None]
        i = np.arange(n)[None, :]
        inwin = (pp >= start[None, :]) & (pp <= start[None, :] + 15)
        near = np.abs(pp - i) <= 2.0
        lab = np.where(sig[:, None] & near, 2, np.where(sig[:, None] & inwin & (lab < 2), np.maximum(lab, 1), lab))
    return lab


# ---------------------------------------------------------------- Mach-M wedge tunnel
WEDGE_INFLOW = (1.4, 10.0, 0.0, 1.0)
# Mach number of the wedge runs.  The impulsive start from the uniform stream
# (quiescent gas behind the rear face) keeps rho, p > 0 at Mach 10 with the
# localized smearing of the initial data (Alg. 4 at t = 0); without it, only
# up to Mach 6.5 on this decomposition
WEDGE_MACH = 10.0


def wedge_geometry(h_index, tip_x=0.2, length=0.2, half_angle_deg=15.0, yc=0.25):
    """The obstacle of the wedge tunnel in lattice index units (spacing
    1 / h_index): tip T, rear corners R+ (upper) and R- (lower), the unit
    vectors u and l of the upper and lower faces (from the tip towards the
    rear) and the rear half-height H."""
    th = np.deg2rad(half_angle_deg)
    Xt, Xr, Yc = tip_x * h_index, (tip_x + length) * h_index, yc * h_index
    H = (Xr - Xt) * np.tan(th)
    u = np.array([np.cos(th), np.sin(th)])
    l = np.array([np.cos(th), -np.sin(th)])
    return dict(T=np.array([Xt, Yc]), Rp=np.array([Xr, Yc + H]), Rm=np.array([Xr, Yc - H]), u=u, l=l, H=H,
                Xt=Xt, Xr=Xr, Yc=Yc, theta=th)


def _affine_patch(h, origin, e1, e2, i0, i1, j0, j1, sides, kind, inflow, mask=None, notch=SLIP):
    """Nodes origin + i e1 + j e2 (index units, scaled by h) for integer i in
    [i0, i1], j in [j0, j1]."""
    I = np.arange(i0, i1 + 1, dtype=float)[None, :]
    J = np.arange(j0, j1 + 1, dtype=float)[:, None]
    X = (origin[0] + I * e1[0] + J * e2[0]) * h
    Y = (origin[1] + I * e1[1] + J * e2[1]) * h
    return PatchSpec(X, Y, mask, dict(sides), notch, inflow, kind)


def _c1_patch(h, C, e1, e2, m, inflow):
    """C1 corner subpatch around the corner C of two straight walls: the map
    q -> l_A(q^1) + l_B(q^2) - C with straight arcs l_A, l_B of directions e1,
    e2 (index units), on (2m + 1)^2 nodes; the quadrant i < m, j < m (the
    obstacle, C - a e1 - b e2 with a, b > 0) is masked; the mask boundary is
    the two walls, the four outer sides are internal."""
    n = 2 * m + 1
    II, JJ = np.meshgrid(np.arange(n), np.arange(n))
    mask = ~((II < m) & (JJ < m))
    return _affine_patch(h, C - m * e1 - m * e2, e1, e2, 0, n - 1, 0, n - 1,
                         {k: INTERNAL for k in "WESN"}, "C1", inflow, mask, SLIP)


def _mirror(spec, Yc_phys):
    """Mirror image of a subpatch in the line y = Yc_phys, rows reversed so
    that the node ordering keeps its orientation (S and N sides swap)."""
    sides = dict(spec.sides)
    sides["S"], sides["N"] = spec.sides["N"], spec.sides["S"]
    mask = None if spec.mask is None else spec.mask[::-1].copy()
    return PatchSpec(spec.x[::-1].copy(), 2 * Yc_phys - spec.y[::-1], mask, sides, spec.notch, spec.inflow,
                     spec.kind)


def _keepout_extent(geo, xa, xb, delta):
    """y-range of the points within distance delta of the obstacle over the
    abscissae [xa, xb] (index units), or None."""
    T, Rp, Rm = geo["T"], geo["Rp"], geo["Rm"]
    pts = []
    for a, b in ((T, Rp), (Rp, Rm), (Rm, T)):
        t = np.linspace(0.0, 1.0, 4001)[:, None]
        pts.append(a[None, :] * (1 - t) + b[None, :] * t)
    pts = np.concatenate(pts)
    dx = np.maximum(0.0, np.maximum(xa - pts[:, 0], pts[:, 0] - xb))
    ok = dx <= delta
    if not ok.any():
        return None
    r = np.sqrt(delta * delta - dx[ok] ** 2)
    return float((pts[ok, 1] - r).min()), float((pts[ok, 1] + r).max())


def wedge_tunnel(h_index=4400, smin=150, smax=300, config_index=5, seed_salt=1, tip_x=0.2, length=0.2,
                 half_angle_deg=15.0, mach=WEDGE_MACH):
    """Mach-10 flow past a wedge with a blunt rear face in the tunnel
    [0, 1] x [0, 0.5] (lattice spacing h = 1 / h_index).  The obstacle is the
    triangle with tip T = (tip_x, 0.25), faces at +-half_angle_deg to the
    flow and a vertical rear face at x = tip_x + length (the prism shape of
    the paper's flow-past-prism experiment, with a narrower front angle).

    Subpatches (Sec. 3 patch types):
    - C1 corner subpatches (2m + 1)^2 around the tip and the two rear
      corners, each the affine map of the L-shaped parameter domain built
      from the two straight walls (non-right angles: 30 degrees of obstacle
      at the tip, 75 at the rear corners);
    - skewed-affine S subpatches along each face (one axis along the face,
      the other vertical), one axis of slip wall;
    - S subpatches on the rear face (lattice, slip wall on the west side);
    - lattice subpatches over the rest, in columns of seeded widths cut at the
      tip abscissa and at the rear face, each column split into rows of
      seeded heights and kept clear of a band of width delta around the
      obstacle; the column behind the rear face holds a wake block that
      starts delta downstream of the face.
    Sides are in [smin, smax] where the seeded draws set them.  Inflow of the
    Mach-M stream (1.4, M, 0, 1) at x = 0, outflow at x = 1, slip walls at
    y = 0, y = 0.5 and on the obstacle."""
    g = rng(config_index, seed_salt)
    h = 1.0 / h_index
    geo = wedge_geometry(h_index, tip_x, length, half_angle_deg)
    T, Rp, Rm, u, l, H = geo["T"], geo["Rp"], geo["Rm"], geo["u"], geo["l"], geo["H"]
    Xt, Xr, Yc = int(round(geo["Xt"])), int(round(geo["Xr"])), geo["Yc"]
    NX, NY = h_index, h_index // 2
    e = 8
    cmin, cmax = smin - 2 * e - 1, smax - 2 * e - 1
    m = min((smax - 1) // 2, int(0.45 * Xt))  # tip C1 arm (points)
    mr = min((smax - 1) // 2, int(0.6 * H))   # rear C1 arm (points)
    Ts = int(round(0.6 * smax))              # face S thickness (points, vertical)
    Tr = smin - 1                            # rear S thickness
    delta = max(3, int(round(0.02 * smax)))  # clearance of the lattice blocks
    inflow = (1.4, float(mach), 0.0, 1.0)
    out = []
    # --- body-fitted subpatches of the upper half, then their mirror images
    out.append(_c1_patch(h, T, -l, -u, m, inflow))  # on the symmetry line
    up = []
    up.append(_c1_patch(h, Rp, u, np.array([0.0, 1.0]), mr, inflow))
    Lf = (Xr - Xt) / np.cos(geo["theta"])
    nS = max(1, int(round(Lf / (0.5 * (smin + smax)))))
    cuts = np.rint(np.linspace(0, Lf, nS + 1)).astype(int)
    cuts[-1] = int(np.floor(Lf))
    for k in range(nS):
        i0 = cuts[k] - (e if k > 0 else 0)
        i1 = cuts[k + 1] + (e if k < nS - 1 else 0)
        up.append(_affine_patch(h, T, u, np.array([0.0, 1.0]), i0, i1, 0, Ts,
                                {"W": INTERNAL, "E": INTERNAL, "S": SLIP, "N": INTERNAL}, "S", inflow))
    out.extend(up)
    out.extend(_mirror(s, Yc * h) for s in up)
    # rear face: lattice S subpatches with the wall on the west side
    ra = int(round(0.35 * mr))
    Ya, Yb = int(np.ceil(Yc - H)) + ra, int(np.floor(Yc + H)) - ra
    nR = max(1, int(round((Yb - Ya) / (0.5 * (smin + smax)))))
    rc = np.rint(np.linspace(Ya, Yb, nR + 1)).astype(int)
    for k in range(nR):
        y0 = rc[k] - (e if k > 0 else 0)
        y1 = rc[k + 1] + (e if k < nR - 1 else 0)
        out.append(lattice_patch(h, Xr, Xr + Tr, y0, y1, {"W": SLIP, "E": INTERNAL, "S": INTERNAL, "N": INTERNAL},
                                 "S", inflow))
    # --- lattice blocks
    def rows(x0, x1, y0, y1, W, E, S, N):
        ys = _split(y0, y1, cmin, cmax, g)
        for r in range(len(ys) - 1):
            s_ = S if r == 0 else INTERNAL
            n_ = N if r == len(ys) - 2 else INTERNAL
            Y0 = ys[r] - (e if (r > 0) else 0)
            Y1 = ys[r + 1] + (e if r < len(ys) - 2 else 0)
            kind = "I" if (W, E, s_, n_) == (INTERNAL,) * 4 else "S"
            out.append(lattice_patch(h, x0, x1, Y0, Y1, {"W": W, "E": E, "S": s_, "N": n_}, kind, inflow))

    def colsplit(a, b, wmax):
        return _split(a, b, cmin, min(cmax, wmax), g)

    # the column just upstream of the tip is split around the axis: its width
    # stays within the reach of the tip patch, which covers that gap
    wl = max(cmin, min(cmax, int(1.4 * (m - 9)), int(1.93 * m - 56)))
    xs = colsplit(0, Xt - wl, cmax) + [Xt]
    xs = xs[:-1] + colsplit(Xt, Xr, int(0.75 * cmax))[:-1] + colsplit(Xr, NX, cmax)
    for c in range(len(xs) - 1):
        c0, c1 = xs[c], xs[c + 1]
        W = INFLOW if c0 == 0 else INTERNAL
        E = OUTFLOW if c1 == NX else INTERNAL
        xa, xb = c0 - (e if c0 > 0 else 0), c1 + (e if c1 < NX else 0)
        if c1 == Xt:
            xb = Xt + 2 * e  # past the vertical edge of the face subpatches at the tip
        ko = _keepout_extent(geo, xa, xb, delta)
        if ko is None:
            rows(xa, xb, 0, NY, W, E, SLIP, SLIP)
            continue
        ylo, yhi = int(np.floor(ko[0])), int(np.ceil(ko[1]))
        rows(xa, xb, 0, ylo, W, E, SLIP, INTERNAL)
        rows(xa, xb, yhi, NY, W, E, INTERNAL, SLIP)
        if c0 == Xr:
            # wake block behind the rear face, overlapping the blocks above and below
            rows(Xr + delta, xb, ylo - 2 * e, yhi + 2 * e, INTERNAL, E, INTERNAL, INTERNAL)
    return out


def wedge_state(patch_list, quiescent_wake=True, mach=WEDGE_MACH):
    """Initial data of the wedge tunnel: the uniform Mach-M stream
    (rho, u, v, p) = (1.4, M, 0, 1) (sound speed 1, the paper's Mach-M flow
    data) everywhere; with quiescent_wake (default), the gas behind the rear
    face (x > rear, |y - 0.25| < H) starts at rest: a stream leaving the rear
    face at Mach M from t = 0 would leave vacuum at the face."""
    out = uniform_state(patch_list, (1.4, float(mach), 0.0, 1.0))
    if quiescent_wake:
        geo = wedge_geometry(1.0)
        for s, w in zip(patch_list, out):
            wake = (s.x > geo["Xr"]) & (np.abs(s.y - geo["Yc"]) < geo["H"])
            w[1] = np.where(wake, 0.0, w[1])
    return out
