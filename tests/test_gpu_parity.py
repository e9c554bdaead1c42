"""GPU parity of the HIP path against the CPU oracle (MI355X, gfx950).

Tolerances (FP64 paths): the library builds its FC operators in quad
precision on the host, the oracle in 256-bit mpmath followed by an FP64 FFT
of the unit vectors; the two operators differ by <= 3e-12 (d = 5, where the
continuation values reach ~5e3 and the FFT rounds them) and <= 1e-14
(d = 2).  A contraction then differs by about that times max|f|, a stage
update by that times dt / h; the tolerances below are a few times those
bounds and are stated per test.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_19370_amd as F  # noqa: E402
import workloads as W  # noqa: E402
from oracle import exact, fcgram, solver as osolver  # noqa: E402


def _sweep_ref(fields):
    out1, out2 = [], []
    for f in fields:
        out1.append(fcgram.fc_apply(f, 5, 27, "d1"))
        out2.append(np.swapaxes(fcgram.fc_apply(np.swapaxes(f, -1, -2), 5, 27, "d1"), -1, -2))
    return out1, out2


def _variants():
    from paper_2506_19370_amd import _lib as L
    return [(p, tol, v) for p, tol in (("fp64", 2e-12), ("fp32", 2e-6), ("bf16x3", 1e-4), ("bf16x6", 2e-6))
            for v in range(L.fcs_gemm_variant_count(L.PREC[p]))]


@pytest.mark.parametrize("prec,tol,variant", _variants())
def test_sweep_parity(prec, tol, variant):
    """Grouped contraction over uneven patches (several 64 x 64 tiles and
    ragged tails) vs the oracle's FFT derivative; error relative to the
    largest field value of the component (the operator error multiplies the
    data, not its derivative).  FP32: unit roundoff 6e-8 times the operator's
    row sums of |entries| (<= 18) and the accumulation length; split BF16:
    two 8-bit halves leave ~2^-16 per product on the offset-free data."""
    sizes, fields = W.deriv_sweep(npatch=12, nmin=20, nmax=300, seed_salt=1)
    flat = np.concatenate([f.ravel() for f in fields])
    sw = F.DerivSweep(sizes, 4, prec, d=5, C=27)
    sw.set_variant(variant)  # every tile shape the autotuner may choose
    x = torch.tensor(flat, device="cuda")
    d1 = torch.zeros_like(x)
    d2 = torch.zeros_like(x)
    r1, r2 = _sweep_ref(fields)
    # twice: the persistent forms must leave their tile counters at zero
    for _ in range(2):
        d1.zero_()
        d2.zero_()
        sw.run(x, d1, d2)
        torch.cuda.synchronize()
        _check_sweep(d1.cpu().numpy(), d2.cpu().numpy(), fields, r1, r2, tol, (prec, variant))


@pytest.mark.parametrize("prec,tol,variant", _variants())
def test_sweep_extreme_sizes(prec, tol, variant):
    """The largest subpatch side (1024 points: 16 output tiles of 64 per line,
    operator tables of 1024 rows) and the shortest line (2 d = 10 points: one
    ragged block of a single chunk) in one grouped launch, every variant.  The
    operator row sums of |entries| reach 19.5 at n = 1024, which keeps the
    FP32 and split-BF16 bounds of test_sweep_parity.  FP64: on lines of 10-12
    points the d = 5 continuation dominates the operator and the library's
    and the oracle's operators differ by up to the 3e-12 (relative to max|f|)
    of the module's error model, so the bound is twice that."""
    if prec == "fp64":
        tol = 6e-12
    sizes = np.array([(1024, 12), (12, 1024), (10, 37), (37, 10), (10, 10), (257, 11)])
    fields = W.sweep_fields(sizes, W.rng(3, 7))
    flat = np.concatenate([f.ravel() for f in fields])
    sw = F.DerivSweep(sizes, 4, prec, d=5, C=27)
    sw.set_variant(variant)
    x = torch.tensor(flat, device="cuda")
    d1 = torch.zeros_like(x)
    d2 = torch.zeros_like(x)
    r1, r2 = _sweep_ref(fields)
    sw.run(x, d1, d2)
    torch.cuda.synchronize()
    _check_sweep(d1.cpu().numpy(), d2.cpu().numpy(), fields, r1, r2, tol, (prec, variant))


def _check_sweep(g1, g2, fields, r1, r2, tol, tag):
    off = 0
    for f, a, b in zip(fields, r1, r2):
        n = f.size
        for c in range(4):
            scale = np.abs(f[c]).max()
            e1 = np.abs(g1[off:off + n].reshape(f.shape)[c] - a[c]).max() / scale
            e2 = np.abs(g2[off:off + n].reshape(f.shape)[c] - b[c]).max() / scale
            assert e1 < tol and e2 < tol, (tag, f.shape, c, e1, e2)
        off += n


def _persistent_variants():
    from paper_2506_19370_amd import _lib as L
    return [(p, tol, v) for p, tol in (("fp64", 2e-12), ("fp32", 2e-6), ("bf16x3", 1e-4))
            for v in range(L.fcs_gemm_variant_count(L.PREC[p])) if "persist" in L.gemm_variant_name(p, v)]


@pytest.mark.parametrize("prec,tol,variant", _persistent_variants())
def test_sweep_persistent_queues(prec, tol, variant):
    """Persistent forms on a tile list several times the resident slots, so
    that every workgroup takes further tiles from its XCD queue's counter;
    three launches in a row (the counters must return to zero)."""
    sizes, fields = W.deriv_sweep(npatch=160, nmin=60, nmax=160, seed_salt=2)
    flat = np.concatenate([f.ravel() for f in fields])
    sw = F.DerivSweep(sizes, 4, prec, d=5, C=27)
    sw.set_variant(variant)
    x = torch.tensor(flat, device="cuda")
    d1 = torch.zeros_like(x)
    d2 = torch.zeros_like(x)
    r1, r2 = _sweep_ref(fields)
    for _ in range(3):
        d1.zero_()
        d2.zero_()
        sw.run(x, d1, d2)
        torch.cuda.synchronize()
        _check_sweep(d1.cpu().numpy(), d2.cpu().numpy(), fields, r1, r2, tol, (prec, variant))


def test_sweep_full_size_sampled():
    """The full derivative-sweep workload (2000 patches, 64..256) in the
    launch configuration the benchmark times: sampled patches against the
    oracle, FP64."""
    sizes, fields = W.deriv_sweep(npatch=2000)
    flat = np.concatenate([f.ravel() for f in fields])
    sw = F.DerivSweep(sizes, 4, "fp64", d=5, C=27)
    x = torch.tensor(flat, device="cuda")
    d1 = torch.zeros_like(x)
    d2 = torch.zeros_like(x)
    sw.run(x, d1, d2)
    torch.cuda.synchronize()
    offs = np.concatenate([[0], np.cumsum([f.size for f in fields])])
    for p in (0, 7, 999, 1999):
        f = fields[p]
        r1, r2 = _sweep_ref([f])
        a = d1[offs[p]:offs[p + 1]].cpu().numpy().reshape(f.shape)
        b = d2[offs[p]:offs[p + 1]].cpu().numpy().reshape(f.shape)
        scale = np.abs(f).max()
        assert np.abs(a - r1[0]).max() < 2e-12 * scale and np.abs(b - r2[0]).max() < 2e-12 * scale


def _vortex_pair(specs, d=5, av="off", n_f=5):
    prm = F.SolverParams(fc_d=d, fc_C=27, n_f=n_f, av=av)
    S = F.Solver(specs, prm)
    O = osolver.Solver(osolver.patches_from_specs(specs), osolver.Params(fc_d=d, fc_C=27, n_f=n_f, av=av),
                       exact=lambda x, y, t: exact.isentropic_vortex(x, y, t))
    w = [exact.isentropic_vortex(s.x, s.y, 0.0) for s in specs]
    for p, wp in enumerate(w):
        S.set_state(p, wp)
    O.set_prim(w)
    return S, O


def _rel(S, O, specs):
    err = 0.0
    scale = np.abs(O.U).max()
    for p in range(len(specs)):
        err = max(err, np.abs(S.cons(p) - O.view(O.U, p)).max())
    return err / scale


def test_vortex_single_patch_steps():
    specs = W.vortex_box(61)
    S, O = _vortex_pair(specs)
    for _ in range(3):
        t = S.advance(5, sync=True)
        O.step()
        assert abs(t - O.t) < 1e-14
    assert _rel(S, O, specs) < 1e-12


def test_vortex_partial_steps_match_full_steps():
    specs = W.vortex_box(41)
    S1, _ = _vortex_pair(specs)
    S2, _ = _vortex_pair(specs)
    S1.advance(10, sync=True)
    for n in (3, 4, 1, 2):
        S2.advance(n)
    S2.advance(0, sync=True)
    assert np.array_equal(S1.cons(0), S2.cons(0))


def test_vortex_multipatch_interpolation():
    """Four overlapping patches whose grids do not coincide: the fringe is
    filled by degree-5 interpolation every stage."""
    specs = W.vortex_multipatch(41)
    S, O = _vortex_pair(specs)
    for _ in range(2):
        S.advance(5, sync=True)
        O.step()
    assert _rel(S, O, specs) < 1e-12


def test_step_channel_no_viscosity():
    """Mach-3 step channel (C1 L-shaped and C2 corner subpatches, slip walls,
    inflow, outflow), FP64, d = 2."""
    specs = W.step_channel()
    prm = F.SolverParams(fc_d=2, fc_C=27, cfl=0.5)
    S = F.Solver(specs, prm)
    w = W.uniform_state(specs, W.STEP_INFLOW)
    for p in range(len(specs)):
        S.set_state(p, w[p])
    O = osolver.Solver(osolver.patches_from_specs(specs), osolver.Params(fc_d=2, fc_C=27, cfl=0.5))
    O.set_prim(w)
    for _ in range(3):
        S.advance(5, sync=True)
        O.step()
    assert _rel(S, O, specs) < 1e-12


def _jump_state(specs):
    """Step-channel state with a density and pressure jump at x = 0.3."""
    out = []
    for s in specs:
        w = np.broadcast_to(np.asarray(W.STEP_INFLOW, float)[:, None, None], (4,) + s.shape).copy()
        right = s.x > 0.3
        w[0] = np.where(right, 2.8, w[0])
        w[3] = np.where(right, 2.5, w[3])
        out.append(w)
    return out


@pytest.mark.parametrize("filt", [False, True])
def test_step_channel_modal_viscosity(filt):
    """Artificial viscosity with the modal indicator (FP64 on both sides):
    classes must agree exactly, then the viscosity and states."""
    specs = W.step_channel()
    prm = F.SolverParams(fc_d=2, fc_C=27, cfl=0.5, av="modal", filter=filt)
    S = F.Solver(specs, prm)
    w = _jump_state(specs)
    for p in range(len(specs)):
        S.set_state(p, w[p])
    O = osolver.Solver(osolver.patches_from_specs(specs), osolver.Params(fc_d=2, fc_C=27, cfl=0.5, av="modal",
                                                                         filter=filt))
    O.set_prim(w)
    for step in range(2):
        S.advance(5, sync=True)
        O.step()
        nz = 0
        for p in range(len(specs)):
            t0, t1 = S.field(p, "tau0"), S.field(p, "tau1")
            assert np.array_equal(t0, O.last_tau[p][0]) and np.array_equal(t1, O.last_tau[p][1]), (step, p)
            mu = S.field(p, "mu")
            mref = O.field(O.mu[0], p)
            assert np.abs(mu - mref).max() <= 1e-12 * max(1e-300, np.abs(O.mu[0]).max())
            nz += int((mref > 0).sum())
        assert nz > 100  # the viscosity is active around the jump
    assert _rel(S, O, specs) < 1e-11


def test_tiled_step_channel_modal_viscosity():
    """The step channel tiled by 73 subpatches of uneven sizes (seeded; the
    decomposition of the full-size tiled configuration at h = 1/200): T
    junctions, a C1 and a C2 corner patch.  Modal viscosity and filter, FP64
    on both sides: classes equal, viscosity and state to FP64 rounding."""
    specs = W.step_channel_tiled(200, 36, 72, 16)
    prm = F.SolverParams(fc_d=2, fc_C=27, cfl=0.5, av="modal", filter=True)
    S = F.Solver(specs, prm)
    w = _jump_state(specs)
    for p in range(len(specs)):
        S.set_state(p, w[p])
    O = osolver.Solver(osolver.patches_from_specs(specs), osolver.Params(fc_d=2, fc_C=27, cfl=0.5, av="modal",
                                                                         filter=True))
    O.set_prim(w)
    for step in range(2):
        S.advance(5, sync=True)
        O.step()
        for p in range(len(specs)):
            assert np.array_equal(S.field(p, "tau0"), O.last_tau[p][0]), (step, p)
            assert np.array_equal(S.field(p, "tau1"), O.last_tau[p][1]), (step, p)
            mref = O.field(O.mu[0], p)
            assert np.abs(S.field(p, "mu") - mref).max() <= 1e-12 * max(1e-300, np.abs(O.mu[0]).max())
    assert _rel(S, O, specs) < 1e-11


def test_tiled_step_channel_full_size():
    """The full-size tiled channel (235 subpatches, 1.17e7 points, sides
    150-300): graph replay equals eager launches bit for bit, the state stays
    finite and physical, and one split-BF16 step differs from the FP64 step
    from the same state by less than the split-BF16 contraction bound (1e-4
    of max|U|).  Error model as for the frozen-class mixed test: the bound
    reaches the state as dt/h (about 0.12 at CFL 0.5) x 2 directions x 1 step
    x max|F| / max|U| (about 1.5), i.e. about 0.4 x the bound; the modal
    classes of the step are those of the common initial state."""
    specs = W.step_channel_tiled()
    assert len(specs) == 235 and sum(s.npoints() for s in specs) == 11666791
    w = _jump_state(specs)
    res = {}
    for name, prec, graph in (("graph", "fp64", True), ("eager", "fp64", False), ("bf16x3", "bf16x3", True)):
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            S = F.Solver(specs, F.SolverParams(fc_d=2, fc_C=27, cfl=0.5, av="modal", filter=True, use_graph=graph,
                                               precision=prec), stream=stream)
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


def _sector():
    spec = W.annular_sector(48, 40)[0]
    spec.sides = {k: W.OUTFLOW for k in "WESN"}
    return [spec]


def test_curvilinear_freestream_preserved():
    specs = _sector()
    w = np.broadcast_to(np.array([1.4, 0.5, 0.2, 1.0])[:, None, None], (4,) + specs[0].shape).copy()
    S = F.Solver(specs, F.SolverParams(fc_d=5, fc_C=27, dt_fixed=1e-3))
    S.set_state(0, w)
    e0 = S.cons(0)
    S.advance(10, sync=True)
    assert np.abs(S.cons(0) - e0).max() < 1e-9 * np.abs(e0).max()


def test_curvilinear_viscous_parity_frozen_classes():
    """Non-affine metrics (16 line products per stage, Laplacian of the index
    coordinates, cross derivatives) with a non-zero viscosity: classes are
    prescribed (frozen) identically on both sides.  The mesh size in the
    viscosity (and in the step size) comes from the FC-derived metric, where
    the two sides' d = 5 operators differ by up to 3e-12: viscosity and state
    agree to 1e-11 relative."""
    specs = _sector()
    s = specs[0]
    r = np.hypot(s.x, s.y)
    w = np.stack([1.4 + 0.2 * np.exp(-40 * (r - 1.5) ** 2), 0.5 + 0 * r, 0.2 + 0 * r, 1.0 + 0.1 * np.exp(-40 * (r - 1.5) ** 2)])
    tau = np.zeros((2,) + s.shape, dtype=np.uint8)
    tau[0, 15:25, 10:30] = 2
    tau[1, 18:22, 20:40] = 1
    S = F.Solver(specs, F.SolverParams(fc_d=5, fc_C=27, av="frozen", dt_fixed=2e-4))
    S.set_state(0, w)
    S.set_tau(0, tau)
    O = osolver.Solver(osolver.patches_from_specs(specs), osolver.Params(fc_d=5, fc_C=27, av="modal", dt_fixed=2e-4))
    O.set_prim([w])
    O.tau_override = [tau.astype(np.int64)]
    for _ in range(2):
        S.advance(5, sync=True)
        O.step()
    assert np.abs(O.mu[0]).max() > 0
    assert np.abs(S.field(0, "mu") - O.field(O.mu[0], 0)).max() < 1e-11 * np.abs(O.mu[0]).max()
    assert _rel(S, O, specs) < 1e-11


@pytest.mark.parametrize("prec,tol", [("fp32", 2e-6), ("bf16x3", 1e-4), ("bf16x6", 2e-6)])
def test_step_channel_mixed_precision_frozen_classes(prec, tol):
    """Mixed forms (FP32 or split-BF16 stage contractions, FP32 stage
    derivatives, FP64 state) against the FP64 oracle on the step channel with
    a viscous band of prescribed classes in every subpatch.  Error model: the
    contraction's bound (the sweep tolerance, relative to max|f|, index
    units) reaches the state as dt/h (0.025 here) x 2 directions x 2 steps x
    max|F| / max|U| (about 1.5), i.e. about 0.15 x the bound; the tolerance
    is the bound itself."""
    specs = W.step_channel()
    w = W.uniform_state(specs, W.STEP_INFLOW)
    for p, s in enumerate(specs):
        bump = np.exp(-((s.x - 1.0) ** 2 + (s.y - 0.6) ** 2) / 0.02)
        w[p][0] = w[p][0] * (1.0 + 0.1 * bump)
        w[p][3] = w[p][3] * (1.0 + 0.1 * bump)
    taus = []
    for s in specs:
        t = np.zeros((2,) + s.shape, dtype=np.uint8)
        t[0][(s.x > 0.9) & (s.x < 1.1)] = 2
        t[1][(s.y > 0.5) & (s.y < 0.7)] = 1
        taus.append(t)
    S = F.Solver(specs, F.SolverParams(fc_d=2, fc_C=27, av="frozen", dt_fixed=1e-4, precision=prec))
    for p in range(len(specs)):
        S.set_state(p, w[p])
        S.set_tau(p, taus[p])
    O = osolver.Solver(osolver.patches_from_specs(specs), osolver.Params(fc_d=2, fc_C=27, av="modal", dt_fixed=1e-4))
    O.set_prim(w)
    O.tau_override = [t.astype(np.int64) for t in taus]
    for _ in range(2):
        S.advance(5, sync=True)
        O.step()
    assert np.abs(O.mu[0]).max() > 0  # mu (global array) is non-zero in the band
    err = _rel(S, O, specs)
    assert err < tol, (prec, err)


def test_graph_replay_equals_eager():
    specs = W.step_channel()
    w = W.uniform_state(specs, W.STEP_INFLOW)
    out = []
    for graph in (False, True):
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            S = F.Solver(specs, F.SolverParams(fc_d=2, fc_C=27, av="modal", filter=True, use_graph=graph),
                         stream=stream)
            for p in range(len(specs)):
                S.set_state(p, w[p])
            for _ in range(3):  # replays with host synchronizations in between
                S.advance(10, sync=True)
            out.append([S.cons(p) for p in range(len(specs))])
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_viscous_line_skip_is_exact():
    """Rows and columns of lattice subpatches along which mu vanishes skip
    their viscous derivatives; those only meet exact zeros (mu and its
    derivative along the line), so the state must equal, bit for bit, that
    of a run that evaluates every line.  The jump moves about 15 points in
    40 steps, so lines switch between skipped and computed (stale
    derivatives of earlier steps stay in the skipped slots)."""
    specs = W.step_channel()
    w = _jump_state(specs)
    out, prof = [], []
    for all_lines in (False, True):
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            S = F.Solver(specs, F.SolverParams(fc_d=2, fc_C=27, cfl=0.5, av="modal", filter=True, use_graph=True,
                                               visc_all_lines=all_lines), stream=stream)
            for p in range(len(specs)):
                S.set_state(p, w[p])
            for _ in range(4):
                S.advance(50, sync=True)
            out.append([S.cons(p) for p in range(len(specs))])
            S.profile(True)
            S.advance(10, sync=True)
            prof.append(S.profile_read())
            S.profile(False)
            # timing the last step's contraction alone leaves the solution as it is
            before = [S.cons(p) for p in range(len(specs))]
            alone = S.profile_stage(5)
            assert alone["avg_ms"] > 0 and 0 < alone["flops"] <= prof[0 if not all_lines else 1]["flops"] * 1.5
            for p in range(len(specs)):
                assert np.array_equal(before[p], S.cons(p)), p
            S.advance(5, sync=True)
            out.append([S.cons(p) for p in range(len(specs))])
    # states after 40 steps, and after one more step taken after the
    # contraction was timed alone
    for k in (0, 1):
        for p, (a, b) in enumerate(zip(out[k], out[k + 2])):
            assert np.array_equal(a, b), (k, p)
    # the profile counts only the lines a step needs
    assert prof[0]["launches"] == prof[1]["launches"] == 8
    assert 0.2 * prof[1]["flops"] < prof[0]["flops"] < 0.9 * prof[1]["flops"], (prof[0]["flops"], prof[1]["flops"])


def test_pinned_tile_shapes_and_retune():
    """Two staged FP64 tile shapes accumulate every output in the same order
    (MFMA steps of 4 columns, chunk after chunk), so pinning either gives the
    same state bit for bit; re-tuning in the middle of a run changes the tile
    shape only; unknown names are refused."""
    from paper_2506_19370_amd import _lib as L
    specs = W.step_channel()
    w = _jump_state(specs)
    out = []
    for name in ("k_gemm_fp<double, 16, 1, 4, 1>", "k_gemm_fp<double, 8, 1, 4, 2>", None):
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            S = F.Solver(specs, F.SolverParams(fc_d=2, fc_C=27, cfl=0.5, av="modal", filter=True, use_graph=True,
                                               autotune=name is None), stream=stream)
            for p in range(len(specs)):
                S.set_state(p, w[p])
            if name is None:
                S.advance(10, sync=True)
                S.retune()
                S.advance(20, sync=True)
            else:
                S.set_stage_variant(name)
                assert L.gemm_variant_name("fp64", S.stats()["stage_variant"]) == name
                S.advance(30, sync=True)
                assert L.gemm_variant_name("fp64", S.stats()["stage_variant"]) == name
            out.append([S.cons(p) for p in range(len(specs))])
            if name is None:
                with pytest.raises(ValueError):
                    S.set_stage_variant("k_gemm_fp<double, 3, 3, 3, 3>")
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
    # the tuned run may pick a shape with another reduction order: FP64 rounding
    scale = max(np.abs(a).max() for a in out[0])
    assert max(np.abs(a - b).max() for a, b in zip(out[0], out[2])) <= 1e-12 * scale


def test_nonfinite_is_reported():
    specs = W.vortex_box(41)
    S = F.Solver(specs, F.SolverParams(fc_d=5, fc_C=27))
    w = exact.isentropic_vortex(specs[0].x, specs[0].y, 0.0)
    w[0, 20, 20] = -1.0
    S.set_state(0, w)
    with pytest.raises(F.FcsError) as ei:
        S.advance(5, sync=True)
    assert ei.value.status == 4


def test_overlap_violation_rejected():
    specs = W.step_channel()
    # drop the L-shaped corner patch: its neighbours' fringes lose their donors
    bad = [s for s in specs if s.kind != "C1"]
    with pytest.raises(F.FcsError) as ei:
        F.Solver(bad, F.SolverParams(fc_d=2, fc_C=27))
    assert ei.value.status == 2
