"""GPU parity of the no-slip adiabatic walls (the paper's obstacle
conditions; FC-Neumann reading for theta) against the oracle (MI355X,
gfx950): the Mach-3 shock tube with no-slip walls at y = 0 and y = 0.25, and
the step channel with every wall no-slip (step face, step top, the C1
corner patch's notch walls, channel floor and ceiling)."""
import copy

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_19370_amd as F  # noqa: E402
import workloads as W  # noqa: E402
from oracle import solver as osolver  # noqa: E402


def _noslip(specs):
    out = []
    for s in specs:
        t = copy.copy(s)
        t.sides = {k: (W.NOSLIP if v == W.SLIP else v) for k, v in s.sides.items()}
        if s.mask is not None and s.notch == W.SLIP:
            t.notch = W.NOSLIP
        out.append(t)
    return out


def _run_pair(specs, w, steps, tol):
    S = F.Solver(specs, F.SolverParams(fc_d=2, fc_C=27, cfl=0.5, av="modal", filter=True, use_graph=True))
    for p in range(len(specs)):
        S.set_state(p, w[p])
    O = osolver.Solver(osolver.patches_from_specs(specs),
                       osolver.Params(fc_d=2, fc_C=27, cfl=0.5, av="modal", filter=True))
    O.set_prim(w)
    for step in range(steps):
        S.advance(5, sync=True)
        O.step()
        for p in range(len(specs)):
            assert np.array_equal(S.field(p, "tau0"), O.last_tau[p][0]), (step, p)
        scale = np.abs(O.U).max()
        err = max(np.abs(S.cons(p) - O.view(O.U, p)).max() for p in range(len(specs))) / scale
        assert err < tol, (step, err)
    return S, O


def test_noslip_shock_tube_matches_oracle():
    specs = _noslip(W.mach_shock_tube(3.0, 200))
    assert all(s.sides["S"] == W.NOSLIP and s.sides["N"] == W.NOSLIP for s in specs)
    w = W.mach_shock_state(specs, 3.0, 0.2)
    S, O = _run_pair(specs, w, 3, 1e-12)
    # the walls hold no momentum (but the corners on the inflow side, which
    # keep the inflow data); the interior next to them does
    for p, s in enumerate(specs):
        mx = S.field(p, "mx")
        lo = 1 if s.sides["W"] == W.INFLOW else 0
        hi = mx.shape[1] - (1 if s.sides["E"] == W.INFLOW else 0)
        assert np.all(mx[0, lo:hi] == 0.0) and np.all(mx[-1, lo:hi] == 0.0)
    assert np.abs(S.field(0, "mx")[1]).max() > 0.1


def test_noslip_step_channel_matches_oracle():
    specs = _noslip(W.step_channel())
    w = W.uniform_state(specs, W.STEP_INFLOW)
    _run_pair(specs, w, 2, 1e-11)
