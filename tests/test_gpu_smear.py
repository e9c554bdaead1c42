"""GPU parity of the localized initial-data smearing (Alg. 4 at t = 0,
reading of Part I's smearing): the first step from t = 0 smears the data
near the discontinuities its classes flag, on the library and in the oracle
alike (MI355X, gfx950)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_19370_amd as F  # noqa: E402
import workloads as W  # noqa: E402
from oracle import solver as osolver  # noqa: E402


def _rel(S, O, n):
    scale = np.abs(O.U).max()
    return max(np.abs(S.cons(p) - O.view(O.U, p)).max() for p in range(n)) / scale


def _pair(specs, w, **kw):
    S = F.Solver(specs, F.SolverParams(fc_d=2, fc_C=27, cfl=0.5, av="modal", filter=True, smear=True, **kw))
    for p in range(len(specs)):
        S.set_state(p, w[p])
    O = osolver.Solver(osolver.patches_from_specs(specs),
                       osolver.Params(fc_d=2, fc_C=27, cfl=0.5, av="modal", filter=True, smear=True))
    O.set_prim(w)
    return S, O


@pytest.mark.parametrize("graph", [True, False])
def test_smeared_shock_tube_matches_oracle(graph):
    """Mach-3 shock tube (four subpatches): the smeared first step and a
    filtered second step, classes equal and states to FP64 rounding; the
    smearing changed the data (against a run without it)."""
    specs = W.mach_shock_tube(3.0, 200)
    w = W.mach_shock_state(specs, 3.0, 0.2)
    S, O = _pair(specs, w, use_graph=graph)
    for step in range(2):
        S.advance(5, sync=True)
        O.step()
        for p in range(len(specs)):
            assert np.array_equal(S.field(p, "tau0"), O.last_tau[p][0]), (step, p)
        assert _rel(S, O, len(specs)) < 1e-12, step
    plain = F.Solver(specs, F.SolverParams(fc_d=2, fc_C=27, cfl=0.5, av="modal", filter=True))
    for p in range(len(specs)):
        plain.set_state(p, w[p])
    plain.advance(10, sync=True)
    assert max(np.abs(plain.cons(p) - S.cons(p)).max() for p in range(len(specs))) > 1e-3


def test_smeared_wedge_start_matches_oracle():
    """The small wedge decomposition (72 subpatches, skewed and corner
    subpatches): the smeared first step, to 1e-11."""
    specs = W.wedge_tunnel(600, 48, 96)
    w = W.wedge_state(specs)
    S, O = _pair(specs, w)
    S.advance(5, sync=True)
    O.step()
    for p in range(len(specs)):
        assert np.array_equal(S.field(p, "tau0"), O.last_tau[p][0]), p
        assert np.array_equal(S.field(p, "tau1"), O.last_tau[p][1]), p
    assert _rel(S, O, len(specs)) < 1e-11
