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


@pytest.mark.parametrize("prec,tol", [("fp32", 2e-6), ("bf16x6", 2e-6), ("bf16x3", 1e-4)])
def test_smeared_wedge_start_mixed_forms(prec, tol):
    """The smeared first step in the mixed forms (FP32 or split-BF16 stage
    contractions, FP32 stage derivatives) against the FP64 form on the small
    wedge: the classes of the first step come from the same initial data,
    the smearing runs in FP64 in every form, so the states differ by the
    contraction's bound only (the sweep tolerance, relative to max|U|).  The
    smearing window must not pass through the derivative arrays that the
    stage kernel reads in FP32 (a window value read as an FP32 pair can be
    a NaN)."""
    specs = W.wedge_tunnel(600, 48, 96)
    w = W.wedge_state(specs)
    res = {}
    for form in ("fp64", prec):
        S = F.Solver(specs, F.SolverParams(fc_d=2, fc_C=27, cfl=0.5, av="modal", filter=True, smear=True,
                                           precision=form))
        for p in range(len(specs)):
            S.set_state(p, w[p])
        S.advance(5, sync=True)
        res[form] = [S.cons(p) for p in range(len(specs))]
        del S
    scale = max(np.abs(r).max() for r in res["fp64"])
    err = max(np.abs(a - b).max() for a, b in zip(res[prec], res["fp64"])) / scale
    assert np.isfinite(err) and err < tol, (prec, err)
