"""Checkpoint and resume through the C ABI (Alg. 1, solution output): the
conserved fields and the time read from one context at a step boundary and
given to a fresh context continue the run bit for bit; set_state and
set_time are refused inside a partial step."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_19370_amd as F  # noqa: E402
from paper_2506_19370_amd import _lib as L  # noqa: E402
import workloads as W  # noqa: E402

GOLD = os.path.join(os.path.dirname(__file__), "golden", "sdnn_oracle_weights.npz")


def _solver(specs, graph):
    prm = F.SolverParams(fc_d=2, fc_C=27, cfl=0.5, av="sdnn", filter=True, use_graph=graph,
                         sdnn_weights=np.load(GOLD)["params"])
    return F.Solver(specs, prm)


@pytest.mark.parametrize("graph", [False, True])
def test_checkpoint_resume_is_bitwise(graph):
    """Step channel with SDNN viscosity and the filter: 7 steps, checkpoint
    (get_field of rho, rho u, rho v, E and the time), resume in a fresh
    context (set_state of the conserved fields, set_time), then 4 more steps
    on both: every field and the time agree bit for bit."""
    specs = W.step_channel()
    A = _solver(specs, graph)
    w = W.uniform_state(specs, W.STEP_INFLOW)
    for p in range(len(specs)):
        A.set_state(p, w[p])
    t = A.advance(35, sync=True)
    ckpt = [A.cons(p) for p in range(len(specs))]
    assert t > 0 and A.stats()["steps"] == 7
    B = _solver(specs, graph)
    for p in range(len(specs)):
        B.set_state(p, ckpt[p], prim=False)
    B.set_time(t)
    ta = A.advance(20, sync=True)
    tb = B.advance(20, sync=True)
    assert ta == tb
    for p in range(len(specs)):
        for f in ("rho", "mx", "my", "E", "mu"):
            assert np.array_equal(A.field(p, f), B.field(p, f)), (p, f)


def test_set_state_and_time_refused_inside_a_step():
    specs = W.vortex_box(41)
    S = F.Solver(specs, F.SolverParams(fc_d=5, fc_C=27, vortex=(5.0, 5.0, 5.0, 1.0, 1.0)))
    from oracle import exact
    w0 = exact.isentropic_vortex(specs[0].x, specs[0].y, 0.0)
    S.set_state(0, w0)
    S.advance(3, sync=True)
    before = S.cons(0)
    with pytest.raises(L.FcsError) as e:
        S.set_state(0, w0)
    assert e.value.status == L.FCS_ESTATE
    with pytest.raises(L.FcsError) as e:
        S.set_time(0.0)
    assert e.value.status == L.FCS_ESTATE
    assert np.array_equal(S.cons(0), before)
    t = S.advance(2, sync=True)  # completes the step
    S.set_state(0, w0)
    S.set_time(0.0)
    t2 = S.advance(5, sync=True)
    assert abs(t2 - t) < 1e-15  # same first step again from the same data
