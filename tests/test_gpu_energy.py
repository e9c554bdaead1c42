"""Energy conservation (Sec. 7.2.2): 2-D Sod problem in a closed box,
reflecting walls, one patch split along x into four overlapping subpatches,
SDNN viscosity and the spectral filter.  First the workload's stages against
the oracle, then the long run against the band the paper reports."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_19370_amd as F  # noqa: E402
import workloads as W  # noqa: E402
from oracle import solver as osolver  # noqa: E402

HERE = os.path.dirname(__file__)
GOLD = json.load(open(os.path.join(HERE, "golden", "sod_reflect_energy.json")))
HIDX = 200


def _mean_energy(S, specs):
    """Trapezoid mean of E over the box, each lattice column taken from the
    subpatch whose core holds it."""
    cols = []
    for p, (c0, c1) in enumerate(W.sod_reflect_cores(HIDX)):
        X0 = int(round(specs[p].x[0, 0] * HIDX))
        cols.append(S.field(p, "E")[:, c0 - X0:c1 - X0])
    E = np.concatenate(cols, axis=1)
    ny, nx = E.shape
    wx = np.ones(nx); wx[[0, -1]] = 0.5
    wy = np.ones(ny); wy[[0, -1]] = 0.5
    return (wy[:, None] * wx[None, :] * E).sum() / ((nx - 1) * (ny - 1))


def test_sod_reflect_stages_match_oracle():
    """Reflecting walls on all four sides (corner points of two slip sides),
    shocks crossing the overlaps, modal viscosity and filter: classes exact,
    states to FP64 rounding."""
    specs = W.sod_reflect(HIDX)
    w = W.sod_state(specs)
    S = F.Solver(specs, F.SolverParams(fc_d=2, fc_C=27, cfl=0.5, av="modal", filter=True))
    for p in range(len(specs)):
        S.set_state(p, w[p])
    O = osolver.Solver(osolver.patches_from_specs(specs),
                       osolver.Params(fc_d=2, fc_C=27, cfl=0.5, av="modal", filter=True))
    O.set_prim(w)
    for _ in range(3):
        S.advance(5, sync=True)
        O.step()
    for p in range(len(specs)):
        assert np.array_equal(S.field(p, "tau0"), O.last_tau[p][0])
        assert np.array_equal(S.field(p, "tau1"), O.last_tau[p][1])
    scale = max(np.abs(O.U).max(), 1.0)
    err = max(np.abs(S.cons(p) - O.view(O.U, p)).max() for p in range(len(specs)))
    assert err < 1e-12 * scale


def test_sod_reflect_energy_long_run():
    """To T = 100 (about 140000 steps, 120 wall reflections): the mean energy
    stays in the paper's band 1.37 +- 0.01 around the exact 1.375, and the
    state stays admissible (the library reports non-finite or non-positive
    states as an error)."""
    specs = W.sod_reflect(HIDX)
    w = W.sod_state(specs)
    blob = np.load(os.path.join(HERE, "golden", "sdnn_oracle_weights.npz"))["params"]
    S = F.Solver(specs, F.SolverParams(fc_d=2, fc_C=27, cfl=0.5, av="sdnn", sdnn_weights=blob, filter=True))
    for p in range(len(specs)):
        S.set_state(p, w[p])
    lo = GOLD["reported_mean_energy"] - GOLD["reported_band"]
    hi = GOLD["reported_mean_energy"] + GOLD["reported_band"]
    t, samples = 0.0, []
    while t < GOLD["final_time"]:
        t = S.advance(5 * 5000, sync=True)
        e = _mean_energy(S, specs)
        samples.append((t, e))
        print("t %.2f mean energy %.6f" % (t, e), flush=True)
        assert lo <= e <= hi, (t, e)
    assert abs(samples[-1][1] - GOLD["exact_mean_energy"]) < GOLD["reported_band"]
