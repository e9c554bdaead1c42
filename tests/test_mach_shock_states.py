"""The Mach-M shock data (initial-conditions section, Mach-M shock equation)
against the Rankine-Hugoniot conditions: in the frame of a shock moving at
speed M into gas at rest, the fluxes of mass, momentum and energy are equal
on both sides; the gas ahead has sound speed 1.  The density behind is the
ratio of the equation times the density ahead (8.0 at M = 10)."""
import numpy as np
import pytest

import workloads as W

G = 1.4


def _fluxes(rho, u, p):
    E = p / (G - 1.0) + 0.5 * rho * u * u
    return np.array([rho * u, rho * u * u + p, u * (E + p)])


@pytest.mark.parametrize("M", [1.4, 3.0, 3.5, 10.0])
def test_states_satisfy_rankine_hugoniot(M):
    behind, ahead = W.mach_shock_states(M)
    assert abs(np.sqrt(G * ahead[3] / ahead[0]) - 1.0) < 1e-15
    # shock frame: subtract the shock speed M
    f1 = _fluxes(behind[0], behind[1] - M, behind[3])
    f0 = _fluxes(ahead[0], ahead[1] - M, ahead[3])
    assert np.abs(f1 - f0).max() < 1e-12 * np.abs(f0).max()
    # a compressive shock: density and pressure rise, the gas behind follows it
    assert behind[0] > ahead[0] and behind[3] > ahead[3] and 0 < behind[1] < M


def test_strong_shock_density():
    assert abs(W.mach_shock_states(10.0)[0][0] - 8.0) < 1e-12
    # the limit of a very strong shock: density ratio (gamma + 1) / (gamma - 1)
    assert abs(W.mach_shock_states(1e4)[0][0] / 1.4 - 6.0) < 1e-6
