"""Pins of the oracle's FC-Gram construction and FC operators (CPU only).

Each check is tied to something other than the oracle's own formulas: the
orthonormality of the Gram basis, exactness on polynomials of degree < d,
an explicit O(M^2) DFT sum, the convergence order of the method, and the
behaviour of the filter on constants and smooth data.
"""
import numpy as np
import pytest

from oracle import fcgram


@pytest.mark.parametrize("d", [2, 5])
def test_gram_basis_orthonormal_and_fit(d):
    r = fcgram.continuation_data(d, 27)
    Q = r["Q"]
    assert np.abs(Q.T @ Q - np.eye(d)).max() < 1e-14
    # each continued Gram polynomial matches on the oversampled matching set
    # and vanishes on the zero set
    assert r["fit_res"].max() < 1e-13
    assert r["zero_res"].max() < 1e-13


@pytest.mark.parametrize("d", [2, 5])
def test_polynomials_reproduced(d):
    """FC derivatives of polynomials of degree < d are exact up to the
    smoothness floor of the continuation (about 1e-12 with five matching
    points, 2e-10 with two: the shorter matching interval constrains the
    continuation less)."""
    floor = {2: 5e-10, 5: 5e-12}[d]
    for n in (40, 101, 160):
        t = np.arange(n, dtype=float)
        D = fcgram.dense_operator(n, d, 27, "d1")
        for k in range(d):
            f = (t / (n - 1)) ** k
            exact = k * (t / (n - 1)) ** max(k - 1, 0) / (n - 1) if k else np.zeros(n)
            assert np.abs(D @ f - exact).max() < floor, (n, k)


@pytest.mark.parametrize("kind", ["d1", "d2", "filter"])
def test_fft_matches_bruteforce_dft(kind):
    rng = np.random.default_rng(1)
    for n in (10, 13, 16):
        f = rng.standard_normal(n)
        ext = fcgram.extend(f, 5, 27)
        ref = fcgram.dft_bruteforce(ext, kind)[:n]
        # rounding of an M-term sum over the extension, whose continued part
        # can exceed the data by the size of the continuation matrix
        tol = 1e-14 * ext.size * np.abs(ext).max()
        assert np.abs(fcgram.fc_apply(f, 5, 27, kind) - ref).max() < tol
        D = fcgram.dense_operator(n, 5, 27, kind)
        assert np.abs(D @ f - ref).max() < tol


def _order(errs, ns):
    return np.log(errs[:-1] / errs[1:]) / np.log(np.array(ns[1:]) / np.array(ns[:-1]))


def test_convergence_order_d5():
    """First derivative of a smooth non-periodic function converges at order
    >= d - 1 = 4 until the error floor."""
    ns = [32, 64, 128, 256]
    errs = []
    for n in ns:
        x = np.linspace(0, 1, n)
        f = np.exp(np.sin(3 * x))
        fp = 3 * np.cos(3 * x) * f
        errs.append(np.abs(fcgram.fc_apply(f, 5, 27, "d1") * (n - 1) - fp).max())
    errs = np.array(errs)
    assert (_order(errs, ns) > 3.8).all(), errs
    assert errs[-1] < 1e-6


def test_convergence_second_derivative_d5():
    ns = [64, 128, 256]
    errs = []
    for n in ns:
        x = np.linspace(0, 1, n)
        f = np.exp(np.sin(3 * x))
        fpp = (9 * np.cos(3 * x) ** 2 - 9 * np.sin(3 * x)) * f
        errs.append(np.abs(fcgram.fc_apply(f, 5, 27, "d2") * (n - 1) ** 2 - fpp).max())
    errs = np.array(errs)
    assert (_order(errs, ns) > 2.5).all(), errs


def test_d2_first_order_near_boundary():
    """With two matching points (degree-1 polynomials) the derivative is
    first-order accurate: halving h halves the error."""
    ns = [64, 128, 256]
    errs = []
    for n in ns:
        x = np.linspace(0, 1, n)
        f = np.exp(np.sin(3 * x))
        errs.append(np.abs(fcgram.fc_apply(f, 2, 27, "d1") * (n - 1) - 3 * np.cos(3 * x) * f).max())
    o = _order(np.array(errs), ns)
    assert (o > 0.9).all() and (o < 1.3).all()


def test_filter_keeps_smooth_data_and_constants():
    n = 101
    x = np.linspace(0, 1, n)
    c = np.full(n, 2.5)
    assert np.abs(fcgram.fc_apply(c, 5, 27, "filter") - c).max() < 5e-11
    f = np.exp(np.sin(3 * x))
    assert np.abs(fcgram.fc_apply(f, 5, 27, "filter") - f).max() < 1e-8
    # a jump is damped: the filtered line has a smaller total variation
    g = (x > 0.5).astype(float)
    fg = fcgram.fc_apply(g, 2, 27, "filter")
    assert np.abs(np.diff(fg)).max() < 1.0


def test_dense_operator_shape_and_zero_row_sum():
    for n in (61, 105, 256):
        D = fcgram.dense_operator(n, 2, 27, "d1")
        assert D.shape == (n, n)
        assert np.abs(D.sum(axis=1)).max() < 5e-10  # derivative of a constant
        D2 = fcgram.dense_operator(n, 2, 27, "d2")
        assert np.abs(D2.sum(axis=1)).max() < 5e-9
