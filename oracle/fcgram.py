"""FC-Gram Fourier continuation and the spectral operators built on it.

Follows Sec. 2 (Preliminaries) of the paper: from N equispaced values of a
non-periodic function on [0, 1] (h = 1/(N-1)), FC-Gram builds a Fourier
expansion that is periodic on a longer interval and matches the data on
[0, 1]; derivatives and filtering are then done in Fourier space.  The
construction details live in the paper's Part I (Sec. I-2.2) and the FC-Gram
literature, which are not reproduced in the paper; this module takes the
following reading:

* ``d`` matching points at each end of a line; the data there are replaced
  by their interpolating polynomial, written in the Gram basis ``Q`` (the
  orthonormal basis of polynomials of degree < d for the discrete inner
  product on the d matching points).
* Each Gram polynomial is continued by a trigonometric polynomial with
  ``K = 25`` modes and period ``76`` (in units of h) that matches the
  polynomial on the matching interval and vanishes on a ``Z = 12`` point
  zero interval that starts right after the ``C`` continuation points; both
  intervals are oversampled 20 times and the fit is a least-squares problem
  solved by Householder QR in 256-bit arithmetic.  Sampling the fitted
  trigonometric polynomials at the C continuation points gives ``A`` (C x d).
* A line f of n points is extended to n + C points by adding the continued
  right-end data and the mirrored continuation of the left-end data; the
  extension is periodic with period (n + C) h.
* Derivatives multiply the DFT coefficients by (2 pi i m / M) or its square
  (M = n + C, index units: the derivative with respect to q / h); the
  Nyquist mode of an even M is zeroed.  The filter multiplies them by
  exp(-alpha (2|m|/M)^(2p)).

All results are FP64 NumPy arrays; the construction itself is done in mpmath.
"""
from __future__ import annotations

import functools

import mpmath as mp
import numpy as np

# Construction constants of the continuation (reading of Sec. I-2.2).
ZERO_POINTS = 12
OVERSAMPLE = 20
N_MODES = 25
PERIOD = 76
PRECISION_BITS = 256

# Filter I-(32) reading: sigma(eta) = exp(-alpha eta^(2p)).
FILTER_ALPHA = 16.0 * np.log(10.0)
FILTER_ORDER = 36
# The stronger filter of the initial-data smearing (Alg. 4 at t = 0; Part
# I's strength is not available): the same exponential with order 8.
SMEAR_ORDER = 8


def gram_basis(d: int, prec: int = PRECISION_BITS):
    """Orthonormal Gram polynomials on the matching points t = 0..d-1.

    Returns ``(Q, coeffs)``: ``Q`` (d x d, mpmath) holds the values of the
    Gram polynomials at the matching points (column k = degree k), and
    ``coeffs`` (d x d, mpmath) their monomial coefficients
    (q_k(t) = sum_j coeffs[j, k] t^j).  Built by Householder QR of the
    Vandermonde matrix, so Q^T Q = I (Sec. 2, FC-Gram of degree d).
    """
    with mp.workprec(prec):
        V = mp.matrix(d, d)
        for i in range(d):
            for j in range(d):
                V[i, j] = mp.mpf(i) ** j
        Q, R = mp.qr(V)
        # Fix signs so that the leading coefficient of every q_k is positive.
        for k in range(d):
            if R[k, k] < 0:
                for i in range(d):
                    Q[i, k] = -Q[i, k]
                for j in range(d):
                    R[k, j] = -R[k, j]
        coeffs = mp.inverse(R)  # V = Q R  =>  Q = V R^{-1}
        return Q, coeffs


def _trig_row(t, K, P):
    row = [mp.mpf(1)]
    for k in range(1, K + 1):
        w = 2 * mp.pi * k * t / P
        row.append(mp.cos(w))
        row.append(mp.sin(w))
    return row


@functools.lru_cache(maxsize=None)
def continuation_data(d: int, C: int):
    """Continuation of the Gram polynomials (Sec. 2; reading of Sec. I-2.2).

    Returns a dict with FP64 arrays:
      ``Q``        d x d Gram basis values at the matching points,
      ``A``        C x d continuation of each Gram polynomial at t = d..d+C-1,
      ``B``        C x d = A Q^T, continuation of raw matching values,
      ``fit_res``  per-polynomial max fit residual on the matching set,
      ``zero_res`` per-polynomial max residual on the zero set.
    Local coordinate t: matching points t = 0..d-1 (t = d-1 is the line's
    last point), continuation points t = d..d+C-1, zero points
    t = d+C..d+C+Z-1.
    """
    K, P, Z, nos = N_MODES, PERIOD, ZERO_POINTS, OVERSAMPLE
    with mp.workprec(PRECISION_BITS):
        Qm, coeffs = gram_basis(d)
        t_match = [mp.mpf(i) / nos for i in range((d - 1) * nos + 1)]
        t_zero = [mp.mpf(d + C) + mp.mpf(i) / nos for i in range((Z - 1) * nos + 1)]
        rows = [_trig_row(t, K, mp.mpf(P)) for t in t_match + t_zero]
        M = mp.matrix(rows)
        Qf, Rf = mp.qr(M, mode="skinny")
        ncol = 2 * K + 1
        A_hp = mp.matrix(C, d)
        fit_res = np.zeros(d)
        zero_res = np.zeros(d)
        cont_rows = [_trig_row(mp.mpf(t), K, mp.mpf(P)) for t in range(d, d + C)]
        for k in range(d):
            rhs = mp.matrix(len(rows), 1)
            for r, t in enumerate(t_match):
                rhs[r] = mp.fsum(coeffs[j, k] * t ** j for j in range(d))
            # least squares through the skinny QR: R x = Q^T rhs
            x = mp.lu_solve(Rf, Qf.T * rhs)
            vals = M * x
            fit_res[k] = float(max(abs(vals[r] - rhs[r]) for r in range(len(t_match))))
            zero_res[k] = float(max(abs(vals[r]) for r in range(len(t_match), len(rows))))
            for c in range(C):
                A_hp[c, k] = mp.fsum(cont_rows[c][j] * x[j] for j in range(ncol))
        B_hp = A_hp * Qm.T
        A = np.array([[float(A_hp[c, k]) for k in range(d)] for c in range(C)])
        B = np.array([[float(B_hp[c, k]) for k in range(d)] for c in range(C)])
        Q = np.array([[float(Qm[i, k]) for k in range(d)] for i in range(d)])
    return {"Q": Q, "A": A, "B": B, "fit_res": fit_res, "zero_res": zero_res}


def extend(f: np.ndarray, d: int, C: int) -> np.ndarray:
    """Periodic FC extension of a line of n >= d values to n + C values.

    Right end: continuation of f[n-d:] ; left end: the mirrored continuation
    of f[:d] read backwards, placed so that it ends next to f[0] in the
    periodic sense (Sec. 2, the interval [0, beta] that contains [0, 1]).
    """
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[-1]
    B = continuation_data(d, C)["B"]
    right = f[..., n - d:] @ B.T                 # (..., C) at t = d..d+C-1
    left = f[..., :d][..., ::-1] @ B.T            # continuation of reversed data
    ext = np.concatenate([f, right + left[..., ::-1]], axis=-1)
    return ext


def _multiplier(M: int, kind: str) -> np.ndarray:
    m = np.fft.fftfreq(M) * M
    if kind == "d1":
        mult = 2j * np.pi * m / M
    elif kind == "d2":
        mult = -((2 * np.pi * m / M) ** 2) + 0j
    elif kind == "filter":
        eta = 2.0 * np.abs(m) / M
        mult = np.exp(-FILTER_ALPHA * eta ** FILTER_ORDER) + 0j
    elif kind == "smear":
        eta = 2.0 * np.abs(m) / M
        mult = np.exp(-FILTER_ALPHA * eta ** SMEAR_ORDER) + 0j
    else:
        raise ValueError(kind)
    if M % 2 == 0:
        mult[M // 2] = 0.0
    return mult


def fc_apply(f: np.ndarray, d: int, C: int, kind: str) -> np.ndarray:
    """FC derivative ('d1', 'd2', index units) or filter of lines along the
    last axis, via FFT of the periodic extension (Sec. 2; Alg. 5 lines on
    FC-based differentiation; Alg. 4 for the filter)."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[-1]
    ext = extend(f, d, C)
    M = n + C
    out = np.fft.ifft(np.fft.fft(ext, axis=-1) * _multiplier(M, kind), axis=-1).real
    return out[..., :n]


@functools.lru_cache(maxsize=None)
def dense_operator(n: int, d: int, C: int, kind: str) -> np.ndarray:
    """n x n matrix of the FC map ``kind`` for lines of n points, obtained by
    applying the FFT pipeline to the unit vectors (row t, column s)."""
    if n < 2 * d:
        raise ValueError("line shorter than twice the matching width")
    op = fc_apply(np.eye(n), d, C, kind)  # row s = image of e_s
    op = op.T.copy()
    op.setflags(write=False)
    return op


def dft_bruteforce(ext: np.ndarray, kind: str) -> np.ndarray:
    """Same spectral multiplier as :func:`fc_apply`, by an explicit O(M^2)
    DFT sum with no FFT (used only as an independent check)."""
    M = ext.shape[-1]
    j = np.arange(M)
    m = np.where(j <= M // 2, j, j - M).astype(np.float64)
    E = np.exp(-2j * np.pi * np.outer(j, j) / M)
    coef = E @ ext
    if kind == "d1":
        mult = 2j * np.pi * m / M
    elif kind == "d2":
        mult = -((2 * np.pi * m / M) ** 2) + 0j
    else:
        eta = 2.0 * np.abs(m) / M
        mult = np.exp(-FILTER_ALPHA * eta ** FILTER_ORDER) + 0j
    if M % 2 == 0:
        mult[M // 2] = 0.0
    return (np.conj(E) @ (coef * mult)).real / M
