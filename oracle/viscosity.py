"""Localized artificial viscosity (Alg. 3, Sec. 4 and Sec. 5 item 2).

Per subpatch and per step: the proxy Phi (Mach number) at every point, the
smoothness class tau of Phi along the two grid lines through every point
outside the fringe, the maximum wave speed bound S~, and the preliminary
viscosity mu^ (zero on the fringe).  The preliminary values are then
smoothed inside each subpatch and blended across subpatches (the operator
Lambda of Sec. 4).  Part I's formulas I-(37), I-(38), I-(42) and I-(44) are
not reproduced in the paper; the readings here are:

* windows of 16 points [i-8, i+7] along the line, shifted to stay inside it;
* S~ = max of |u| + a over the point's two windows;
* mu^ = c_mu * h_x * S~ * max(alpha(tau_1), alpha(tau_2)), alpha = (0, 1/2, 1),
  h_x the distance to the nearest grid neighbour;
* smoothing: mu~(i, j) = max over |k-i|, |l-j| <= n_v of
  mu^(k, l) w(|k-i|/n_v) w(|l-j|/n_v), w(t) = exp(1 - 1/(1 - t^2));
* blend: mu = sum_s W_s mu~_s / sum_s W_s with the windows of overlap.py.

parity unpinned: the viscosity constants and windows of Part I.
"""
from __future__ import annotations

import numpy as np

from . import euler, sdnn

ALPHA = np.array([0.0, 0.5, 1.0])
W = sdnn.WINDOW


def window_starts(run_start: int, run_len: int, pos: np.ndarray) -> np.ndarray:
    return np.clip(pos - W // 2, run_start, run_start + run_len - W)


def line_windows(field2d: np.ndarray, grid, direction: int):
    """All 16-point windows of ``field2d`` along q^1 (0) or q^2 (1).
    Returns (points (j, i) arrays, windows (m, 16))."""
    js, is_, wins = [], [], []
    runs = grid.row_runs if direction == 0 else grid.col_runs
    for line, (s, n) in enumerate(runs):
        if n < W:
            continue
        pos = np.arange(s, s + n)
        st = window_starts(s, n, pos)
        idx = st[:, None] + np.arange(W)[None, :]
        if direction == 0:
            wins.append(field2d[line][idx])
            js.append(np.full(n, line)); is_.append(pos)
        else:
            wins.append(field2d[:, line][idx])
            js.append(pos); is_.append(np.full(n, line))
    if not wins:
        return (np.zeros(0, int), np.zeros(0, int)), np.zeros((0, W))
    return (np.concatenate(js), np.concatenate(is_)), np.concatenate(wins)


def classify_patch(e: np.ndarray, grid, classifier, gamma=euler.GAMMA):
    """tau along q^1 and q^2 (two int arrays (n2, n1)) for one subpatch;
    ``classifier(windows) -> tau``."""
    m = grid.p.mask
    phi = np.where(m, euler.mach(np.where(m, e, 1.0), gamma), 0.0)
    taus = []
    for direction in (0, 1):
        tau = np.zeros(m.shape, dtype=np.int64)
        (jj, ii), wins = line_windows(phi, grid, direction)
        if len(jj):
            tau[jj, ii] = classifier(wins)
        tau[~m] = 0
        taus.append(tau)
    return taus


def wave_speed_bound(e: np.ndarray, grid, gamma=euler.GAMMA) -> np.ndarray:
    """S~: max of |u| + a over the two 16-point windows of each point."""
    m = grid.p.mask
    ee = np.where(m, e, 1.0)
    s = np.sqrt(ee[1] ** 2 + ee[2] ** 2) / ee[0] + euler.sound_speed(ee, gamma)
    s = np.where(m, s, 0.0)
    out = np.zeros(m.shape)
    for direction in (0, 1):
        (jj, ii), wins = line_windows(s, grid, direction)
        if len(jj):
            out[jj, ii] = np.maximum(out[jj, ii], wins.max(axis=1))
    return np.where(m, out, 0.0)


def preliminary(e, grid, taus, c_mu, gamma=euler.GAMMA):
    """mu^ outside the fringe (Alg. 3)."""
    s = wave_speed_bound(e, grid, gamma)
    a = np.maximum(ALPHA[taus[0]], ALPHA[taus[1]])
    mu = c_mu * grid.hx * s * a
    keep = grid.p.mask & ~grid.fringe & ~grid.xfringe
    return np.where(keep, mu, 0.0)


def window_weight(t: np.ndarray) -> np.ndarray:
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros_like(t)
    inside = t < 1.0
    out[inside] = np.exp(1.0 - 1.0 / (1.0 - t[inside] ** 2))
    return out


def smooth(mu_hat: np.ndarray, n_v: int) -> np.ndarray:
    """mu~(i, j) = max_{k, l} mu^(k, l) w(|k-i|/n_v) w(|l-j|/n_v)."""
    n2, n1 = mu_hat.shape
    w = window_weight(np.arange(n_v + 1) / n_v)
    out = np.zeros_like(mu_hat)
    for j in range(n2):
        for i in range(n1):
            best = 0.0
            for l in range(max(0, j - n_v), min(n2, j + n_v + 1)):
                wl = w[abs(l - j)]
                for k in range(max(0, i - n_v), min(n1, i + n_v + 1)):
                    v = (mu_hat[l, k] * w[abs(k - i)]) * wl
                    if v > best:
                        best = v
            out[j, i] = best
    return out


def smooth_fast(mu_hat: np.ndarray, n_v: int) -> np.ndarray:
    """Same values as :func:`smooth`, computed as a max along q^1 followed by
    a max along q^2 (valid because the weights are non-negative and the
    products are formed in the same order)."""
    n2, n1 = mu_hat.shape
    w = window_weight(np.arange(n_v + 1) / n_v)
    tmp = np.zeros_like(mu_hat)
    for off in range(-n_v, n_v + 1):
        lo, hi = max(0, -off), min(n1, n1 - off)
        tmp[:, lo:hi] = np.maximum(tmp[:, lo:hi], mu_hat[:, lo + off:hi + off] * w[abs(off)])
    out = np.zeros_like(mu_hat)
    for off in range(-n_v, n_v + 1):
        lo, hi = max(0, -off), min(n2, n2 - off)
        out[lo:hi, :] = np.maximum(out[lo:hi, :], tmp[lo + off:hi + off, :] * w[abs(off)])
    return out
