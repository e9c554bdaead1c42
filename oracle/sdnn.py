"""Shock-detecting neural network (SDNN) and its modal-decay fallback.

The paper obtains the smoothness class tau of the proxy variable along grid
lines from a previously trained ANN (Sec. 4 and Sec. 5 item 2; the network
itself is specified in Part I, Sec. 5.1, and its references, which are not
reproduced).  Reading used here: a multilayer perceptron over windows of 16
consecutive normalized values of a grid line, hidden layers of 64 and 64
ReLU units, three output classes (0 smooth, 1 discontinuity in the window,
2 discontinuity at the window's centre), argmax with ties to the higher
class.  Forward, backward and Adam are written out in FP64 for gradient
checks and as the reference trainer.

parity unpinned: the class semantics and training targets of Part I are not
available; the network is judged by its accuracy on labelled synthetic lines
and by the viscosity it yields.
"""
from __future__ import annotations

import numpy as np

WINDOW = 16
HIDDEN = 64
CLASSES = 3
FLAT_TOL = 1e-3


def init_params(rng: np.random.Generator):
    """He-normal initial weights (FP32 values kept in FP64 arrays)."""
    def he(fan_in, shape):
        return (rng.standard_normal(shape) * np.sqrt(2.0 / fan_in)).astype(np.float32).astype(np.float64)
    return {
        "W1": he(WINDOW, (HIDDEN, WINDOW)), "b1": np.zeros(HIDDEN),
        "W2": he(HIDDEN, (HIDDEN, HIDDEN)), "b2": np.zeros(HIDDEN),
        "W3": he(HIDDEN, (CLASSES, HIDDEN)), "b3": np.zeros(CLASSES),
    }


def normalize_windows(v: np.ndarray):
    """(v - min) / (max - min) per window; windows whose range is below
    FLAT_TOL * max(max|v|, 1) are flagged flat (classified smooth)."""
    lo = v.min(axis=-1, keepdims=True)
    hi = v.max(axis=-1, keepdims=True)
    rng = hi - lo
    scale = np.maximum(np.abs(v).max(axis=-1, keepdims=True), 1.0)
    flat = (rng < FLAT_TOL * scale)[..., 0]
    x = (v - lo) / np.where(rng > 0, rng, 1.0)
    return x, flat


def forward(params, x: np.ndarray):
    """Logits of the MLP for normalized windows x (m, 16); also returns the
    activations needed by :func:`backward`."""
    z1 = x @ params["W1"].T + params["b1"]
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ params["W2"].T + params["b2"]
    a2 = np.maximum(z2, 0.0)
    z3 = a2 @ params["W3"].T + params["b3"]
    return z3, (x, z1, a1, z2, a2)


def argmax_high(logits: np.ndarray) -> np.ndarray:
    """Argmax over classes with ties resolved to the higher class."""
    rev = logits[..., ::-1]
    return (logits.shape[-1] - 1 - np.argmax(rev, axis=-1)).astype(np.int64)


def classify(params, v: np.ndarray) -> np.ndarray:
    """tau for raw (unnormalized) windows v (m, 16)."""
    x, flat = normalize_windows(v)
    tau = argmax_high(forward(params, x)[0])
    return np.where(flat, 0, tau)


def loss_and_grads(params, x: np.ndarray, labels: np.ndarray, class_weight=None):
    """Mean (optionally class-weighted) softmax cross-entropy and its
    gradients with respect to every parameter."""
    logits, (x, z1, a1, z2, a2) = forward(params, x)
    m = x.shape[0]
    zmax = logits.max(axis=1, keepdims=True)
    ex = np.exp(logits - zmax)
    prob = ex / ex.sum(axis=1, keepdims=True)
    w = np.ones(m) if class_weight is None else class_weight[labels]
    wsum = w.sum()
    loss = -(w * np.log(prob[np.arange(m), labels])).sum() / wsum
    g3 = prob.copy()
    g3[np.arange(m), labels] -= 1.0
    g3 *= (w / wsum)[:, None]
    grads = {"W3": g3.T @ a2, "b3": g3.sum(axis=0)}
    g2 = (g3 @ params["W3"]) * (z2 > 0)
    grads["W2"] = g2.T @ a1
    grads["b2"] = g2.sum(axis=0)
    g1 = (g2 @ params["W2"]) * (z1 > 0)
    grads["W1"] = g1.T @ x
    grads["b1"] = g1.sum(axis=0)
    return loss, grads


def loss_and_grads_lowp(params, x: np.ndarray, labels: np.ndarray, class_weight=None):
    """loss_and_grads with the training's low-precision products: the
    inputs, the weight matrices and the hidden activations rounded to bf16
    (nearest even) wherever they enter a product, forward and backward; all
    other arithmetic in FP64.  Gradients are those of the rounded network,
    taken as the gradients of the unrounded weights."""
    W1, W2, W3 = (round_bf16(np.asarray(params[k], dtype=np.float64)) for k in ("W1", "W2", "W3"))
    xr = round_bf16(np.asarray(x, dtype=np.float64))
    z1 = xr @ W1.T + params["b1"]
    a1 = round_bf16(np.maximum(z1, 0.0))
    z2 = a1 @ W2.T + params["b2"]
    a2 = round_bf16(np.maximum(z2, 0.0))
    logits = a2 @ W3.T + params["b3"]
    m = xr.shape[0]
    zmax = logits.max(axis=1, keepdims=True)
    ex = np.exp(logits - zmax)
    prob = ex / ex.sum(axis=1, keepdims=True)
    w = np.ones(m) if class_weight is None else class_weight[labels]
    wsum = w.sum()
    loss = -(w * np.log(prob[np.arange(m), labels])).sum() / wsum
    g3 = prob.copy()
    g3[np.arange(m), labels] -= 1.0
    g3 *= (w / wsum)[:, None]
    grads = {"W3": g3.T @ a2, "b3": g3.sum(axis=0)}
    g2 = (g3 @ W3) * (z2 > 0)
    grads["W2"] = g2.T @ a1
    grads["b2"] = g2.sum(axis=0)
    g1 = (g2 @ W2) * (z1 > 0)
    grads["W1"] = g1.T @ xr
    grads["b1"] = g1.sum(axis=0)
    return loss, grads


def adam_update(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) with bias correction; state holds m, v, t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m[...] = b1 * m + (1 - b1) * grads[k]
        v[...] = b2 * v + (1 - b2) * grads[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return params


# ---------------------------------------------------------------- modal fallback
MODAL_HIGH = 8          # modes of degree >= MODAL_HIGH count as "high"
MODAL_T2 = 10.0 ** -1.5  # energy fraction above which tau = 2
MODAL_T1 = 10.0 ** -3.0  # energy fraction above which tau = 1


def modal_basis():
    """Orthonormal discrete polynomials of degree 0..15 on 16 equispaced
    points (columns), by high-precision QR of the Vandermonde matrix."""
    import mpmath as mp
    with mp.workprec(256):
        V = mp.matrix(WINDOW, WINDOW)
        for i in range(WINDOW):
            for k in range(WINDOW):
                V[i, k] = (mp.mpf(2 * i) / (WINDOW - 1) - 1) ** k
        Q, R = mp.qr(V)
        out = np.array([[float(Q[i, k]) * (1.0 if R[k, k] > 0 else -1.0) for k in range(WINDOW)]
                        for i in range(WINDOW)])
    return out


_MODAL_P = None


def modal_classify(v: np.ndarray) -> np.ndarray:
    """Modal-decay smoothness indicator (fallback; in the spirit of
    Persson & Peraire 2006): fraction of the non-constant modal energy of
    the normalized window carried by the modes of degree >= 8."""
    global _MODAL_P
    if _MODAL_P is None:
        _MODAL_P = modal_basis()
    x, flat = normalize_windows(v)
    c = x @ _MODAL_P
    e_all = (c[:, 1:] ** 2).sum(axis=1)
    e_hi = (c[:, MODAL_HIGH:] ** 2).sum(axis=1)
    frac = e_hi / np.where(e_all > 0, e_all, 1.0)
    tau = np.where(frac > MODAL_T2, 2, np.where(frac > MODAL_T1, 1, 0))
    return np.where(flat, 0, tau).astype(np.int64)


def round_bf16(a: np.ndarray) -> np.ndarray:
    """Round FP64 values to the nearest bfloat16 (ties to even), returned as
    FP64.  Values go through FP32 first, as a device conversion does."""
    f = np.asarray(a, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    bits = (bits + 0x7FFF + lsb) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_lowp(params, x: np.ndarray) -> np.ndarray:
    """Logits with bfloat16 inputs, weights and hidden activations and
    FP32 accumulation (the precision in which the device takes the argmax
    decision)."""
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    h = round_bf16(x)
    for k in ("1", "2"):
        z = f32(f32(h @ round_bf16(params["W" + k]).T) + f32(params["b" + k]))
        h = round_bf16(np.maximum(z, 0.0))
    return f32(f32(h @ round_bf16(params["W3"]).T) + f32(params["b3"]))


def classify_lowp(params, v: np.ndarray):
    """tau as the device takes it (see :func:`forward_lowp`); also returns the
    gap between the two largest logits, to recognise near-ties."""
    x, flat = normalize_windows(v)
    z = forward_lowp(params, x)
    tau = argmax_high(z)
    zs = np.sort(z, axis=-1)
    gap = zs[..., -1] - zs[..., -2]
    return np.where(flat, 0, tau), np.where(flat, np.inf, gap)
