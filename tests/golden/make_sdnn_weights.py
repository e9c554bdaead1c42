"""Train the reference smoothness classifier with the CPU oracle and store it.

Writes ``sdnn_oracle_weights.npz`` next to this script: the FP32 parameter
blob (W1, b1, W2, b2, W3, b3) of a 16-64-64-3 MLP trained in FP64 by the
oracle's forward/backward/Adam on windows of synthetic lines passed once
through the oracle's FC filter (d = 2, C = 27), with labels from the known
jump positions.  Only ``oracle`` and the seeded input generators are used.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import fcgram, sdnn  # noqa: E402


def training_windows(nlines, seed_salt, per_class=None):
    lines, pos, amp = W.classifier_lines(nlines, seed_salt=seed_salt)
    filt = fcgram.fc_apply(lines, 2, 27, "filter")
    lab = W.window_labels(pos, amp, lines)
    n = lines.shape[1]
    start = np.clip(np.arange(n) - 8, 0, n - 16)
    idx = start[:, None] + np.arange(16)[None, :]
    wins = filt[:, idx].reshape(-1, 16)
    labels = lab.reshape(-1)
    x, flat = sdnn.normalize_windows(wins)
    keep = ~flat
    return x[keep], labels[keep]


def blob(params):
    return np.concatenate([params[k].astype(np.float32).ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def main(out=os.path.join(HERE, "sdnn_oracle_weights.npz"), nlines=4000, epochs=12, batch=2048):
    x, y = training_windows(nlines, seed_salt=11)
    rng = W.rng(4, 12)
    params = W.sdnn_init(rng)
    params = {k: v.astype(np.float64) for k, v in params.items()}
    counts = np.bincount(y, minlength=3).astype(float)
    cw = counts.sum() / (3 * np.maximum(counts, 1))
    state = {}
    for ep in range(epochs):
        perm = rng.permutation(len(y))
        tot = 0.0
        for b in range(0, len(y) - batch + 1, batch):
            sel = perm[b:b + batch]
            loss, g = sdnn.loss_and_grads(params, x[sel], y[sel], cw)
            params = sdnn.adam_update(params, g, state, lr=2e-3)
            tot += loss
        print(f"epoch {ep} loss {tot / max(1, len(y) // batch):.4f}", flush=True)
    xt, yt = training_windows(1000, seed_salt=13)
    pred = sdnn.argmax_high(sdnn.forward(params, xt)[0])
    acc = float((pred == yt).mean())
    print("held-out accuracy", acc)
    np.savez(out, params=blob(params), heldout_accuracy=acc, class_weight=cw)


if __name__ == "__main__":
    main()
