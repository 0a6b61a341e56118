"""Learned filter bounds: features and a small MLP (oracle, test infrastructure only).

The paper leaves the filter bounds' source open (it defines the filter only
through its centre c and half-width e, Sec. V-A.3); the engine adds a model
that predicts a subdomain's (lambda_max, lambda_cut, degree) from cheap
features of its local potential and geometry, trained on what the method
itself produces (Lanczos upper bounds, converged lambda_Ns, converged degree),
with Lanczos kept as the fallback.

Model: 64 -> 128 -> 128 -> 3, ReLU on the hidden layers, mean-squared error
on standardised targets, Adam (lr 1e-3, beta 0.9/0.999, eps 1e-8).
Layout: row-major activations X[b, f]; W_l is (fan_in, fan_out); y = x W + b.
Features (zero-padded to 64): 32-bin histogram of V over [min V, max V]
(fractions), n_atoms, n_x, n_y, n_z, h, buffer width (bohr), V min, max, mean,
std, N_s, projector count, sum |gamma|, core fraction, and the closed-form
largest eigenvalue of -1/2 Lap on the grid.
Pins: central finite differences of the gradients; with no hidden layer the
trained model converges to numpy.linalg.lstsq; Adam's first step has the
closed form -lr g / (|g| + eps) (tests/test_oracle_mlp.py).
"""
from __future__ import annotations

from typing import Dict, List, Sequence

import numpy as np

from . import grid as ogrid

N_FEAT = 64
HIDDEN = (128, 128)
N_OUT = 3


def features(sd) -> np.ndarray:
    v = np.asarray(sd.v, dtype=np.float64)
    f = np.zeros(N_FEAT)
    lo, hi = float(v.min()), float(v.max())
    if hi > lo:
        hist, _ = np.histogram(v, bins=32, range=(lo, hi))
    else:
        hist = np.zeros(32)
        hist[0] = v.size
    f[:32] = hist / v.size
    n = np.asarray(sd.n, dtype=np.float64)
    buf = float(np.min(np.asarray(sd.core_lo))) * sd.h
    k = 32
    vals = [len(sd.atoms), n[0], n[1], n[2], sd.h, buf, lo, hi, float(v.mean()), float(v.std()),
            float(sd.ns), 4.0 * len(sd.atoms), float(np.abs(np.asarray(sd.proj)[:, 2:6]).sum()),
            float(np.prod(np.asarray(sd.core_hi) - np.asarray(sd.core_lo)) / np.prod(n)),
            lap_lambda_max(sd)]
    f[k:k + len(vals)] = vals
    return f


def lap_lambda_max(sd) -> float:
    """Largest eigenvalue of -1/2 Lap on the grid (periodic closed form; an
    upper bound for the zero-Dirichlet box): (1/(2h^2)) sum_a s(pi)."""
    s_pi = float(ogrid.laplacian_symbol(np.array([np.pi]), 6)[0])
    return 1.5 * s_pi / sd.h ** 2


def forward(params: List[np.ndarray], X: np.ndarray):
    """params = [W1, b1, W2, b2, W3, b3]; returns (Y, cache)."""
    acts = [X]
    pre = []
    h = X
    nl = len(params) // 2
    for l in range(nl):
        W, b = params[2 * l], params[2 * l + 1]
        z = h @ W + b
        pre.append(z)
        h = np.maximum(z, 0.0) if l < nl - 1 else z
        acts.append(h)
    return h, (acts, pre)


def mse(Y: np.ndarray, T: np.ndarray) -> float:
    return float(np.mean((Y - T) ** 2))


def backward(params: List[np.ndarray], cache, Y: np.ndarray, T: np.ndarray) -> List[np.ndarray]:
    """Gradients of mse(Y, T) = mean over all B*out entries."""
    acts, pre = cache
    nl = len(params) // 2
    g = 2.0 * (Y - T) / Y.size
    grads = [None] * len(params)
    for l in reversed(range(nl)):
        if l < nl - 1:
            g = g * (pre[l] > 0)
        grads[2 * l] = acts[l].T @ g
        grads[2 * l + 1] = g.sum(axis=0)
        g = g @ params[2 * l].T
    return grads


def adam_init(params):
    return {"m": [np.zeros_like(p) for p in params], "v": [np.zeros_like(p) for p in params], "t": 0}


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    state["t"] += 1
    t = state["t"]
    out = []
    for i, (p, g) in enumerate(zip(params, grads)):
        state["m"][i] = b1 * state["m"][i] + (1 - b1) * g
        state["v"][i] = b2 * state["v"][i] + (1 - b2) * g * g
        mh = state["m"][i] / (1 - b1 ** t)
        vh = state["v"][i] / (1 - b2 ** t)
        out.append(p - lr * mh / (np.sqrt(vh) + eps))
    return out


def train(params, X, T, batches: Sequence[np.ndarray], lr=1e-3):
    """Adam over the given minibatch index lists (order fixed by the caller)."""
    st = adam_init(params)
    losses = []
    for idx in batches:
        Y, cache = forward(params, X[idx])
        losses.append(mse(Y, T[idx]))
        g = backward(params, cache, Y, T[idx])
        params = adam_step(params, g, st, lr)
    return params, losses
