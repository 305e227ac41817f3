"""Learned initial guess: a small convolutional network in plain NumPy FP64.
Test infrastructure only.

The paper has no learned component; the network is this project's own
design for the Newton initial guess of the nonlinear problem.  Layers, in
NHWC layout (batch, y, x, channel) on the interior vertex grid:

  Z_l = conv3x3(A_{l-1}, W_l) + b_l,   A_l = max(Z_l, 0)   (l = 1..L-1),
  O   = conv3x3(A_{L-1}, W_L) + b_L,
  U   = env[y, x] * oscale[k] * O[..., k]

conv3x3 is a cross-correlation with zero padding of one vertex:
  Z[b, y, x, o] = sum_{dy, dx, i} A[b, y+dy-1, x+dx-1, i] W[dy, dx, i, o].
The loss is the mean squared error of U in units of oscale:
  loss = mean_{b,y,x,k} (env O - T / oscale)^2.
The optimiser is Adam (Kingma and Ba, 2015) with bias correction.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np


def conv3x3(A: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """A [B,H,Wd,Ci], W [3,3,Ci,Co], b [Co] -> [B,H,Wd,Co]."""
    Bn, H, Wd, _ = A.shape
    Ap = np.pad(A, ((0, 0), (1, 1), (1, 1), (0, 0)))
    out = np.zeros((Bn, H, Wd, W.shape[3])) + b
    for dy in range(3):
        for dx in range(3):
            out += Ap[:, dy:dy + H, dx:dx + Wd, :] @ W[dy, dx]
    return out


def conv3x3_backward(A: np.ndarray, W: np.ndarray, dZ: np.ndarray):
    """Gradients of sum(dZ * conv3x3(A, W, b)) w.r.t. A, W and b."""
    Bn, H, Wd, _ = A.shape
    Ap = np.pad(A, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dAp = np.zeros_like(Ap)
    dW = np.zeros_like(W)
    for dy in range(3):
        for dx in range(3):
            win = Ap[:, dy:dy + H, dx:dx + Wd, :]
            dW[dy, dx] = np.einsum("byxi,byxo->io", win, dZ)
            dAp[:, dy:dy + H, dx:dx + Wd, :] += dZ @ W[dy, dx].T
    db = dZ.sum(axis=(0, 1, 2))
    return dAp[:, 1:-1, 1:-1, :], dW, db


def init_params(sizes: List[int], seed: int = 0) -> List[Tuple[np.ndarray, np.ndarray]]:
    """He-normal weights, zero biases; sizes = [cin, hidden..., cout]."""
    rng = np.random.default_rng(seed)
    out = []
    for ci, co in zip(sizes[:-1], sizes[1:]):
        W = rng.standard_normal((3, 3, ci, co)) * np.sqrt(2.0 / (9 * ci))
        out.append((W, np.zeros(co)))
    return out


def forward(params, X: np.ndarray):
    """Returns O (network output) and the activations [X, A_1, ..., A_{L-1}]."""
    acts = [X]
    A = X
    for l, (W, b) in enumerate(params):
        Z = conv3x3(A, W, b)
        if l + 1 < len(params):
            A = np.maximum(Z, 0.0)
            acts.append(A)
        else:
            return Z, acts
    raise ValueError("empty network")


def predict(params, X, env, oscale):
    O, _ = forward(params, X)
    return env[None, :, :, None] * oscale[None, None, None, :] * O


def loss_and_grads(params, X, T, env, oscale):
    """loss = mean (env O - T/oscale)^2 and its gradient per (W, b)."""
    O, acts = forward(params, X)
    E = env[None, :, :, None] * O - T / oscale[None, None, None, :]
    count = E.size
    loss = float((E * E).sum() / count)
    dZ = 2.0 * env[None, :, :, None] * E / count
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        dA, dW, db = conv3x3_backward(acts[l], W, dZ)
        grads[l] = (dW, db)
        if l > 0:
            dZ = dA * (acts[l] > 0.0)
    return loss, grads


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update; state = {"t": int, "m": [...], "v": [...]} (created
    when empty).  Returns the new parameters."""
    if not state:
        state["t"] = 0
        state["m"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        state["v"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    state["t"] += 1
    t = state["t"]
    out = []
    for l, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        new = []
        for j, (p, g) in enumerate(((W, gW), (b, gb))):
            m = beta1 * state["m"][l][j] + (1.0 - beta1) * g
            v = beta2 * state["v"][l][j] + (1.0 - beta2) * g * g
            mh = m / (1.0 - beta1 ** t)
            vh = v / (1.0 - beta2 ** t)
            new.append(p - lr * mh / (np.sqrt(vh) + eps))
            ms = list(state["m"][l]); ms[j] = m; state["m"][l] = tuple(ms)
            vs = list(state["v"][l]); vs[j] = v; state["v"][l] = tuple(vs)
        out.append((new[0], new[1]))
    return out


def flatten(params) -> np.ndarray:
    """Concatenate W_1, b_1, ..., W_L, b_L (C order)."""
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params])


def unflatten(vec: np.ndarray, sizes: List[int]):
    out, q = [], 0
    for ci, co in zip(sizes[:-1], sizes[1:]):
        nw = 9 * ci * co
        W = vec[q:q + nw].reshape(3, 3, ci, co)
        q += nw
        b = vec[q:q + co]
        q += co
        out.append((W.astype(np.float64), b.astype(np.float64)))
    if q != vec.size:
        raise ValueError("parameter vector size mismatch")
    return out


def input_channels(g0: np.ndarray, g: np.ndarray) -> np.ndarray:
    """The network's input channels at npts points: [c0, g_1 .. g_M] with c0
    the mean of the log-normal coefficient (Eq. inputlogn), taken from the
    input chaos expansion (its zero-order coefficient).  g0 [npts],
    g [M, npts] -> [npts, M + 1]."""
    from . import pce
    M = g.shape[0]
    c0 = pce.lognormal_coefficients(g0, g, np.zeros((1, M), dtype=np.int64))[0]
    return np.concatenate([c0[:, None], g.T], axis=1)


def output_map(shape: np.ndarray, T: np.ndarray):
    """env = shape / max(shape); oscale[k] = max(RMS of T[..., k] over samples
    and pixels, 1e-30) / RMS(env).  shape [H*W], T [B, H*W, c_L]."""
    env = shape / shape.max()
    rms_t = np.sqrt((T.reshape(-1, T.shape[-1]) ** 2).mean(axis=0))
    return env, np.maximum(rms_t, 1e-30) / np.sqrt((env ** 2).mean())
