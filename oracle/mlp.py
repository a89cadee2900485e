"""FP64 reference for the learned seed network (TEST INFRASTRUCTURE ONLY).

A fully connected ReLU network trained by back-propagation on events with
known positions (Sec. 5.1.3), written out plainly in NumPy float64:

  inputs   x_a = n_a * n_active / N over the active sensors (zero padded)
  hidden   h_l = relu(W_l h_{l-1} + b_l)
  output   y = W_out h_L + b_out = (p_x, p_y, p_z, s)
  loss     mean over events of 0.5 exp(-s) |p - t|^2 + 1.5 s,
           t = (position - offset) / scale

With `emulate=True` every quantity the GPU stores in bfloat16 is rounded to
bfloat16 (round to nearest even) at the same place: inputs, the weight
copies used in products, hidden activations, the output gradient used for
the output-layer weight gradient, and back-propagated hidden gradients.
Sums are exact FP64 here (the GPU accumulates in FP32).

Flat parameter order: W_1 [hidden][n_in_pad], b_1, ..., W_out [4][hidden],
b_out.
"""
from __future__ import annotations

import numpy as np


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    x32 = np.asarray(x, np.float64).astype(np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


class Layout:
    def __init__(self, n_in, hidden=256, layers=3):
        self.n_in, self.hidden, self.layers = n_in, hidden, layers
        self.n_in_pad = (n_in + 31) // 32 * 32
        self.shapes = []
        off = 0
        for l in range(layers + 1):
            di = self.n_in_pad if l == 0 else hidden
            do = 4 if l == layers else hidden
            self.shapes.append((off, do, di))
            off += do * di + do
        self.n_params = off

    def unpack(self, p):
        Ws, bs = [], []
        for off, do, di in self.shapes:
            Ws.append(np.asarray(p[off:off + do * di], np.float64).reshape(do, di))
            bs.append(np.asarray(p[off + do * di:off + do * di + do], np.float64))
        return Ws, bs

    def pack(self, Ws, bs):
        out = np.zeros(self.n_params)
        for (off, do, di), W, b in zip(self.shapes, Ws, bs):
            out[off:off + do * di] = W.reshape(-1)
            out[off + do * di:off + do * di + do] = b
        return out

    def random(self, seed, scale=1.0):
        """He-uniform weights (fan-in of the real inputs), small random biases."""
        rng = np.random.default_rng(seed)
        Ws, bs = [], []
        for l, (off, do, di) in enumerate(self.shapes):
            fan = self.n_in if l == 0 else self.hidden
            W = rng.uniform(-1, 1, (do, di)) * np.sqrt(6.0 / fan) * scale
            if l == 0:
                W[:, self.n_in:] = 0.0
            Ws.append(W)
            bs.append(rng.uniform(-0.05, 0.05, do))
        return self.pack(Ws, bs)


def inputs(lay, signals, emulate):
    """Normalised inputs; events with a non-positive or non-finite sum get 0."""
    s = np.asarray(signals, np.float64)
    N = s.astype(np.float32).sum(1, dtype=np.float32).astype(np.float64)
    ok = np.isfinite(s).all(1) & (s >= 0).all(1) & (N > 0)
    scale = np.where(ok, (np.float32(lay.n_in) / np.where(ok, N, 1).astype(np.float32)), 0)
    scale = scale.astype(np.float32).astype(np.float64)
    x = (s * scale[:, None])
    x = x.astype(np.float32).astype(np.float64) if emulate else x
    x = np.where(ok[:, None], x, 0.0)
    if emulate:
        x = bf16(x)
    X = np.zeros((s.shape[0], lay.n_in_pad))
    X[:, :lay.n_in] = x
    return X


def forward(lay, p, signals, emulate=True):
    """Returns (y [n][4], list of layer inputs/activations)."""
    Ws, bs = lay.unpack(p)
    if emulate:
        Ws = [bf16(W) for W in Ws]
    h = inputs(lay, signals, emulate)
    acts = [h]
    for l in range(lay.layers):
        h = np.maximum(h @ Ws[l].T + bs[l], 0.0)
        if emulate:
            h = bf16(h)
        acts.append(h)
    y = h @ Ws[-1].T + bs[-1]
    return y, acts


def loss_and_grad(lay, p, signals, targets, scale, offset, emulate=True):
    """Mean loss over the batch and its gradient with respect to p."""
    Ws, bs = lay.unpack(p)
    Wq = [bf16(W) for W in Ws] if emulate else Ws
    y, acts = forward(lay, p, signals, emulate)
    n = y.shape[0]
    t = (np.asarray(targets, np.float64)[:, :3] - np.asarray(offset)) / np.asarray(scale)
    r = y[:, :3] - t
    s = y[:, 3]
    es = np.exp(-s)
    r2 = (r * r).sum(1)
    loss = np.mean(0.5 * es * r2 + 1.5 * s)
    dY = np.concatenate([es[:, None] * r, (1.5 - 0.5 * es * r2)[:, None]], 1) / n
    gW = [None] * (lay.layers + 1)
    gb = [None] * (lay.layers + 1)
    L = lay.layers
    gb[L] = dY.sum(0)
    gW[L] = (bf16(dY) if emulate else dY).T @ acts[L]
    dH = (dY @ Wq[L]) * (acts[L] > 0)
    if emulate:
        dH = bf16(dH)
    for l in range(L - 1, -1, -1):
        gb[l] = dH.sum(0)
        gW[l] = dH.T @ acts[l]
        if l > 0:
            dH = (dH @ Wq[l]) * (acts[l] > 0)
            if emulate:
                dH = bf16(dH)
    return loss, lay.pack(gW, gb)


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba) with bias correction; returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
