"""FP64 numpy oracle of the learned proposal network (test infrastructure only).

The network is not in the paper: it is an added serving pattern that
proposes the initial disparity and a confidence at the 1/16 pyramid level,
so that the coarse BDIS levels can be skipped.  This module states what the
GPU kernels compute, in plain numpy loops over the nine taps of each 3x3
convolution, in float64, on operands the caller has already rounded to
bfloat16 where the GPU holds bfloat16 (bf16() below).  Layout: activations
NHWC, weights [3, 3, C_in, C_out] (tap dy, tap dx), biases [C_out].

Only the tests, the smoke check and the benchmark's CPU leg use this module.
"""
from __future__ import annotations

import numpy as np


def bf16(a):
    """Round float values to bfloat16 (round to nearest, ties to even) and
    return them as float64.  NaN/inf are not expected here."""
    a32 = np.asarray(a, np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def conv3x3(x, w, b):
    """y[n, i, j, co] = b[co] + sum_{dy, dx, ci} x[n, i + dy - 1, j + dx - 1, ci] w[dy, dx, ci, co],
    zero outside the image (same-size output)."""
    N, H, W, Ci = x.shape
    Co = w.shape[3]
    xp = np.zeros((N, H + 2, W + 2, Ci))
    xp[:, 1:-1, 1:-1, :] = x
    y = np.broadcast_to(np.asarray(b, np.float64), (N, H, W, Co)).copy()
    for dy in range(3):
        for dx in range(3):
            y += xp[:, dy:dy + H, dx:dx + W, :] @ w[dy, dx]
    return y


def conv3x3_backward(x, w, gy):
    """Gradients of sum(gy * conv3x3(x, w, b)) with respect to x, w and b."""
    N, H, W, Ci = x.shape
    xp = np.zeros((N, H + 2, W + 2, Ci))
    xp[:, 1:-1, 1:-1, :] = x
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w, dtype=np.float64)
    for dy in range(3):
        for dx in range(3):
            win = xp[:, dy:dy + H, dx:dx + W, :]
            gw[dy, dx] = np.einsum("nhwc,nhwo->co", win, gy)
            gxp[:, dy:dy + H, dx:dx + W, :] += gy @ w[dy, dx].T
    gb = gy.sum(axis=(0, 1, 2))
    return gxp[:, 1:-1, 1:-1, :], gw, gb


def relu(x):
    return np.maximum(x, 0.0)


class Net:
    """Layer list [(w, b), ...]; ReLU after every layer but the last.  The
    last layer has two outputs: disparity (coarse pixels) and the logit of
    the confidence."""

    def __init__(self, layers):
        self.layers = [(np.asarray(w, np.float64), np.asarray(b, np.float64)) for w, b in layers]

    def forward(self, x, round_act=True):
        """Returns (output, cache).  With round_act, hidden activations are
        rounded to bfloat16 as the GPU stores them."""
        acts = [x]
        h = x
        for i, (w, b) in enumerate(self.layers):
            z = conv3x3(h, w, b)
            if i < len(self.layers) - 1:
                h = relu(z)
                if round_act:
                    h = bf16(h)
            else:
                h = z
            acts.append(h)
        return h, acts

    def backward(self, acts, gout, round_grad=True):
        """Gradients of sum(gout * forward(x)) for every layer, given the
        cached activations.  With round_grad, the gradient entering each
        layer is rounded to bfloat16 as the GPU stores it."""
        grads = [None] * len(self.layers)
        g = gout
        for i in range(len(self.layers) - 1, -1, -1):
            w, _ = self.layers[i]
            if round_grad:
                g = bf16(g)
            gx, gw, gb = conv3x3_backward(acts[i], w, g)
            grads[i] = (gw, gb)
            if i > 0:
                g = gx * (acts[i] > 0)
        return grads


def loss_and_grad(out, target, valid, conf_tol=0.5, delta=1.0, conf_weight=0.1):
    """Per valid pixel: Huber(d - t, delta) + conf_weight * BCE(sigmoid(c), q)
    with q = 1 if |d - t| < conf_tol else 0 (no gradient through q); mean
    over the valid pixels.  Returns (loss, dloss/dout)."""
    d = out[..., 0]
    c = out[..., 1]
    n = max(int(valid.sum()), 1)
    e = d - target
    a = np.abs(e)
    hub = np.where(a <= delta, 0.5 * e * e, delta * (a - 0.5 * delta))
    gd = np.where(a <= delta, e, delta * np.sign(e))
    q = (a < conf_tol).astype(np.float64)
    # BCE with logits: softplus(c) - q c
    bce = np.maximum(c, 0) - q * c + np.log1p(np.exp(-np.abs(c)))
    sig = 1.0 / (1.0 + np.exp(-c))
    gc = sig - q
    m = valid.astype(np.float64)
    loss = float(((hub + conf_weight * bce) * m).sum() / n)
    g = np.zeros_like(out)
    g[..., 0] = gd * m / n
    g[..., 1] = conf_weight * gc * m / n
    return loss, g


def adam(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def net_input(Lc, Rc, ndisp=14, scale=64.0, offset=128.0):
    """Input channels at the coarse level from the coarse left and right
    images (values in gray levels): (L - offset)/scale, (R - offset)/scale,
    then |L(x) - R(x - d)| / scale for d = 0..ndisp-1 with R's column clamped
    to the image.  Returns (H, W, 2 + ndisp)."""
    H, W = Lc.shape
    ch = [(Lc - offset) / scale, (Rc - offset) / scale]
    for d in range(ndisp):
        idx = np.clip(np.arange(W) - d, 0, W - 1)
        ch.append(np.abs(Lc - Rc[:, idx]) / scale)
    return np.stack(ch, axis=-1)
