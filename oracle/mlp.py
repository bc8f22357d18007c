"""Reference multilayer perceptron for the learned foot-of-normal seed (oracle side).

Not part of the paper: a small network maps (x, y, curve descriptors) of a
point near Gamma to a guess of its foot of the normal, which then seeds the
Newton solve of Sec. 3.4.  Architecture: 16 inputs, three hidden layers of 64
tanh units, 2 linear outputs; weights stored flat, layer by layer, each layer
as W (row-major [fan_in][fan_out]) followed by b [fan_out].

Features of a point (x, y) near a curve r(t) = 1 + sum_{m=2..8} (a_m cos mt + b_m sin mt):
    (x, y, a_2 s_2, b_2 s_2, ..., a_8 s_8, b_8 s_8),  s_m = m / 0.15
Targets: (delta / DELTA_SCALE, eta / width) with delta = theta^Q - atan2(y, x)
wrapped to (-pi, pi] and eta the signed distance; width = C k1 of the strip.
Loss: mean over the batch of 0.5 |out - target|^2.

This module computes in float64 and is the reference for the library's FP32
forward / backward kernels.
"""
import math

import numpy as np

LAYERS = [(16, 64), (64, 64), (64, 64), (64, 2)]
NW = sum(i * o + o for i, o in LAYERS)
DELTA_SCALE = 0.05
DESC_SCALE = 1.0 / 0.15


def features(x, y, desc):
    """desc [14] = (a_2, b_2, ..., a_8, b_8); returns [n, 16]."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    d = np.asarray(desc, dtype=np.float64).reshape(7, 2) * (np.arange(2, 9)[:, None] * DESC_SCALE)
    out = np.empty((x.size, 16))
    out[:, 0] = x.ravel()
    out[:, 1] = y.ravel()
    out[:, 2:] = d.ravel()[None, :]
    return out


def targets(x, y, theta, eta, width):
    delta = np.mod(theta - np.arctan2(y, x) + math.pi, 2 * math.pi) - math.pi
    return np.stack([delta / DELTA_SCALE, eta / width], axis=1)


def unpack(w):
    out = []
    o = 0
    for fi, fo in LAYERS:
        W = w[o:o + fi * fo].reshape(fi, fo)
        o += fi * fo
        b = w[o:o + fo]
        o += fo
        out.append((W, b))
    return out


def init_weights(seed):
    """Glorot-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for fi, fo in LAYERS:
        lim = math.sqrt(6.0 / (fi + fo))
        parts.append(rng.uniform(-lim, lim, fi * fo))
        parts.append(np.zeros(fo))
    return np.concatenate(parts)


def forward(w, X):
    """Returns output [n, 2] and the activations of every layer."""
    acts = [X]
    h = X
    layers = unpack(w)
    for li, (W, b) in enumerate(layers):
        z = h @ W + b
        h = np.tanh(z) if li < len(layers) - 1 else z
        acts.append(h)
    return h, acts


def loss_and_grad(w, X, Y):
    """Mean 0.5 |f(X) - Y|^2 and its gradient with respect to the flat weights."""
    out, acts = forward(w, X)
    n = X.shape[0]
    r = out - Y
    loss = 0.5 * np.sum(r * r) / n
    layers = unpack(w)
    grads = [None] * len(layers)
    delta = r / n                                   # d loss / d z of the output layer
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        gW = acts[li].T @ delta
        gb = delta.sum(axis=0)
        grads[li] = (gW, gb)
        if li > 0:
            dh = delta @ W.T
            delta = dh * (1.0 - acts[li] ** 2)      # tanh' through the layer below's output
    return loss, np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


def adam_step(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, 2015) in place; t counts from 1."""
    m *= b1
    m += (1 - b1) * g
    v *= b2
    v += (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    w -= lr * mh / (np.sqrt(vh) + eps)
