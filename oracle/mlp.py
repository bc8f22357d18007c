"""Reference multilayer perceptron for the learned foot-of-normal seed (oracle side).

TEST INFRASTRUCTURE ONLY: this module is the float64 reference that the
library's FP32 training and inference kernels are checked against.  It is not
part of the paper: a small network maps a point near a polar curve to a guess
of its foot of the normal, which then seeds the Newton solve of Sec. 3.4.

Architecture: 8 inputs, three hidden layers of 64 tanh units, 2 linear
outputs.  Weights are stored flat, layer by layer, each layer as W (row-major
[fan_in][fan_out]) followed by b [fan_out].

Features.  For a polar curve r(t) = c_0 + sum_m (a_m cos mt + b_m sin mt) and a
point Q = rho (cos phi, sin phi) (phi = atan2(y, x)), the foot depends on Q
and the curve only through rho and the derivatives R_k = r^(k)(phi): rotating
the picture by -phi changes neither.  With w the strip width C k1:
    f0 = (rho - R_0) / w                 radial offset in strip widths
    f1 = R_0 - 1
    f2 = R_1 / R_0
    f3..f6 = R_k / (R_0 S_k), k = 2..5   (S_k = 2, 10, 60, 400)
    f7 = f0 f2 / (1 + f2^2)              the first-order Newton step from phi, / w
Targets.  With delta = theta^Q - phi wrapped to (-pi, pi] and eta the signed
distance, one Newton step on g(t) = (q(t) - Q) . q'(t) from t = phi gives the
first-order estimates  delta / w ~ f7 / R_0  and  eta / w ~ f0 / sqrt(1 + f2^2);
the network learns what these miss, scaled by TARGET_SCALE:
    target = TARGET_SCALE (delta / w - f7 / R_0,  eta / w - f0 / sqrt(1 + f2^2)).
Loss: mean over the batch of 0.5 |out - target|^2.  The Newton seed is
    theta^(0) = phi + w (f7 / R_0 + out_0 / TARGET_SCALE).
"""
import math

import numpy as np

NIN = 8
LAYERS = [(NIN, 64), (64, 64), (64, 64), (64, 2)]
NW = sum(i * o + o for i, o in LAYERS)
DERIV_SCALE = (1.0, 1.0, 2.0, 10.0, 60.0, 400.0)
TARGET_SCALE = 100.0


def polar_derivatives(coef, t, kmax=5):
    """r^(k)(t) for k = 0..kmax of r = c0 + sum_m (a_m cos mt + b_m sin mt),
    coef = [c0, a1, b1, a2, b2, ...].  Uses d^k/dt^k cos(mt) = m^k cos(mt + k pi/2)
    and likewise for sin."""
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros((kmax + 1,) + t.shape)
    out[0] += coef[0]
    nm = (len(coef) - 1) // 2
    for m in range(1, nm + 1):
        a, b = coef[2 * m - 1], coef[2 * m]
        for k in range(kmax + 1):
            ph = m * t + k * math.pi / 2
            out[k] += float(m) ** k * (a * np.cos(ph) + b * np.sin(ph))
    return out


def features(x, y, coef, width):
    """Points (x, y) near the polar curve coef -> [n, 8] features."""
    x = np.asarray(x, dtype=np.float64).ravel()
    y = np.asarray(y, dtype=np.float64).ravel()
    phi = np.arctan2(y, x)
    rho = np.hypot(x, y)
    R = polar_derivatives(coef, phi)
    f = np.empty((x.size, NIN))
    f[:, 0] = (rho - R[0]) / width
    f[:, 1] = R[0] - 1.0
    f[:, 2] = R[1] / R[0]
    for k in range(2, 6):
        f[:, k + 1] = R[k] / (R[0] * DERIV_SCALE[k])
    f[:, 7] = f[:, 0] * f[:, 2] / (1.0 + f[:, 2] ** 2)
    return f


def first_order(F):
    """First-order estimates (delta / w, eta / w) from the features [n, 8]."""
    return np.stack([F[:, 7] / (1.0 + F[:, 1]), F[:, 0] / np.sqrt(1.0 + F[:, 2] ** 2)], axis=1)


def targets(x, y, theta, eta, width, F):
    """Training targets for points (x, y) with foot theta and distance eta; F their features."""
    delta = np.mod(theta - np.arctan2(y, x) + math.pi, 2 * math.pi) - math.pi
    exact = np.stack([delta / width, eta / width], axis=1)
    return TARGET_SCALE * (exact - first_order(F))


def seed_theta(out, x, y, width, F):
    """Network output -> Newton seed theta^(0)."""
    return np.arctan2(y, x) + width * (first_order(F)[:, 0] + out[:, 0] / TARGET_SCALE)


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
