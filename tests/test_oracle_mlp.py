"""Pins for the oracle MLP (learned foot seed): analytic gradient against
central finite differences, shapes, Adam's first step, the polar derivative
series against closed forms, and the features against the first-order Newton
step from the polar angle checked on the oracle's own foot solve."""
import math

import numpy as np

import workloads as W
from oracle import mlp
from oracle import curves as OC
from oracle import plan as OP


def test_sizes():
    assert mlp.NW == 8 * 64 + 64 + 64 * 64 + 64 + 64 * 64 + 64 + 64 * 2 + 2
    w = mlp.init_weights(0)
    assert w.size == mlp.NW


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    w = mlp.init_weights(2) + rng.normal(0, 0.01, mlp.NW)
    X = rng.normal(0, 1, (13, mlp.NIN))
    Y = rng.normal(0, 1, (13, 2))
    _, g = mlp.loss_and_grad(w, X, Y)
    idx = rng.choice(mlp.NW, 40, replace=False)
    idx[:4] = [0, mlp.NW - 1, mlp.NW - 3, 8 * 64 + 5]     # first weight, output biases, a hidden bias
    for k in idx:
        e = np.zeros(mlp.NW)
        e[k] = 1e-6
        fd = (mlp.loss_and_grad(w + e, X, Y)[0] - mlp.loss_and_grad(w - e, X, Y)[0]) / 2e-6
        assert abs(fd - g[k]) < 1e-7 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_zero_weights_output_biases():
    w = np.zeros(mlp.NW)
    w[-2:] = [0.3, -0.2]
    out, _ = mlp.forward(w, np.ones((4, mlp.NIN)))
    assert np.allclose(out, [[0.3, -0.2]] * 4)


def test_adam_first_step_moves_by_lr():
    w = np.zeros(3)
    g = np.array([1.0, -2.0, 0.5])
    m = np.zeros(3)
    v = np.zeros(3)
    mlp.adam_step(w, g, m, v, 1, 0.01)
    assert np.allclose(w, -0.01 * np.sign(g), atol=1e-9)


def test_targets_wrap():
    F = np.zeros((1, mlp.NIN))
    t = mlp.targets(np.array([-1.0]), np.array([-1e-9]), np.array([math.pi - 1e-3]), np.array([0.01]), 0.02, F)
    # atan2 is close to -pi, theta close to +pi: the wrapped difference is small
    assert abs(t[0, 0] / mlp.TARGET_SCALE * 0.02) < 2e-3 and abs(t[0, 1] / mlp.TARGET_SCALE - 0.5) < 1e-12


def test_polar_derivatives_closed_form():
    a, b, m = 0.07, -0.03, 3
    coef = [1.2] + [0.0] * 8
    coef[2 * m - 1], coef[2 * m] = a, b
    t = np.linspace(0, 2 * math.pi, 11)
    R = mlp.polar_derivatives(coef, t)
    c, s = np.cos(m * t), np.sin(m * t)
    ref = [1.2 + a * c + b * s, m * (-a * s + b * c), -m ** 2 * (a * c + b * s), m ** 3 * (a * s - b * c),
           m ** 4 * (a * c + b * s), m ** 5 * (-a * s + b * c)]
    for k in range(6):
        assert np.allclose(R[k], ref[k], rtol=0, atol=1e-12), k


def test_features_on_the_disc():
    w = 0.02
    th = np.linspace(0.1, 6.0, 7)
    r = 1.0 + 0.3 * w
    x, y = r * np.cos(th), r * np.sin(th)
    f = mlp.features(x, y, [1.0], w)
    assert np.allclose(f[:, 0], 0.3, atol=1e-12)
    assert np.all(f[:, 1:] == 0.0)
    # the foot of the normal on the circle is the polar angle: nothing left to learn
    T = mlp.targets(x, y, th, 0.3 * w * np.ones(7), w, f)
    assert np.abs(T).max() < 1e-9
    s0 = mlp.seed_theta(np.zeros((7, 2)), x, y, w, f)
    assert np.abs(np.mod(s0 - th + math.pi, 2 * math.pi) - math.pi).max() < 1e-15


def test_first_order_feature_predicts_the_foot():
    """Close to Gamma the foot offset delta = theta^Q - phi is w f7 / R_0 to first
    order in the distance: checked against the oracle's Newton foot solve."""
    (kind, coef), _, _ = W.random_polar(3)
    cv = OC.Curve(kind, coef)
    B = 4096
    bd = OC.boundary_grid(cv, B)
    rng = np.random.default_rng(4)
    t = rng.uniform(0, 2 * math.pi, 50)
    x, y, x1, y1, _, _ = cv.eval_vec(t)
    sp = np.hypot(x1, y1)
    w = 0.02
    for eta in (1e-3, 1e-4):
        X = x + eta * y1 / sp
        Y = y - eta * x1 / sp
        p = np.rint(np.mod(np.arctan2(Y, X), 2 * math.pi) / bd["k2"]).astype(np.int64) % B
        th, et, _ = OP.foot_solve(cv, bd, X, Y, p, 8)
        assert np.abs(et - eta).max() < 1e-13
        assert np.abs(np.mod(th - t + math.pi, 2 * math.pi) - math.pi).max() < 1e-12
        f = mlp.features(X, Y, coef, w)
        T = mlp.targets(X, Y, th, et, w, f) / mlp.TARGET_SCALE
        # what the first-order estimates miss is O(eta^2)
        assert np.abs(T[:, 0]).max() < 40 * eta ** 2, (eta, np.abs(T[:, 0]).max())
        assert np.abs(T[:, 1]).max() < 40 * eta ** 2, (eta, np.abs(T[:, 1]).max())
        # the seed from a zero correction is the first-order Newton step
        s0 = mlp.seed_theta(np.zeros((X.size, 2)), X, Y, w, f)
        assert np.abs(np.mod(s0 - th + math.pi, 2 * math.pi) - math.pi).max() < 40 * w * eta ** 2
