"""Pins for the oracle MLP (learned foot seed): analytic gradient against
central finite differences, shapes, Adam's first step, feature/target maps."""
import math

import numpy as np

from oracle import mlp


def test_sizes():
    assert mlp.NW == 16 * 64 + 64 + 64 * 64 + 64 + 64 * 64 + 64 + 64 * 2 + 2
    w = mlp.init_weights(0)
    assert w.size == mlp.NW


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    w = mlp.init_weights(2) + rng.normal(0, 0.01, mlp.NW)
    X = rng.normal(0, 1, (13, 16))
    Y = rng.normal(0, 1, (13, 2))
    _, g = mlp.loss_and_grad(w, X, Y)
    idx = rng.choice(mlp.NW, 40, replace=False)
    for k in idx:
        e = np.zeros(mlp.NW)
        e[k] = 1e-6
        fd = (mlp.loss_and_grad(w + e, X, Y)[0] - mlp.loss_and_grad(w - e, X, Y)[0]) / 2e-6
        assert abs(fd - g[k]) < 1e-7 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_zero_weights_output_biases():
    w = np.zeros(mlp.NW)
    w[-2:] = [0.3, -0.2]
    out, _ = mlp.forward(w, np.ones((4, 16)))
    assert np.allclose(out, [[0.3, -0.2]] * 4)


def test_adam_first_step_moves_by_lr():
    w = np.zeros(3)
    g = np.array([1.0, -2.0, 0.5])
    m = np.zeros(3)
    v = np.zeros(3)
    mlp.adam_step(w, g, m, v, 1, 0.01)
    assert np.allclose(w, -0.01 * np.sign(g), atol=1e-9)


def test_targets_wrap():
    t = mlp.targets(np.array([-1.0]), np.array([-1e-9]), np.array([math.pi - 1e-3]), np.array([0.01]), 0.02)
    # atan2 is close to -pi, theta close to +pi: the wrapped difference is small
    assert abs(t[0, 0] * mlp.DELTA_SCALE) < 2e-3 and abs(t[0, 1] - 0.5) < 1e-12
