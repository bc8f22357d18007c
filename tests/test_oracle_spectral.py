"""Pins for the oracle's spectral stage and consumers (Secs. 3.5, 4.1, 4.2):
brute-force DFT, exact single-mode inversion and propagation, group property."""
import numpy as np
import pytest

from oracle import spectral as S


def _dft2(u):
    nx, ny = u.shape
    i = np.arange(nx)
    j = np.arange(ny)
    Ex = np.exp(-2j * np.pi * np.outer(i, i) / nx)
    Ey = np.exp(-2j * np.pi * np.outer(j, j) / ny)
    return (Ex @ u @ Ey)[:, : ny // 2 + 1]


@pytest.mark.parametrize("shape", [(8, 8), (16, 12), (32, 32), (6, 10)])
def test_forward_matches_brute_force_dft(shape):
    u = np.random.default_rng(3).standard_normal(shape)
    U = S.fft2_forward(u)
    ref = _dft2(u)
    assert np.abs(U - ref).max() < 1e-13 * np.abs(ref).max()
    assert np.allclose(S.fft2_inverse(U, shape[1]), u, atol=1e-14)


def _mode(nx, ny, h, l, m):
    x = np.arange(nx) * h
    y = np.arange(ny) * h
    X, Y = np.meshgrid(x, y, indexing="ij")
    return np.cos(2 * np.pi * (l * X / (nx * h) + m * Y / (ny * h)))


def test_laplace_inverse_single_mode():
    nx, ny, h = 32, 24, 0.1
    l, m = 3, 5
    f = _mode(nx, ny, h, l, m)
    u = S.fft2_inverse(S.laplace_inverse(S.fft2_forward(f), nx, ny, h), ny)
    k2 = (2 * np.pi * l / (nx * h)) ** 2 + (2 * np.pi * m / (ny * h)) ** 2
    assert np.allclose(u, -f / k2, atol=1e-14)


def test_laplace_inverse_round_trip():
    nx, ny, h = 16, 16, 0.2
    U = S.fft2_forward(np.random.default_rng(4).standard_normal((nx, ny)))
    B = S.laplace_inverse(U, nx, ny, h)
    k2, _, _ = S._abs_k2(nx, ny, h)
    back = -k2 * B
    back[0, 0] = U[0, 0]
    assert np.allclose(back, U, atol=1e-12)
    assert B[0, 0] == 0


def test_derivative_single_mode():
    nx, ny, h = 32, 16, 0.05
    f = _mode(nx, ny, h, 2, 3)
    x = np.arange(nx) * h
    y = np.arange(ny) * h
    X, Y = np.meshgrid(x, y, indexing="ij")
    arg = 2 * np.pi * (2 * X / (nx * h) + 3 * Y / (ny * h))
    dx = S.fft2_inverse(S.derivative(S.fft2_forward(f), nx, ny, h, 0), ny)
    dy = S.fft2_inverse(S.derivative(S.fft2_forward(f), nx, ny, h, 1), ny)
    assert np.allclose(dx, -np.sin(arg) * 2 * np.pi * 2 / (nx * h), atol=1e-12)
    assert np.allclose(dy, -np.sin(arg) * 2 * np.pi * 3 / (ny * h), atol=1e-12)


def test_ff_single_mode_closed_form():
    nx, ny, h, c, t = 32, 32, 0.1, 1.3, 0.7
    l, m = 4, -3
    f = _mode(nx, ny, h, l, m)
    w = 2 * np.pi * c * np.hypot(l / (nx * h), m / (ny * h))
    a, at = S.ff_propagate(S.fft2_forward(f), S.fft2_forward(0.5 * f), nx, ny, h, c, t)
    u = S.fft2_inverse(a, ny)
    ut = S.fft2_inverse(at, ny)
    assert np.allclose(u, (np.cos(w * t) + 0.5 * np.sin(w * t) / w) * f, atol=1e-13)
    assert np.allclose(ut, (-w * np.sin(w * t) + 0.5 * np.cos(w * t)) * f, atol=1e-12)


def test_ff_zero_mode_and_group_property():
    nx, ny, h = 16, 16, 0.1
    rng = np.random.default_rng(5)
    U0 = S.fft2_forward(rng.standard_normal((nx, ny)))
    U1 = S.fft2_forward(rng.standard_normal((nx, ny)))
    a, at = S.ff_propagate(U0, U1, nx, ny, h, 1.0, 0.3)
    assert np.isclose(a[0, 0], U0[0, 0] + 0.3 * U1[0, 0]) and at[0, 0] == U1[0, 0]
    b, bt = U0, U1
    for _ in range(100):
        b, bt = S.ff_propagate(b, bt, nx, ny, h, 1.0, 0.01)
    a1, at1 = S.ff_propagate(U0, U1, nx, ny, h, 1.0, 1.0)
    scale = np.abs(a1).max()
    assert np.abs(b - a1).max() < 1e-12 * scale and np.abs(bt - at1).max() < 1e-11 * np.abs(at1).max()


def test_plane_wave_is_free_space_solution():
    """The manufactured solution of Example 4.4, u = cos(2k(x+t)/3) + cos(k(y+t)),
    is propagated exactly when it is box-periodic."""
    nx = ny = 64
    L = 2 * np.pi * 3 / 2          # period of cos(2 k x / 3) with k = 1 ... times 1
    h = L / nx
    k = 3.0 * 2 * np.pi / L * 1.0  # makes 2k/3 and k integer multiples of 2 pi / L
    x = np.arange(nx) * h
    X, Y = np.meshgrid(x, x, indexing="ij")
    u = lambda t: np.cos(2 * k * (X + t) / 3) + np.cos(k * (Y + t))
    ut = lambda t: -2 * k / 3 * np.sin(2 * k * (X + t) / 3) - k * np.sin(k * (Y + t))
    a, at = S.ff_propagate(S.fft2_forward(u(0)), S.fft2_forward(ut(0)), nx, ny, h, 1.0, 0.8)
    assert np.allclose(S.fft2_inverse(a, ny), u(0.8), atol=1e-12)
    assert np.allclose(S.fft2_inverse(at, ny), ut(0.8), atol=1e-11)


def test_upsample_exact_for_band_limited():
    nx = ny = 16
    h = 0.25
    f = _mode(nx, ny, h, 3, 2) + 0.5 * _mode(nx, ny, h, 1, 5)
    up = S.upsample_h2(f)
    x2 = np.arange(2 * nx) * h / 2
    X, Y = np.meshgrid(x2, x2, indexing="ij")
    ex = np.cos(2 * np.pi * (3 * X + 2 * Y) / (nx * h)) + 0.5 * np.cos(2 * np.pi * (X + 5 * Y) / (nx * h))
    assert np.allclose(up, ex, atol=1e-13)
