"""Spectral stage and consumers (oracle side).

* ``fft2_forward`` / ``fft2_inverse``: the 2D FFT of Sec. 3.5 step 7 in the
  real-to-half-complex convention (forward unnormalised over axes (i, j), the
  half spectrum along j; inverse carries 1/(N_x N_y)).  The Fourier
  coefficients of eq. fc_2d_srs are the forward DFT divided by N_x N_y, with
  l in (-N_x/2, N_x/2] and m in [0, N_y/2] (Hermitian half).
* ``laplace_inverse``: the particular solution of eq. poisson_ps_coeffs:
  b_lm = -f_lm / ((2 pi l/L_x)^2 + (2 pi m/L_y)^2), b_00 = 0.
* ``derivative``: multiplication by i 2 pi l / L_x (x) or i 2 pi m / L_y (y),
  with the Nyquist mode zeroed.
* ``ff_propagate``: exact modal solution of eq. wave_2d_ff_modal,
  a(t) = cos(w t) f + sin(w t)/w g and a_t(t) = -w sin(w t) f + cos(w t) g with
  w = 2 pi c |(l/L_x, m/L_y)| (the square root of alpha_lm of the paper),
  and a(t) = f + t g, a_t = g for the zero mode (eq. wave_2d_ff).
* ``upsample_h2``: values on the h/2 grid by zero-padding the spectrum (the
  error measurement of Sec. 3.6).
"""
from __future__ import annotations

import numpy as np


def fft2_forward(u):
    return np.fft.rfft2(u)


def fft2_inverse(U, ny):
    return np.fft.irfft2(U, s=(U.shape[-2], ny))


def wavenumbers(nx, ny, h):
    """Integer mode indices (l, m) of the half spectrum [nx, ny//2+1]."""
    l = np.fft.fftfreq(nx, d=1.0 / nx)
    m = np.arange(ny // 2 + 1, dtype=np.float64)
    return l, m


def _abs_k2(nx, ny, h):
    Lx, Ly = nx * h, ny * h
    l, m = wavenumbers(nx, ny, h)
    # Nyquist index of the full range (-N/2, N/2] is +N/2
    l = np.where(l == -nx / 2, nx / 2, l)
    kx = 2 * np.pi * l / Lx
    ky = 2 * np.pi * m / Ly
    return kx[:, None] ** 2 + ky[None, :] ** 2, kx, ky


def laplace_inverse(U, nx, ny, h):
    k2, _, _ = _abs_k2(nx, ny, h)
    out = np.zeros_like(U)
    nz = k2 > 0
    out[nz] = -U[nz] / k2[nz]
    return out


def derivative(U, nx, ny, h, axis):
    _, kx, ky = _abs_k2(nx, ny, h)
    if axis == 0:
        k = kx.copy()
        if nx % 2 == 0:
            k[nx // 2] = 0.0
        return U * (1j * k)[:, None]
    k = ky.copy()
    if ny % 2 == 0:
        k[ny // 2] = 0.0
    return U * (1j * k)[None, :]


def ff_propagate(U0, U1, nx, ny, h, c, t):
    Lx, Ly = nx * h, ny * h
    l, m = wavenumbers(nx, ny, h)
    l = np.where(l == -nx / 2, nx / 2, l)
    w = 2 * np.pi * c * np.sqrt((l[:, None] / Lx) ** 2 + (m[None, :] / Ly) ** 2)
    cw = np.cos(w * t)
    sw = np.sin(w * t)
    with np.errstate(divide="ignore", invalid="ignore"):
        sinc = np.where(w > 0, sw / w, t)
    a = cw * U0 + sinc * U1
    at = -w * sw * U0 + cw * U1
    a[0, 0] = U0[0, 0] + t * U1[0, 0]
    at[0, 0] = U1[0, 0]
    return a, at


def upsample_h2(u):
    """Trigonometric interpolant of u on the grid of half the step (2N x 2N)."""
    nx, ny = u.shape
    U = np.fft.fft2(u)
    P = np.zeros((2 * nx, 2 * ny), dtype=complex)
    hx, hy = nx // 2, ny // 2
    # split the Nyquist rows/columns symmetrically
    idx_x = np.r_[0:hx, 2 * nx - hx:2 * nx]
    src_x = np.r_[0:hx, nx - hx:nx]
    idx_y = np.r_[0:hy, 2 * ny - hy:2 * ny]
    src_y = np.r_[0:hy, ny - hy:ny]
    P[np.ix_(idx_x, idx_y)] = U[np.ix_(src_x, src_y)]
    # Nyquist halves
    P[hx, idx_y] += 0.5 * U[hx, src_y]
    P[2 * nx - hx, idx_y] += 0.5 * U[hx, src_y]
    P[idx_x, hy] += 0.5 * U[src_x, hy]
    P[idx_x, 2 * ny - hy] += 0.5 * U[src_x, hy]
    for a in (hx, 2 * nx - hx):
        for b in (hy, 2 * ny - hy):
            P[a, b] += 0.25 * U[hx, hy]
    return np.real(np.fft.ifft2(P)) * 4.0
