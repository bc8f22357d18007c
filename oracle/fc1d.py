"""One-dimensional FC of Sec. 2.3 (oracle side; used to pin the tables).

Given phi on x_j = j k, j = 0..N-1, k = 1/(N-1): the rightward blend
phi_r^r = A Q^T phi_r of the last d values, the leftward blend
phi_l^l = R^C A Q^T R^d phi_l of the first d values, the continuation vector
phi^c = (phi_0..phi_{N-1}, phi_l^l + phi_r^r) of length N + C (eq. fc_1d_cont),
and its FFT gives the trigonometric polynomial of eq. fc_1d_srs with period
b = (N + C) k.
"""
import numpy as np


def fc1d_continuation(phi, Q, A):
    d = Q.shape[0]
    right = A @ (Q.T @ phi[-d:])
    left = (A @ (Q.T @ phi[:d][::-1]))[::-1]
    return np.concatenate([phi, left + right])


def fc1d_eval(phi, Q, A, x_eval):
    """Evaluate the 1D-FC trigonometric polynomial of phi at x_eval in [0, 1]."""
    n = phi.size
    k = 1.0 / (n - 1)
    pc = fc1d_continuation(phi, Q, A)
    L = pc.size
    c = np.fft.fft(pc) / L
    freqs = np.fft.fftfreq(L, d=1.0 / L)
    if L % 2 == 0:
        # split the Nyquist term symmetrically so the interpolant is real
        freqs = freqs.copy()
    b = L * k
    E = np.exp(2j * np.pi * np.outer(x_eval, freqs) / b)
    vals = E @ c
    if L % 2 == 0:
        ny = L // 2
        vals = vals - c[ny] * E[:, ny] + c[ny] * np.cos(2 * np.pi * ny * x_eval / b)
    return np.real(vals)
