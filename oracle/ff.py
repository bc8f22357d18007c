"""Fourier-Forwarding time step on the extended grid (oracle side), Sec. 4.2.

One large step of the auxiliary solution U_FC (eq. aux_sol): extend u and u_t
(2D-FC), transform, advance every mode by the closed-form solution of
eq. wave_2d_ff_modal over dt (``spectral.ff_propagate``), transform back on
the whole box.  The near-boundary solver U_B of the paper is out of scope; the
boundary data of the next step are the values of the new full-box field at the
plan's boundary points, by degree-(M-1) tensor-product Lagrange interpolation
on the centred M x M block of grid nodes around each point (reading of the
paper for steps j > 0, where it takes them from U_B).
"""
import numpy as np

from . import extend as E
from . import spectral as S
from .interp import lagrange_weights
from .plan import boundary_points


def boundary_interp(u, grid, pts, M):
    """Values of the grid field u [nx, ny] at points pts [n, 2]."""
    x = (pts[:, 0] - grid.x0) / grid.h
    y = (pts[:, 1] - grid.y0) / grid.h
    i0 = np.floor(x).astype(np.int64) - M // 2 + 1
    j0 = np.floor(y).astype(np.int64) - M // 2 + 1
    a = np.arange(M)
    xi = i0[:, None] + a[None, :]
    yj = j0[:, None] + a[None, :]
    wx = lagrange_weights((grid.x0 + xi * grid.h).astype(np.float64), pts[:, 0])
    wy = lagrange_weights((grid.y0 + yj * grid.h).astype(np.float64), pts[:, 1])
    vals = u[xi[:, :, None] % grid.nx, yj[:, None, :] % grid.ny]       # [n, M, M]
    return np.einsum("na,nab,nb->n", wx, vals, wy)


def ff_step(pl, u, ut, dt, c=1.0):
    """(u, u_t) on the full box -> (u, u_t) after one step dt."""
    g = pl.grid
    bp = boundary_points(pl)
    bu = boundary_interp(u, g, bp, pl.M)
    bt = boundary_interp(ut, g, bp, pl.M)
    U = S.fft2_forward(E.extend(pl, u, bu))
    Ut = S.fft2_forward(E.extend(pl, ut, bt))
    a, at = S.ff_propagate(U, Ut, g.nx, g.ny, g.h, c, dt)
    return S.fft2_inverse(a, g.ny), S.fft2_inverse(at, g.ny)
