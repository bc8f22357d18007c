"""Cartesian Evaluation of 2D-FC (oracle side): Sec. 3.5 steps 5-6.

* ``matching_values``: f_{D_p} on the d matching points of every normal
  (Sec. 3.2, two-step degree-(M-1) interpolation; the point on Gamma takes the
  boundary sample, or with a plan built from interior data only (Remark 3.1 II)
  the same interpolation at depth 0).  Evaluated in numpy.longdouble: the continuation below
  amplifies a relative perturbation of f_D by |A_r Q^T| ~ 1e4, so f_D and
  Q^T f_D are carried with more than float64 precision and rounded once.
* ``blend``: blending to zero along each normal on the refined grid,
  c_p = Q^T f_{D_p} and F[l, p] = (A_r c_p)_{l-1}, l = 1..C_r, with
  F[0, p] = f_{D_p}[d-1] (eq. b_to_z, Remark 2.2, eq. vnbj_p: level l of
  V+_{B,C_r} sits at distance l k1/n_r from Gamma, the 1D coordinate
  (d-1) + l/n_r of the refined continuation points).
* ``strip_values``: interpolation onto H n V+ (Sec. 3.4, Fig. 4): along each
  of the M normals of S_{theta^Q} a degree-(M-1) interpolation in the level
  variable at distance eta_Q ("blue asterisks"), then a degree-(M-1)
  interpolation in theta over S_{theta^Q}.
* ``assemble``: IN points keep f, STRIP points take the interpolated values,
  FAR points are 0 (the continuation vanishes beyond V+).
"""
from __future__ import annotations

import numpy as np

from .interp import lagrange_weights
from .plan import FAR, IN, STRIP, stencil_offsets

LD = np.longdouble


def matching_values(pl, f_grid, f_bdry):
    """f_D [B, d] (longdouble) from grid values and boundary samples.

    f_grid: [nx, ny] float64 (only IN entries are read); f_bdry: boundary
    samples in the order of ``plan.boundary_points`` (B feet, then squares).
    """
    B, M, d = pl.B, pl.M, pl.d
    fg = np.asarray(f_grid, dtype=np.float64).ravel()
    ref = pl.match_ref
    if getattr(pl, "interior_only", False):   # no boundary samples are read (f_bdry may be None)
        assert np.all(ref >= 0)
        vals = fg[ref]
    else:
        fb = np.asarray(f_bdry, dtype=np.float64)
        vals = np.where(ref >= 0, fg[np.clip(ref, 0, None)], fb[B + np.clip(-ref - 1, 0, None)])
    if np.any(ref >= 0):
        assert np.all(pl.cls.ravel()[ref[ref >= 0]] == IN)
    stars = np.sum(pl.match_wv * vals.astype(LD), axis=2)                 # [B, M]
    fD = np.zeros((B, d), dtype=LD)
    if getattr(pl, "interior_only", False):
        fD[:, :] = np.sum(pl.match_wn * stars[:, None, :], axis=2)         # [B, d], Remark 3.1 II
    else:
        stars[:, M - 1] = fb[:B].astype(LD)                                # the point on Gamma
        fD[:, : d - 1] = np.sum(pl.match_wn * stars[:, None, :], axis=2)    # [B, d-1]
        fD[:, d - 1] = fb[:B].astype(LD)
    return fD


def gram_coefficients(pl, fD):
    """c_p = Q^T f_{D_p} in longdouble, rounded to float64 once.  [B, d]"""
    return (fD @ pl.Q.astype(LD)).astype(np.float64)


def blend(pl, fD):
    """Continuation values on V+_{B,C_r}: F [C_r + 1, B] (float64)."""
    c = gram_coefficients(pl, fD)
    F = np.zeros((pl.Cr + 1, pl.B))
    F[0] = fD[:, pl.d - 1].astype(np.float64)
    F[1:] = pl.Ar @ c.T
    return F


def strip_values(pl, F):
    """Interpolated continuation values at the STRIP points (row-major order)."""
    M, B, Cr = pl.M, pl.B, pl.Cr
    th = pl.strip_theta
    eta = pl.strip_eta
    k2 = pl.k2
    off = stencil_offsets(M)
    if M % 2 == 0:
        p0 = np.floor(th / k2).astype(np.int64)
    else:
        p0 = np.rint(th / k2).astype(np.int64)
    pj = p0[:, None] + off[None, :]                      # unwrapped normal indices
    w = lagrange_weights(pj * k2, th)                    # theta weights [S, M]
    s = eta * (pl.n_r / pl.k1)                           # level coordinate in (0, C_r]
    l0 = np.clip(np.floor(s).astype(np.int64) - M // 2 + 1, 0, Cr - M + 1)
    lev = l0[:, None] + np.arange(M)[None, :]
    v = lagrange_weights(lev.astype(np.float64), s)      # level weights [S, M]
    cols = pj % B
    # blue asterisks: G[S, j] = sum_l v_l F[l, p_j]
    G = np.zeros((th.size, M))
    for l in range(M):
        G += v[:, l, None] * F[lev[:, l, None], cols]
    return np.sum(w * G, axis=1)


def assemble(pl, f_grid, strip_vals):
    out = np.zeros(pl.grid.nx * pl.grid.ny)
    cls = pl.cls.ravel()
    fg = np.asarray(f_grid, dtype=np.float64).ravel()
    out[cls == IN] = fg[cls == IN]
    out[pl.strip_idx] = strip_vals
    return out.reshape(pl.grid.nx, pl.grid.ny)


def extend(pl, f_grid, f_bdry):
    """The 2D-FC extension f^c on H (before the FFT)."""
    fD = matching_values(pl, f_grid, f_bdry)
    F = blend(pl, fD)
    return assemble(pl, f_grid, strip_values(pl, F))
