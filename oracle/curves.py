"""Boundary parametrisations q(theta) = (x(theta), y(theta)), 0 <= theta < 2 pi (eq. param).

Two families cover every domain used here:

* polar Fourier  r(t) = c0 + sum_m (a_m cos m t + b_m sin m t),  q = r (cos t, sin t)
  (unit disc, the five-petal star, random smooth perturbations of the circle);
* Cartesian Fourier x(t) = x0 + sum_m (ax_m cos m t + bx_m sin m t), likewise y
  (the kite x = cos t + A cos 2t - A, y = B sin t and the ellipse).

Curves are traversed counter-clockwise, so the outward unit normal of
Sec. 3.1 is n = (y', -x') / |q'| and the signed curvature
kappa = (x' y'' - y' x'') / |q'|^3 is positive where the domain is convex.

``eval_scalar`` uses Python's math module (the C library) and is what the
boundary grid uses; ``eval_vec`` is the numpy form used in iterations.
"""
from __future__ import annotations

import math

import numpy as np


class Curve:
    """kind: 'polar' with coef = [c0, a1, b1, a2, b2, ...];
    'cartesian' with coef = ([x0, ax1, bx1, ...], [y0, ay1, by1, ...])."""

    def __init__(self, kind, coef):
        self.kind = kind
        if kind == "polar":
            self.coef = [float(v) for v in coef]
        elif kind == "cartesian":
            self.coef = ([float(v) for v in coef[0]], [float(v) for v in coef[1]])
        else:
            raise ValueError(kind)

    # -- series helpers -------------------------------------------------
    @staticmethod
    def _series_scalar(c, t):
        """value, first and second derivative of c0 + sum (a_m cos mt + b_m sin mt)."""
        v = c[0]
        d1 = 0.0
        d2 = 0.0
        n = (len(c) - 1) // 2
        for m in range(1, n + 1):
            a = c[2 * m - 1]
            b = c[2 * m]
            cm = math.cos(m * t)
            sm = math.sin(m * t)
            v += a * cm + b * sm
            d1 += m * (b * cm - a * sm)
            d2 -= (m * m) * (a * cm + b * sm)
        return v, d1, d2

    @staticmethod
    def _series_vec(c, t):
        t = np.asarray(t, dtype=np.float64)
        v = np.full_like(t, c[0])
        d1 = np.zeros_like(t)
        d2 = np.zeros_like(t)
        n = (len(c) - 1) // 2
        for m in range(1, n + 1):
            a = c[2 * m - 1]
            b = c[2 * m]
            cm = np.cos(m * t)
            sm = np.sin(m * t)
            v = v + (a * cm + b * sm)
            d1 = d1 + m * (b * cm - a * sm)
            d2 = d2 - (m * m) * (a * cm + b * sm)
        return v, d1, d2

    # -- evaluation -----------------------------------------------------
    def eval_scalar(self, t):
        """(x, y, x', y', x'', y'') at a float t."""
        if self.kind == "polar":
            r, r1, r2 = self._series_scalar(self.coef, t)
            ct = math.cos(t)
            st = math.sin(t)
            x = r * ct
            y = r * st
            x1 = r1 * ct - r * st
            y1 = r1 * st + r * ct
            x2 = r2 * ct - 2.0 * r1 * st - r * ct
            y2 = r2 * st + 2.0 * r1 * ct - r * st
            return x, y, x1, y1, x2, y2
        x, x1, x2 = self._series_scalar(self.coef[0], t)
        y, y1, y2 = self._series_scalar(self.coef[1], t)
        return x, y, x1, y1, x2, y2

    def eval_vec(self, t):
        if self.kind == "polar":
            r, r1, r2 = self._series_vec(self.coef, t)
            ct = np.cos(t)
            st = np.sin(t)
            return (r * ct, r * st, r1 * ct - r * st, r1 * st + r * ct,
                    r2 * ct - 2.0 * r1 * st - r * ct, r2 * st + 2.0 * r1 * ct - r * st)
        x, x1, x2 = self._series_vec(self.coef[0], t)
        y, y1, y2 = self._series_vec(self.coef[1], t)
        return x, y, x1, y1, x2, y2

    def curvature_vec(self, t):
        x, y, x1, y1, x2, y2 = self.eval_vec(t)
        return (x1 * y2 - y1 * x2) / (x1 * x1 + y1 * y1) ** 1.5


def boundary_grid(curve, B):
    """theta_p = p k2, k2 = 2 pi / B (eq. bdry_grid); q_p, q'_p, q''_p and the outward normal n_p."""
    k2 = 2.0 * math.pi / B
    out = np.zeros((B, 9))
    for p in range(B):
        t = p * k2
        x, y, x1, y1, x2, y2 = curve.eval_scalar(t)
        sp = math.sqrt(x1 * x1 + y1 * y1)
        out[p] = (t, x, y, x1, y1, x2, y2, y1 / sp, -x1 / sp)
    return {
        "k2": k2, "theta": out[:, 0], "x": out[:, 1], "y": out[:, 2],
        "x1": out[:, 3], "y1": out[:, 4], "x2": out[:, 5], "y2": out[:, 6],
        "nx": out[:, 7], "ny": out[:, 8],
    }


def reach(curve, nsamp):
    """(exterior reach, interior reach) from curvature on a dense parameter grid:
    the smallest radius of curvature over concave (kappa < 0) and convex points."""
    t = np.arange(nsamp) * (2.0 * np.pi / nsamp)
    k = curve.curvature_vec(t)
    neg = k[k < 0]
    pos = k[k > 0]
    r_ext = float(1.0 / np.max(-neg)) if neg.size else math.inf
    r_int = float(1.0 / np.max(pos)) if pos.size else math.inf
    return r_ext, r_int
