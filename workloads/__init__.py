"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no part of the 2D-FC method: it only names domains (curve
coefficients), boxes and grids, closed-form test functions and seeded random
parameters.  Both the oracle and the HIP path evaluate curves, feet, stencils
and extensions on their own.

Domains (counter-clockwise parametrisations, theta in [0, 2 pi)):
  disc        r = 1
  star5       r = 1 + 0.3 cos 5t
  kite(A, B)  x = cos t + A cos 2t - A, y = B sin t   (A, B) = (0.65, 1.5) or the
              paper's (0.35, 0.7)
  ellipse     x = a cos t, y = b sin t with a = 1, b = 0.5
  random      r = 1 + sum_{m=2..8} a_m cos(m t + phi_m), |a_m| <= 0.15/m
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# --------------------------------------------------------------------------
# domains: ('polar', [c0, a1, b1, ...]) or ('cartesian', ([x...], [y...]))
# --------------------------------------------------------------------------


def disc():
    return ("polar", [1.0])


def star5(eps=0.3):
    c = [1.0] + [0.0] * 10
    c[2 * 5 - 1] = eps
    return ("polar", c)


def kite(A=0.65, B=1.5):
    return ("cartesian", ([-A, 1.0, 0.0, A, 0.0], [0.0, 0.0, B]))


def ellipse(a=1.0, b=0.5):
    return ("cartesian", ([0.0, a, 0.0], [0.0, 0.0, b]))


def random_polar(seed, mmin=2, mmax=8, amp=0.15):
    """r(t) = 1 + sum_m a_m cos(m t + phi_m), a_m ~ U[-amp/m, amp/m], phi_m ~ U[0, 2pi)."""
    rng = np.random.default_rng(seed)
    a = np.array([rng.uniform(-amp / m, amp / m) for m in range(mmin, mmax + 1)])
    ph = np.array([rng.uniform(0.0, 2 * math.pi) for _ in range(mmin, mmax + 1)])
    c = [1.0] + [0.0] * (2 * mmax)
    for k, m in enumerate(range(mmin, mmax + 1)):
        # a cos(mt + phi) = a cos(phi) cos(mt) - a sin(phi) sin(mt)
        c[2 * m - 1] = a[k] * math.cos(ph[k])
        c[2 * m] = -a[k] * math.sin(ph[k])
    return ("polar", c), a, ph


def _xy(curve, t):
    kind, c = curve
    if kind == "polar":
        r = np.full_like(t, c[0])
        for m in range(1, (len(c) - 1) // 2 + 1):
            r = r + c[2 * m - 1] * np.cos(m * t) + c[2 * m] * np.sin(m * t)
        return r * np.cos(t), r * np.sin(t)
    cx, cy = c
    x = np.full_like(t, cx[0])
    y = np.full_like(t, cy[0])
    for m in range(1, (len(cx) - 1) // 2 + 1):
        x = x + cx[2 * m - 1] * np.cos(m * t) + cx[2 * m] * np.sin(m * t)
    for m in range(1, (len(cy) - 1) // 2 + 1):
        y = y + cy[2 * m - 1] * np.cos(m * t) + cy[2 * m] * np.sin(m * t)
    return x, y


def bbox(curve, n=200000):
    t = np.arange(n) * (2 * math.pi / n)
    x, y = _xy(curve, t)
    return float(x.min()), float(x.max()), float(y.min()), float(y.max())


def inside_mask(curve, X, Y, n=20000):
    """Point-in-domain test by crossing parity (used only to place Gaussian pulses)."""
    t = np.arange(n) * (2 * math.pi / n)
    px, py = _xy(curve, t)
    qx, qy = np.roll(px, -1), np.roll(py, -1)
    X = np.asarray(X)[..., None]
    Y = np.asarray(Y)[..., None]
    cond = ((py <= Y) & (qy > Y)) | ((qy <= Y) & (py > Y))
    xc = px + (Y - py) * (qx - px) / np.where(qy != py, qy - py, 1.0)
    return (np.sum(cond & (xc > X), axis=-1) % 2) == 1


# --------------------------------------------------------------------------
# grids
# --------------------------------------------------------------------------
@dataclass
class Case:
    name: str
    curve: tuple
    x0: float
    y0: float
    h: float
    n: int
    B: int
    k1: float
    d: int = 5
    C: int = 27
    M: int = 8
    extra: dict = field(default_factory=dict)


def box_case(name, curve, lo, hi, n, B, k1=None, **kw):
    h = (hi - lo) / n
    return Case(name, curve, lo, lo, h, n, B, h if k1 is None else k1, **kw)


def fitted_case(name, curve, n, B=None, k1=None, C=27, **kw):
    """Square box around the domain: side n h with h = D / (n - 2C - 4), D the
    larger extent of the domain, centred on its bounding box; B = the power of
    two nearest 2 pi / h when not given."""
    xmin, xmax, ymin, ymax = bbox(curve)
    D = max(xmax - xmin, ymax - ymin)
    h = D / (n - 2 * C - 4)
    cx, cy = 0.5 * (xmin + xmax), 0.5 * (ymin + ymax)
    x0 = cx - 0.5 * n * h
    y0 = cy - 0.5 * n * h
    if B is None:
        B = 2 ** int(round(math.log2(2 * math.pi / h)))
    return Case(name, curve, x0, y0, h, n, B, h if k1 is None else k1, C=C, **kw)


STAR_K1 = 0.0024  # 0.9 x exterior reach of the star (0.0721) / C, rounded down


def cfg_disc128():
    """Unit disc, B = 256, box [-1.5, 1.5]^2 on 128^2, blend width 0.2 (k1 = 0.2/27)."""
    return box_case("disc128", disc(), -1.5, 1.5, 128, 256, k1=0.2 / 27)


def cfg_disc(n=256):
    """Unit disc, B = 2n, box [-1.6, 1.6]^2 on n^2, k1 = h."""
    return box_case("disc%d" % n, disc(), -1.6, 1.6, n, 2 * n)


def cfg_star(n=1024):
    """Star r = 1 + 0.3 cos 5t, B = 2n, box [-1.6, 1.6]^2 on n^2."""
    h = 3.2 / n
    return box_case("star%d" % n, star5(), -1.6, 1.6, n, 2 * n, k1=min(h, STAR_K1))


FF_DOMAINS = {"disc": disc, "star5": star5, "kite": lambda: kite(0.65, 1.5), "ellipse": ellipse}


def cfg_ff(domain, n):
    """Batched Fourier-Forwarding workload: one common box [-2, 2]^2 for every
    domain (so fields of one grid size share transform sizes and wavenumbers),
    B = 2n, k1 = h except the star (k1 = min(h, 0.0024))."""
    h = 4.0 / n
    k1 = min(h, STAR_K1) if domain == "star5" else h
    return box_case("%s%d" % (domain, n), FF_DOMAINS[domain](), -2.0, 2.0, n, 2 * n, k1=k1)


def cfg_kite(n=2048):
    return fitted_case("kite%d" % n, kite(0.65, 1.5), n)


def mlp_k1():
    """Normal step of the learned-seed workload: h of the fitted 4096^2 box
    around the held-out random curve (seed 1)."""
    return fitted_case("rnd4096", random_polar(1)[0], 4096).h


def cfg_mlp(n=4096):
    """Held-out random curve (seed 1) in its fitted box on n^2 points, with the
    normal step of the 4096^2 box at every n (so the strip width C k1 the
    network was trained for is the same) and B = 8192 at n = 4096, B = 2n below."""
    curve = random_polar(1)[0]
    return fitted_case("rnd%d" % n, curve, n, B=8192 if n >= 4096 else 2 * n, k1=mlp_k1())


def random_polar_batch(seed, ncurves, mmin=2, mmax=8, amp=0.15):
    """ncurves curves of the random_polar family from one generator -> [ncurves, 1 + 2 mmax]."""
    rng = np.random.default_rng(seed)
    out = np.zeros((ncurves, 1 + 2 * mmax))
    out[:, 0] = 1.0
    for c in range(ncurves):
        a = np.array([rng.uniform(-amp / m, amp / m) for m in range(mmin, mmax + 1)])
        ph = rng.uniform(0.0, 2 * math.pi, mmax - mmin + 1)
        for k, m in enumerate(range(mmin, mmax + 1)):
            out[c, 2 * m - 1] = a[k] * math.cos(ph[k])
            out[c, 2 * m] = -a[k] * math.sin(ph[k])
    return out


def mlp_training_draws(seed=0, ncurves=1000, npts=1000, width=1.0):
    """Training set of the learned foot seed: ncurves random curves and, per
    curve, npts parameters theta ~ U[0, 2 pi) and distances eta ~ U(0, width]
    (the point is placed at q(theta) + eta n(theta) by the consumer).
    Returns (curves [ncurves, 17], curve index [n] int32, theta [n], eta [n])."""
    curves = random_polar_batch(seed, ncurves)
    rng = np.random.default_rng(seed + 1000)
    cidx = np.repeat(np.arange(ncurves, dtype=np.int32), npts)
    theta = rng.uniform(0.0, 2 * math.pi, cidx.size)
    eta = width * (1.0 - rng.uniform(0.0, 1.0, cidx.size))
    return curves, cidx, theta, eta


# --------------------------------------------------------------------------
# test functions (closed forms) and seeded parameters
# --------------------------------------------------------------------------
def f_cfg1(x, y):
    return np.exp(np.sin(3 * x) + np.cos(2 * y))


def star_wavenumbers(seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(1.0, 20.0), rng.uniform(1.0, 20.0)


def f_star(seed):
    k1, k2 = star_wavenumbers(seed)
    return lambda x, y: np.sin(k1 * x) * np.cos(k2 * y) + x ** 3 * y


def f_paper_disc(x, y):
    """Example 3.1: -sin(5 pi x) sin(5 pi y)."""
    return -np.sin(5 * np.pi * x) * np.sin(5 * np.pi * y)


def f_paper_kite(x, y):
    """Example 3.2: -(x^6 + y^6) sin(10 pi x) sin(10 pi y)."""
    return -(x ** 6 + y ** 6) * np.sin(10 * np.pi * x) * np.sin(10 * np.pi * y)


def poisson_rhs(seed=0, nmodes=32, Lf=4.0):
    """Smooth random Fourier series: Re sum c_pq max(1,|kappa|)^-4 exp(i kappa.x),
    kappa = 2 pi (p, q)/Lf, p, q in [-16, 15], c = (g1 + i g2)/sqrt 2."""
    rng = np.random.default_rng(seed)
    p = np.arange(-nmodes // 2, nmodes // 2)
    g = (rng.standard_normal((nmodes, nmodes)) + 1j * rng.standard_normal((nmodes, nmodes))) / math.sqrt(2)
    kx = 2 * math.pi * p / Lf
    K = np.sqrt(kx[:, None] ** 2 + kx[None, :] ** 2)
    c = g * np.maximum(1.0, K) ** -4

    def f(x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        ex = np.exp(1j * np.multiply.outer(x, kx))      # [..., P]
        ey = np.exp(1j * np.multiply.outer(y, kx))      # [..., Q]
        return np.real(np.einsum("...p,pq,...q->...", ex, c, ey))

    def on_grid(xs, ys):
        """f on the tensor grid xs x ys (same values, separable evaluation)."""
        ex = np.exp(1j * np.multiply.outer(np.asarray(xs, dtype=np.float64), kx))
        ey = np.exp(1j * np.multiply.outer(np.asarray(ys, dtype=np.float64), kx))
        return np.real(ex @ c @ ey.T)
    f.on_grid = on_grid
    return f


def gaussian_pulse(curve, seed, sigma_range=(0.05, 0.15)):
    """u0 = exp(-|x - xc|^2 / sigma^2) with xc uniform in the domain at distance >= 3 sigma from Gamma."""
    rng = np.random.default_rng(seed)
    sigma = rng.uniform(*sigma_range)
    xmin, xmax, ymin, ymax = bbox(curve, 20000)
    t = np.arange(20000) * (2 * math.pi / 20000)
    px, py = _xy(curve, t)
    while True:
        xc, yc = rng.uniform(xmin, xmax), rng.uniform(ymin, ymax)
        if inside_mask(curve, xc, yc) and np.min(np.hypot(px - xc, py - yc)) >= 3 * sigma:
            break
    return (lambda x, y: np.exp(-((x - xc) ** 2 + (y - yc) ** 2) / sigma ** 2)), (xc, yc, sigma)


def grid_values(case, f):
    i = np.arange(case.n)
    x = case.x0 + i * case.h
    y = case.y0 + i * case.h
    if hasattr(f, "on_grid"):
        return f.on_grid(x, y)
    X, Y = np.meshgrid(x, y, indexing="ij")
    return f(X, Y)
