"""Full 2D-FC Poisson solver of Sec. 4.1 (oracle side).

TEST INFRASTRUCTURE ONLY: the float64 reference the library's Poisson entry
point is checked against.  It solves
    Delta u = f in Omega,  u = g on Gamma                       (eq. def_poisson)
as u = u_p + v (eq. total_soln):

* u_p, the 2D-FC particular solution on the whole periodic box (eq. poisson_ps):
  the extension's Fourier coefficients divided by -|k|^2 (eq. poisson_ps_coeffs,
  mode (0, 0) set to 0) plus the mean term f_00 (x^2 + y^2) / 4, f_00 the mean of
  the extension over the box.  (The printed formula carries a minus sign on this
  term; with it Delta u_p would be f - 2 f_00, so the sign is read as +.)
* g_hom = g - u_p on Gamma (eq. laplace_bc) at NB equispaced parameter nodes
  t_j = 2 pi j / NB, u_p there by tensor-product Lagrange interpolation of degree
  MP - 1 from the grid (the paper's iterated 1D interpolation).
* v, harmonic with v = g_hom on Gamma (eq. def_laplace), as the double-layer
  potential v(x) = int_Gamma phi(y) dPhi(x, y)/dnu(y) ds(y), Phi = -log|x - y|/(2 pi),
  nu the outward normal: the interior limit gives phi - 2 K phi = -2 g_hom, solved
  by the Nystrom method with the trapezoidal rule on the NB nodes (Kress, Linear
  Integral Equations, Sec. 12.2); the kernel on Gamma is smooth, with the limit
  -(x'y'' - y'x'') / (4 pi |q'|^2) on the diagonal.  The small dense system is
  solved directly here.
* v at grid points of Omega by the trapezoidal rule with the density carried to
  R NB nodes by its trigonometric interpolant (the Dirichlet kernel), R = 128:
  enough that the points h/2 inside Gamma, the closest the sums are taken at,
  lie several node spacings from the nodes even for NB = N on a tight box.  Points
  closer to Gamma than h/2 (foot of the normal of Sec. 3.4) take v at the foot
  (g_hom interpolated trigonometrically) and at MP - 1 points h/2, h, ... inward
  along the normal, interpolated in the distance with degree MP - 1: a reading
  of the paper's local refinement followed by interpolation of degree MP - 1.
"""
import math

import numpy as np

from . import extend as E
from . import spectral as S
from .ff import boundary_interp
from .interp import lagrange_weights
from .plan import IN, foot_solve

REFINE = 128   # density refinement factor R of the near-boundary sums


def particular_solution(pl, f_grid, f_bdry):
    """u_p on the whole box [nx, ny]."""
    g = pl.grid
    U = S.fft2_forward(E.extend(pl, f_grid, f_bdry))
    mean = U[0, 0].real / (g.nx * g.ny)
    up = S.fft2_inverse(S.laplace_inverse(U, g.nx, g.ny, g.h), g.ny)
    X, Y = np.meshgrid(g.xs(), g.ys(), indexing="ij")
    return up + mean * (X * X + Y * Y) / 4.0


def nodes(curve, n):
    """t_j = 2 pi j / n; points q(t_j), tangents q'(t_j), second derivatives."""
    t = 2.0 * math.pi * np.arange(n) / n
    x, y, x1, y1, x2, y2 = curve.eval_vec(t)
    return t, np.stack([x, y], 1), np.stack([x1, y1], 1), np.stack([x2, y2], 1)


def nystrom_matrix(curve, nb):
    """I - 2 K on the NB nodes (trapezoidal weights 2 pi / NB)."""
    t, q, q1, q2 = nodes(curve, nb)
    nu = np.stack([q1[:, 1], -q1[:, 0]], 1)            # outward normal times |q'|
    dx = q[:, None, :] - q[None, :, :]                  # x_i - y_j
    r2 = np.einsum("ijk,ijk->ij", dx, dx)
    num = np.einsum("ijk,jk->ij", dx, nu)
    np.fill_diagonal(r2, 1.0)
    K = num / r2 / (2.0 * math.pi)
    sp2 = q1[:, 0] ** 2 + q1[:, 1] ** 2
    np.fill_diagonal(K, -(q1[:, 0] * q2[:, 1] - q1[:, 1] * q2[:, 0]) / (4.0 * math.pi * sp2))
    return np.eye(nb) - 2.0 * K * (2.0 * math.pi / nb)


def density(curve, g_hom):
    """Double-layer density phi with interior limit g_hom at the nodes."""
    return np.linalg.solve(nystrom_matrix(curve, g_hom.size), -2.0 * g_hom)


def trig_interp(vals, tau):
    """Trigonometric interpolant of the periodic samples vals (nodes 2 pi j / n;
    for even n the Nyquist term split evenly) at parameters tau, through the
    Dirichlet kernel sin(n s / 2) / (n sin(s / 2)), times cos(s / 2) for even n."""
    n = vals.size
    t = 2.0 * math.pi * np.arange(n) / n
    tau = np.atleast_1d(np.asarray(tau, dtype=np.float64))
    out = np.empty(tau.shape)
    flat, res = tau.ravel(), out.ravel()
    step = max(1, (1 << 24) // n)          # rows per block (bounded memory)
    for a in range(0, flat.size, step):
        s = flat[a:a + step, None] - t
        half = 0.5 * s
        sn = np.sin(half)
        with np.errstate(divide="ignore", invalid="ignore"):
            w = np.sin(0.5 * n * s) * (np.cos(half) if n % 2 == 0 else 1.0) / (n * sn)
        hit = np.abs(sn) < 1e-300
        w = np.where(hit, 1.0, w)
        w = np.where(hit.any(-1, keepdims=True) & ~hit, 0.0, w)
        res[a:a + step] = w @ vals
    return out


def double_layer(curve, phi, pts):
    """Trapezoidal double-layer sum at points pts [n, 2] with the density given at its nodes."""
    n = phi.size
    _, q, q1, _ = nodes(curve, n)
    nu = np.stack([q1[:, 1], -q1[:, 0]], 1)
    out = np.empty(pts.shape[0])
    step = max(1, (1 << 23) // n)          # points per block (bounded memory)
    for a in range(0, pts.shape[0], step):
        dx = pts[a:a + step, None, :] - q[None, :, :]
        r2 = np.einsum("ijk,ijk->ij", dx, dx)
        num = np.einsum("ijk,jk->ij", dx, nu)
        out[a:a + step] = (num / r2) @ phi / n          # (1 / 2 pi) x (2 pi / n)
    return out


def solve(pl, f_grid, f_bdry, g_nodes, nb, MP=None, sample=None):
    """u on the IN points of the plan's grid (other points 0).  g_nodes: g at
    the nb nodes q(2 pi j / nb).  With ``sample`` (flat grid indices of IN
    points) only those points are evaluated and their values returned."""
    MP = pl.M if MP is None else MP
    grid, curve = pl.grid, pl.curve
    up = particular_solution(pl, f_grid, f_bdry)
    t, q, q1, _ = nodes(curve, nb)
    g_hom = g_nodes - boundary_interp(up, grid, q, MP)
    phi = density(curve, g_hom)
    phif = trig_interp(phi, 2.0 * math.pi * np.arange(REFINE * nb) / (REFINE * nb))
    X, Y = np.meshgrid(grid.xs(), grid.ys(), indexing="ij")
    if sample is None:
        ins = np.argwhere(pl.cls == IN)
    else:
        sample = np.asarray(sample)
        assert np.all(pl.cls.ravel()[sample] == IN)
        ins = np.stack(np.unravel_index(sample, pl.cls.shape), 1)
    P = np.stack([X[ins[:, 0], ins[:, 1]], Y[ins[:, 0], ins[:, 1]]], 1)
    v = double_layer(curve, phif, P)
    # points within h/2 of Gamma: along the normal from the foot
    bd = pl.bd
    bq = np.stack([bd["x"], bd["y"]], 1)
    near, dnear = [], []
    for a in range(0, P.shape[0], 4096):
        d2 = ((P[a:a + 4096, None, :] - bq[None, :, :]) ** 2).sum(-1)
        near.append(np.argmin(d2, 1))
        dnear.append(np.sqrt(d2.min(1)))
    seed = np.concatenate(near)
    dnear = np.concatenate(dnear)
    h = grid.h
    # only points that can lie within h/2 of Gamma take the foot of the normal (a
    # point's nearest boundary sample is at most half a sample spacing farther than
    # its foot); far inside, e.g. at a disc's centre, the foot is not defined
    spacing = bd["k2"] * float(np.hypot(bd["x1"], bd["y1"]).max())
    cand = np.nonzero(dnear <= 0.5 * h + spacing)[0]
    th = np.zeros(P.shape[0])
    eta = np.full(P.shape[0], np.inf)
    th[cand], eta[cand], _ = foot_solve(curve, bd, P[cand, 0], P[cand, 1], seed[cand], pl.M)
    sel = np.nonzero(np.abs(eta) < 0.5 * h)[0]
    if sel.size:
        x, y, x1, y1, _, _ = curve.eval_vec(th[sel])
        sp = np.hypot(x1, y1)
        inward = np.stack([-y1 / sp, x1 / sp], 1)
        s_nodes = 0.5 * h * np.arange(MP)
        vals = np.empty((sel.size, MP))
        vals[:, 0] = trig_interp(g_hom, th[sel])
        for m in range(1, MP):
            pts = np.stack([x, y], 1) + s_nodes[m] * inward
            vals[:, m] = double_layer(curve, phif, pts)
        w = lagrange_weights(np.broadcast_to(s_nodes, (sel.size, MP)).copy(), -eta[sel])
        v[sel] = (w * vals).sum(1)
    if sample is not None:
        return up[ins[:, 0], ins[:, 1]] + v
    u = np.zeros_like(up)
    u[ins[:, 0], ins[:, 1]] = up[ins[:, 0], ins[:, 1]] + v
    return u
