"""Pins for the oracle's Fourier-Forwarding step (Sec. 4.2): tensor
interpolation of boundary data is exact on polynomials, and one step of the
paper's manufactured plane wave (Ex. 4.4) is accurate away from the boundary
(the domain of dependence Omega_dT of eq. ff_soln)."""
import numpy as np
import pytest

import workloads as W
from oracle import fcgram
from oracle import ff as OF
from oracle import plan as P
from oracle.curves import Curve


def test_boundary_interp_exact_on_tensor_polynomials():
    g = P.Grid(-1.0, -1.0, 0.05, 40, 40)
    x = g.xs()
    X, Y = np.meshgrid(x, g.ys(), indexing="ij")
    f = lambda x, y: (1 + x - x ** 7) * (0.5 - y ** 3 + 0.1 * y ** 7)
    pts = np.random.default_rng(0).uniform(-0.7, 0.7, (50, 2))
    v = OF.boundary_interp(f(X, Y), g, pts, 8)
    assert np.abs(v - f(pts[:, 0], pts[:, 1])).max() < 1e-12


def test_boundary_interp_degree_is_not_higher():
    # a degree-8 term is not reproduced exactly: the stencil really has 8 nodes
    g = P.Grid(-1.0, -1.0, 0.05, 40, 40)
    X, Y = np.meshgrid(g.xs(), g.ys(), indexing="ij")
    pts = np.array([[0.013, 0.021]])
    v = OF.boundary_interp(X ** 8, g, pts, 8)
    assert abs(v[0] - 0.013 ** 8) > 1e-12


@pytest.mark.slow
def test_plane_wave_step_disc():
    """u = cos(2k(x+t)/3) + cos(k(y+t)) solves the free-space wave equation; one
    FF step of dt from t = 0 matches it at points deeper than c dt + margin."""
    case = W.cfg_disc(256)
    tab = fcgram.load_tables(5)
    g = P.Grid(case.x0, case.y0, case.h, case.n, case.n)
    pl = P.make_plan(Curve(*case.curve), g, tab, case.B, k1=case.k1, M=case.M)
    k = 6.0
    u = lambda x, y, t: np.cos(2 * k * (x + t) / 3) + np.cos(k * (y + t))
    ut = lambda x, y, t: -2 * k / 3 * np.sin(2 * k * (x + t) / 3) - k * np.sin(k * (y + t))
    X, Y = np.meshgrid(g.xs(), g.ys(), indexing="ij")
    dt = 0.05
    u1, ut1 = OF.ff_step(pl, u(X, Y, 0), ut(X, Y, 0), dt)
    deep = np.hypot(X, Y) < 1.0 - dt - 0.05
    assert np.abs(u1 - u(X, Y, dt))[deep].max() < 1e-6
    assert np.abs(ut1 - ut(X, Y, dt))[deep].max() < 1e-5
