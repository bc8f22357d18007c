"""Pins of the oracle's Fourier Forwarding solver (Sec. 4.2; oracle/ffsolve.py)
against what the mathematics fixes: the 1D-FC second derivative converges at
order d - 2 on the function of Fig. 1, the Lagrange second-derivative weights
are exact for polynomials, the boundary region covers every grid point within
c dT of Gamma, and the solver reproduces the manufactured plane-wave solution
of Ex. 4.4 (unit disc, Dirichlet data from the exact solution) with the error
of the large step's interior part at 2D-FC accuracy and the whole error
converging under refinement."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import fcgram
from oracle import ffsolve as FS
from oracle import plan as OP
from oracle.curves import Curve

KAPPA = 10.0


def ue(x, y, t):
    """Ex. 4.4's manufactured solution (c = 1)."""
    return np.cos(2 * KAPPA * (x + t) / 3) + np.cos(KAPPA * (y + t))


def ute(x, y, t):
    return -(2 * KAPPA / 3) * np.sin(2 * KAPPA * (x + t) / 3) - KAPPA * np.sin(KAPPA * (y + t))


def _plan(n, d=5):
    case = W.cfg_disc(n)
    g = OP.Grid(case.x0, case.y0, case.h, n, n)
    return OP.make_plan(Curve(*case.curve), g, fcgram.load_tables(d), case.B, k1=case.h, M=d + 3)


@pytest.fixture(scope="module")
def disc256():
    pl = _plan(256)
    return pl, FS.make_setup(pl)


def test_fc1d_second_derivative_converges_on_fig1():
    """Second derivative of the 1D-FC (both blends) of Fig. 1's function on
    [0, 1]: the error at the data points falls at order >= d - 2 - 0.3."""
    import sympy as sp
    X = sp.symbols("x")
    phi = sp.exp(sp.sin(sp.Rational(27, 5) * sp.pi * X - sp.Rational(27, 10) * sp.pi) - sp.cos(2 * sp.pi * X)) \
        - sp.sin(sp.Rational(5, 2) * sp.pi * X) + 1
    f = sp.lambdify(X, phi, "numpy")
    f2 = sp.lambdify(X, sp.diff(phi, X, 2), "numpy")
    tab = fcgram.load_tables(5)
    A = tab["A"]
    errs = []
    for n in (101, 201, 401):
        x = np.linspace(0.0, 1.0, n)
        d2 = FS.fc1d_d2(f(x), x[1] - x[0], tab["Q"], A)
        errs.append(np.abs(d2 - f2(x)).max() / np.abs(f2(x)).max())
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert errs[-1] < 1e-4 and min(orders) > 5 - 2 - 0.3, (errs, orders)


def test_fc1d_second_derivative_of_a_wrong_sign_is_caught():
    """The operator's sign: the second derivative of sin(3x + 1) is -9 sin(3x + 1)."""
    tab = fcgram.load_tables(5)
    x = np.linspace(0.0, 1.0, 161)
    d2 = FS.fc1d_d2(np.sin(3 * x + 1), x[1] - x[0], tab["Q"], tab["A"])
    assert np.abs(d2 + 9 * np.sin(3 * x + 1)).max() < 1e-4


def test_lagrange_second_derivative_weights_exact_for_polynomials():
    rng = np.random.default_rng(3)
    nodes = np.sort(rng.uniform(-1.0, 6.0, 7))
    x = 2.3
    w = FS.lagrange_d2_weights(nodes, x)
    for k in range(7):
        p2 = k * (k - 1) * x ** (k - 2) if k >= 2 else 0.0
        assert abs(w @ nodes ** k - p2) < 1e-9 * max(1.0, abs(p2)), k


def test_boundary_region_covers_the_band_within_c_dT(disc256):
    """Every IN point outside the boundary region lies at least c dT from
    Gamma (the domain of dependence of U_FC over a large step); on the unit
    disc the distance is 1 - |x|."""
    pl, st = disc256
    X, Y = np.meshgrid(pl.grid.xs(), pl.grid.ys(), indexing="ij")
    dist = 1.0 - np.hypot(X, Y)
    far = st.inside & ~st.ub
    assert dist[far].min() >= st.c * st.dT
    assert st.ub.sum() > 0 and far.sum() > 0
    assert st.K == 48 and abs(st.dt * st.K - st.dT) < 1e-15 and st.dt <= 0.125 * pl.grid.h / st.c * (1 + 1e-12)


def test_segments_and_boundary_stencils(disc256):
    """Each stepped point is differentiated by exactly one x and one y
    segment; boundary points interpolate from M_b nodes including a crossing
    on Gamma between the run end and its outside neighbour."""
    pl, st = disc256
    cnt = np.zeros((2,) + st.inside.shape, dtype=np.int64)
    for ax, line, lo, hi, kind, pts in st.segments:
        sel = pts if kind == "fc" else pts[0]
        for p in sel:
            cnt[(ax,) + ((p, line) if ax == 0 else (line, p))] += 1
        if kind == "fc":
            assert hi - lo + 1 >= 2 * pl.d
    assert np.array_equal(cnt[0][st.stepped], np.ones(st.stepped.sum(), dtype=np.int64))
    assert np.array_equal(cnt[1][st.stepped], np.ones(st.stepped.sum(), dtype=np.int64))
    assert cnt[:, ~st.stepped].sum() == 0
    r = np.hypot(st.cross_xy[:, 0], st.cross_xy[:, 1])
    assert np.abs(r - 1.0).max() < 1e-13
    for (i, j), (refs, wts) in st.bstencil.items():
        assert st.bnd[i, j]
        assert any(k == "cross" for k, _ in refs)
        assert len(refs) == min(st.M_b, len(refs)) and abs(wts.sum() - 1.0) < 1e-12
    for (ax, line, end, outn), pos in st.cross.items():
        assert min(end, outn) - 1e-9 <= pos <= max(end, outn) + 1e-9


def test_one_large_step_interior_at_fc_accuracy(disc256):
    """After one large step the points of Omega_dT carry U_FC, whose error is
    that of the 2D-FC of the exact data (1e-7; measured 5.6e-9); the boundary
    region carries U_B (2e-3; measured 2.3e-4)."""
    pl, st = disc256
    X, Y = np.meshgrid(pl.grid.xs(), pl.grid.ys(), indexing="ij")
    u0 = np.where(st.inside, ue(X, Y, 0.0), 0.0)
    v0 = np.where(st.inside, ute(X, Y, 0.0), 0.0)
    u1, v1 = FS.advance(st, u0, v0, 0.0, ue, ute)
    e = np.abs(u1 - ue(X, Y, st.dT))
    far = st.inside & ~st.ub
    assert e[far].max() < 1e-7
    assert e[st.ub].max() < 2e-3
    assert np.all(u1[~st.inside] == 0.0)


def test_plane_wave_converges_under_refinement():
    """Ex. 4.4 on the unit disc to t = 0.15 (two large steps at 256^2, four at
    512^2): the largest error over Omega falls at order > 3 (the 1D-FC second
    derivative is O(h^(d-2)) next to the segment ends; measured 2.2e-4 ->
    1.3e-5, order 4.0)."""
    errs = []
    for n, steps in ((256, 2), (512, 4)):
        pl = _plan(n)
        st = FS.make_setup(pl)
        X, Y = np.meshgrid(pl.grid.xs(), pl.grid.ys(), indexing="ij")
        u = np.where(st.inside, ue(X, Y, 0.0), 0.0)
        v = np.where(st.inside, ute(X, Y, 0.0), 0.0)
        t = 0.0
        for _ in range(steps):
            u, v = FS.advance(st, u, v, t, ue, ute)
            t += st.dT
        assert abs(t - 0.15) < 1e-12
        errs.append(np.abs(u - ue(X, Y, t))[st.inside].max())
    assert errs[0] < 5e-4 and math.log2(errs[0] / errs[1]) > 3.0, errs
