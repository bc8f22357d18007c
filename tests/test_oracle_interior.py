"""Pins for the oracle's extension from interior data only (Remark 3.1 II):
stencils without boundary samples, exact matching values (the point on Gamma
included) for polynomials of degree M - 1, a planted weight mistake caught, and
convergence on the paper's Example 3.1 with the accuracy a little below that
of the extension with boundary data."""
import numpy as np
import pytest

import workloads as W
from oracle import extend as E
from oracle import fcgram
from oracle import plan as P
from oracle import spectral as S
from oracle.curves import Curve


def _plan(case, d=5, io=True):
    g = P.Grid(case.x0, case.y0, case.h, case.n, case.n)
    return P.make_plan(Curve(*case.curve), g, fcgram.load_tables(d), case.B, k1=case.k1, M=d + 3,
                       interior_only=io)


@pytest.fixture(scope="module")
def plans():
    return {"disc": _plan(W.cfg_disc128()), "star": _plan(W.cfg_star(256 + 64))}


def _poly7(x, y):
    return 0.3 + x - 0.7 * y + x * y ** 2 - 0.2 * x ** 4 * y + 0.05 * x ** 3 * y ** 4 + 0.01 * y ** 7


def _matching_points(pl):
    q = np.arange(pl.d)
    rx = pl.bd["x"][:, None] + pl.bd["nx"][:, None] * ((q - pl.d + 1) * pl.k1)[None, :]
    ry = pl.bd["y"][:, None] + pl.bd["ny"][:, None] * ((q - pl.d + 1) * pl.k1)[None, :]
    return rx, ry


@pytest.mark.parametrize("which", ["disc", "star"])
def test_stencils_use_interior_points_only(plans, which):
    pl = plans[which]
    assert len(pl.squares) == 0
    assert np.all(pl.match_ref >= 0)
    assert np.all(pl.cls.ravel()[pl.match_ref] == P.IN)
    assert pl.match_wn.shape == (pl.B, pl.d, pl.M)


@pytest.mark.parametrize("which", ["disc", "star"])
def test_matching_values_exact_for_degree_M_minus_1(plans, which):
    """Every matching value, the one on Gamma included, reproduces a polynomial
    of total degree 7 = M - 1 from grid values alone (no boundary samples)."""
    pl = plans[which]
    fg = _poly7(*np.meshgrid(pl.grid.xs(), pl.grid.ys(), indexing="ij"))
    fD = E.matching_values(pl, fg, None).astype(np.float64)
    rx, ry = _matching_points(pl)
    assert np.abs(fD - _poly7(rx, ry)).max() < 1e-11


def test_boundary_row_mistake_is_caught(plans):
    """Taking the row of the innermost interior matching point for the point on
    Gamma (a plausible off-by-one in the depth) breaks exactness there."""
    pl = plans["disc"]
    fg = _poly7(*np.meshgrid(pl.grid.xs(), pl.grid.ys(), indexing="ij"))
    saved = pl.match_wn
    try:
        bad_wn = saved.copy()
        bad_wn[:, pl.d - 1] = saved[:, pl.d - 2]
        pl.match_wn = bad_wn
        fD = E.matching_values(pl, fg, None).astype(np.float64)
    finally:
        pl.match_wn = saved
    rx, ry = _matching_points(pl)
    assert np.abs(fD[:, -1] - _poly7(rx[:, -1], ry[:, -1])).max() > 1e-3


def _disc_error(n, B, io, d=5):
    case = W.box_case("t1", W.disc(), -1.6, 1.6, n, B, d=d, M=d + 3)
    pl = _plan(case, d=d, io=io)
    f = W.f_paper_disc
    bp = P.boundary_points(pl)
    ext = E.extend(pl, W.grid_values(case, f), None if io else f(bp[:, 0], bp[:, 1]))
    up = S.upsample_h2(ext)
    x = case.x0 + np.arange(2 * n) * case.h / 2
    X, Y = np.meshgrid(x, x, indexing="ij")
    ins = X ** 2 + Y ** 2 < 1
    ex = f(X, Y)
    return np.abs(up - ex)[ins].max() / np.abs(ex[ins]).max()


def test_convergence_example_3_1():
    """Disc, f = -sin(5 pi x) sin(5 pi y), d = 5 (Table 1's setting) on 320^2 and
    640^2: order above d - 0.7 over the halving, and within 5x of the error of
    the extension that reads the boundary samples."""
    errs = []
    for n, B in ((320, 628), (640, 1257)):
        e_io, e_bd = _disc_error(n, B, True), _disc_error(n, B, False)
        print("\n[interior-only] N=%d: %.2e (with boundary data %.2e)" % (n, e_io, e_bd))
        assert e_io < 5 * e_bd
        errs.append(e_io)
    assert np.log2(errs[0] / errs[1]) > 5 - 0.7
