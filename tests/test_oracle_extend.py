"""Pins for the oracle's Cartesian Evaluation (Secs. 3.2, 3.4, 3.5): exactness on
polynomials, the one-dimensional reduction on the disc, assembly rules, and the
paper's printed convergence tables."""
import math

import numpy as np
import pytest

import workloads as W
from conftest import load_golden
from oracle import extend as E
from oracle import fcgram
from oracle import plan as P
from oracle import spectral as S
from oracle.curves import Curve


def _plan(case, d=5, M=None):
    tab = fcgram.load_tables(d)
    g = P.Grid(case.x0, case.y0, case.h, case.n, case.n)
    return P.make_plan(Curve(*case.curve), g, tab, case.B, k1=case.k1, M=M or d + 3)


@pytest.fixture(scope="module")
def star_plan():
    return _plan(W.cfg_star(256 + 64))


@pytest.fixture(scope="module")
def disc_plan():
    return _plan(W.cfg_disc128())


def _poly7(x, y):
    return 0.3 + x - 0.7 * y + x * y ** 2 - 0.2 * x ** 4 * y + 0.05 * x ** 3 * y ** 4 + 0.01 * y ** 7


@pytest.mark.parametrize("which", ["disc", "star"])
def test_matching_values_exact_for_degree_M_minus_1(which, disc_plan, star_plan):
    pl = disc_plan if which == "disc" else star_plan
    bp = P.boundary_points(pl)
    fg = _poly7(*np.meshgrid(pl.grid.xs(), pl.grid.ys(), indexing="ij"))
    fD = E.matching_values(pl, fg, _poly7(bp[:, 0], bp[:, 1])).astype(np.float64)
    q = np.arange(pl.d)
    rx = pl.bd["x"][:, None] + pl.bd["nx"][:, None] * ((q - pl.d + 1) * pl.k1)[None, :]
    ry = pl.bd["y"][:, None] + pl.bd["ny"][:, None] * ((q - pl.d + 1) * pl.k1)[None, :]
    assert np.abs(fD - _poly7(rx, ry)).max() < 1e-12


def test_matching_mistake_is_caught(disc_plan):
    """A transposed weight table (a plausible indexing slip) breaks exactness."""
    pl = disc_plan
    bp = P.boundary_points(pl)
    fg = _poly7(*np.meshgrid(pl.grid.xs(), pl.grid.ys(), indexing="ij"))
    good = E.matching_values(pl, fg, _poly7(bp[:, 0], bp[:, 1]))
    saved = pl.match_wv
    try:
        pl.match_wv = np.swapaxes(saved, 1, 2).copy()
        bad = E.matching_values(pl, fg, _poly7(bp[:, 0], bp[:, 1]))
    finally:
        pl.match_wv = saved
    assert np.abs((bad - good).astype(float)).max() > 1e-3


def test_radial_data_reduces_to_1d(disc_plan):
    """On the disc, radial polynomial data gives the same 1D problem along every
    normal: the extension at Q depends only on eta_Q and equals the degree-(M-1)
    interpolant in the level variable of [f(1); A_r Q^T f(r_q)] (Sec. 3.2-3.4)."""
    pl = disc_plan
    f = lambda x, y: (x * x + y * y) ** 3 - 0.5 * (x * x + y * y)
    bp = P.boundary_points(pl)
    fg = f(*np.meshgrid(pl.grid.xs(), pl.grid.ys(), indexing="ij"))
    fb = f(bp[:, 0], bp[:, 1])
    F = E.blend(pl, E.matching_values(pl, fg, fb))
    ext = E.strip_values(pl, F)
    # independent 1D computation
    r = 1.0 + (np.arange(pl.d) - pl.d + 1) * pl.k1
    phi = r ** 6 - 0.5 * r ** 2
    col = np.concatenate([[phi[-1]], pl.Ar @ (pl.Q.T @ phi)])
    s = pl.strip_eta * pl.n_r / pl.k1
    expect = np.empty_like(s)
    for k, sk in enumerate(s):
        l0 = min(max(int(math.floor(sk)) - pl.M // 2 + 1, 0), pl.Cr - pl.M + 1)
        nodes = np.arange(l0, l0 + pl.M, dtype=float)
        w = np.array([np.prod([(sk - nodes[m]) / (nodes[j] - nodes[m]) for m in range(pl.M) if m != j])
                      for j in range(pl.M)])
        expect[k] = w @ col[l0:l0 + pl.M]
    assert np.abs(ext - expect).max() < 1e-11 * max(1.0, np.abs(expect).max())


def test_strip_interpolation_exact_on_tensor_polynomials(star_plan):
    """F[l, p] = P(l) T(theta_p) with degree <= M-1 factors: the two-step
    interpolation reproduces P(s) T(theta^Q) (checks the theta and level stencils)."""
    pl = star_plan
    Pl = lambda l: 1.0 + 0.01 * l - 1e-4 * l ** 2 + 1e-12 * l ** 7
    Tt = lambda t: 0.5 + (t - 3.0) - 0.1 * (t - 3.0) ** 3 + 0.01 * (t - 3.0) ** 7
    l = np.arange(pl.Cr + 1, dtype=float)
    th = np.arange(pl.B) * pl.k2
    F = Pl(l)[:, None] * Tt(th)[None, :]
    ext = E.strip_values(pl, F)
    ok = (pl.strip_theta > 0.2) & (pl.strip_theta < 2 * np.pi - 0.2)
    s = pl.strip_eta * pl.n_r / pl.k1
    expect = Pl(s) * Tt(pl.strip_theta)
    assert np.abs(ext - expect)[ok].max() < 1e-10


def test_assembly_rules(disc_plan):
    pl = disc_plan
    f = W.f_cfg1
    bp = P.boundary_points(pl)
    fg = f(*np.meshgrid(pl.grid.xs(), pl.grid.ys(), indexing="ij"))
    fg_noisy = fg.copy()
    fg_noisy[pl.cls != P.IN] = np.nan      # only IN entries may be read
    ext = E.extend(pl, fg_noisy, f(bp[:, 0], bp[:, 1]))
    assert np.array_equal(ext[pl.cls == P.IN], fg[pl.cls == P.IN])
    assert np.all(ext[pl.cls == P.FAR] == 0.0)
    assert np.all(np.isfinite(ext))
    # the extension decays to ~0 at the outer edge of the strip
    outer = pl.strip_eta > 0.97 * pl.C * pl.k1
    assert np.abs(ext.ravel()[pl.strip_idx[outer]]).max() < 1e-4 * np.abs(fg).max()


def _disc_error(d, h, B):
    n = int(round(3.2 / h))
    case = W.box_case("t1", W.disc(), -1.6, 1.6, n, B, d=d, M=d + 3)
    pl = _plan(case, d=d)
    f = W.f_paper_disc
    bp = P.boundary_points(pl)
    ext = E.extend(pl, W.grid_values(case, f), f(bp[:, 0], bp[:, 1]))
    up = S.upsample_h2(ext)
    x = case.x0 + np.arange(2 * n) * case.h / 2
    X, Y = np.meshgrid(x, x, indexing="ij")
    ins = X ** 2 + Y ** 2 < 1
    ex = f(X, Y)
    return np.abs(up - ex)[ins].max() / np.abs(ex[ins]).max()


@pytest.mark.slow
def test_paper_table1_disc():
    rows = [r for r in load_golden("paper_table1_disc.txt") if r[0] in (4, 5)]
    for d in (4, 5):
        errs = []
        for r in [r for r in rows if r[0] == d]:
            e = _disc_error(d, r[1], int(r[3]))
            errs.append(e)
            assert r[4] / 2 < e < 2 * r[4], (d, r, e)        # measured 0.82 - 1.07
        orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
        assert orders[-1] > d - 0.7, (d, errs)


def _kite_error(d, M, h, nx, ny):
    curve = W.kite(0.35, 0.7)
    xmin, xmax, ymin, ymax = W.bbox(curve)
    f = W.f_paper_kite
    x0 = 0.5 * (xmin + xmax) - 0.5 * nx * h
    y0 = 0.5 * (ymin + ymax) - 0.5 * ny * h
    g = P.Grid(x0, y0, h, nx, ny)
    pl = P.make_plan(Curve(*curve), g, fcgram.load_tables(d), int(round(2 * np.pi / h)), k1=h, M=M)
    bp = P.boundary_points(pl)
    X, Y = np.meshgrid(g.xs(), g.ys(), indexing="ij")
    ext = E.extend(pl, f(X, Y), f(bp[:, 0], bp[:, 1]))
    U = np.fft.fft2(ext)
    # values on the h/2 grid by zero padding
    P2 = np.zeros((2 * nx, 2 * ny), dtype=complex)
    hx, hy = nx // 2, ny // 2
    P2[:hx + 1, :hy + 1] = U[:hx + 1, :hy + 1]
    P2[-hx:, :hy + 1] = U[-hx:, :hy + 1]
    P2[:hx + 1, -hy:] = U[:hx + 1, -hy:]
    P2[-hx:, -hy:] = U[-hx:, -hy:]
    up = np.real(np.fft.ifft2(P2)) * 4
    X2, Y2 = np.meshgrid(x0 + np.arange(2 * nx) * h / 2, y0 + np.arange(2 * ny) * h / 2, indexing="ij")
    ins = P.column_parity_inside(Curve(*curve), P.Grid(x0, y0, h / 2, 2 * nx, 2 * ny), 16384)
    return np.abs(up - f(X2, Y2))[ins].max()


@pytest.mark.slow
def test_paper_table1_disc_d10():
    """Table 1's d = 10 rows (M = 13): within 10x at h = 2e-2 and 3x at h = 1e-2
    (measured 7.4x and 1.9x; the tables here use the band limit of d = 4, 5)."""
    rows = [r for r in load_golden("paper_table1_disc.txt") if r[0] == 10]
    for (_, h, _, B, ref), bar in zip(rows, (10.0, 3.0)):
        e = _disc_error(10, h, int(B))
        assert ref / bar < e < bar * ref, (h, e, ref)


@pytest.mark.slow
def test_paper_table2_kite():
    """Kite of Example 3.2 on the printed N_x x N_y grids, every M column
    (M = d + 1, d + 2, d + 3) of the rows h = 1e-2, 5e-3: each error within a
    factor 3 of the printed one (measured 0.48 - 2.1)."""
    for d, h, nx, ny, *refs in [r for r in load_golden("paper_table2_kite.txt") if r[1] >= 5e-3]:
        d, nx, ny = int(d), int(nx), int(ny)
        for M, ref in zip((d + 1, d + 2, d + 3), refs):
            err = _kite_error(d, M, h, nx, ny)
            assert ref / 3 < err < 3 * ref, (d, M, h, err, ref)
