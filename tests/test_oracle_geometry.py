"""Pins for the oracle's Geometrical Setup (Sec. 3.1, 3.3, 3.4): closed-form
boundaries, reach, foot of the normal, classification of H."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import fcgram
from oracle import plan as P
from oracle.curves import Curve, boundary_grid, reach


def test_disc_boundary_closed_form():
    bd = boundary_grid(Curve(*W.disc()), 64)
    t = bd["theta"]
    assert np.allclose(bd["x"], np.cos(t), atol=1e-15) and np.allclose(bd["y"], np.sin(t), atol=1e-15)
    assert np.allclose(bd["nx"], np.cos(t), atol=1e-15) and np.allclose(bd["ny"], np.sin(t), atol=1e-15)


def test_ellipse_normals_are_outward_unit():
    bd = boundary_grid(Curve(*W.ellipse()), 128)
    n = np.stack([bd["nx"], bd["ny"]], 1)
    assert np.allclose(np.linalg.norm(n, axis=1), 1.0)
    # gradient of x^2/a^2 + y^2/b^2 points outward
    g = np.stack([bd["x"] / 1.0, bd["y"] / 0.25], 1)
    g /= np.linalg.norm(g, axis=1)[:, None]
    assert np.allclose(n, g, atol=1e-14)


@pytest.mark.parametrize("curve,ext,intr", [
    (W.star5(), 0.0721, 0.192),
    (W.kite(0.65, 1.5), 1.406, 0.0855),
    (W.kite(0.35, 0.7), 1.225, 0.143),
    (W.ellipse(), math.inf, 0.25),
    (W.disc(), math.inf, 1.0),
])
def test_reach(curve, ext, intr):
    re, ri = reach(Curve(*curve), 200000)
    if math.isinf(ext):
        assert math.isinf(re)
    else:
        assert abs(re - ext) < 2e-3 * max(1.0, ext)
    assert abs(ri - intr) < 1e-3 * max(1.0, intr)


def test_ellipse_analytic_curvature_radius():
    # minimum radius of curvature of an ellipse is b^2/a
    _, ri = reach(Curve(*W.ellipse(1.0, 0.5)), 100000)
    assert abs(ri - 0.25) < 1e-9


def test_foot_disc_exact():
    curve = Curve(*W.disc())
    bd = boundary_grid(curve, 256)
    rng = np.random.default_rng(1)
    r = rng.uniform(0.8, 1.2, 500)
    a = rng.uniform(0, 2 * np.pi, 500)
    X, Y = r * np.cos(a), r * np.sin(a)
    p = np.rint(np.mod(a, 2 * np.pi) / bd["k2"]).astype(int) % 256
    th, eta, it = P.foot_solve(curve, bd, X, Y, p, 8)
    assert np.allclose(th, np.mod(np.arctan2(Y, X), 2 * np.pi), atol=4e-15)
    assert np.allclose(eta, np.hypot(X, Y) - 1.0, atol=1e-15)
    assert it.max() <= 4


def test_foot_ellipse_brute_force():
    curve = Curve(*W.ellipse())
    bd = boundary_grid(curve, 512)
    rng = np.random.default_rng(2)
    t0 = rng.uniform(0, 2 * np.pi, 200)
    x, y, x1, y1, *_ = curve.eval_vec(t0)
    s = np.hypot(x1, y1)
    dist = rng.uniform(-0.1, 0.2, 200)
    X, Y = x + dist * y1 / s, y - dist * x1 / s
    p = np.rint(t0 / bd["k2"]).astype(int) % 512
    th, eta, _ = P.foot_solve(curve, bd, X, Y, p, 8)
    # brute force: minimise |Q - q(t)| over a fine parameter grid, then compare
    tt = np.linspace(0, 2 * np.pi, 400001)
    qx, qy, *_ = curve.eval_vec(tt)
    for k in range(0, 200, 20):
        dmin = np.min(np.hypot(qx - X[k], qy - Y[k]))
        assert abs(abs(eta[k]) - dmin) < 1e-8
    assert np.allclose(eta, dist, atol=1e-13)
    assert np.allclose(np.mod(th - t0 + np.pi, 2 * np.pi) - np.pi, 0.0, atol=1e-12)


@pytest.fixture(scope="module")
def disc_plan():
    case = W.cfg_disc128()
    tab = fcgram.load_tables(5)
    g = P.Grid(case.x0, case.y0, case.h, case.n, case.n)
    return case, P.make_plan(Curve(*case.curve), g, tab, case.B, k1=case.k1, M=case.M)


def test_disc_classification_closed_form(disc_plan):
    case, pl = disc_plan
    x = case.x0 + np.arange(case.n) * case.h
    X, Y = np.meshgrid(x, x, indexing="ij")
    r = np.hypot(X, Y)
    width = case.C * case.k1
    expect = np.where(r <= 1.0, P.IN, np.where(r - 1.0 <= width, P.STRIP, P.FAR))
    safe = (np.abs(r - 1.0) > 1e-12) & (np.abs(r - 1.0 - width) > 1e-12)
    assert np.array_equal(pl.cls[safe], expect[safe])


def test_proximity_map_seeds_are_near(disc_plan):
    case, pl = disc_plan
    pm = P.proximity_map(pl)
    assert np.all(pm >= 0)
    # the partner normal is within a few normals of the exact foot
    dp = np.abs(((pm - pl.strip_theta / pl.k2) + pl.B / 2) % pl.B - pl.B / 2)
    assert dp.max() < 4


def test_admissibility_rejects_wide_strip():
    # star with k1 = h on 256^2 leaves the reach (Appendix A of the design notes)
    case = W.box_case("s", W.star5(), -1.6, 1.6, 256, 512)
    g = P.Grid(case.x0, case.y0, case.h, case.n, case.n)
    with pytest.raises(P.GeometryError):
        P.make_plan(Curve(*case.curve), g, fcgram.load_tables(5), case.B, k1=case.h)


def test_admissibility_rejects_small_box():
    case = W.box_case("s", W.disc(), -1.1, 1.1, 128, 256)
    g = P.Grid(case.x0, case.y0, case.h, case.n, case.n)
    with pytest.raises(P.GeometryError):
        P.make_plan(Curve(*case.curve), g, fcgram.load_tables(5), case.B, k1=case.h)
