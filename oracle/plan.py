"""Geometrical Setup of 2D-FC (oracle side): Sec. 3.5 steps 1-4 and the
matching stencils of Sec. 3.2.

Grid arrays are indexed [i, j] <-> (x_i, y_j) = (x0 + i h, y0 + j h) with j
fastest (eq. cart_grid); the box is periodic with period N h (the right edge
is excluded).  Point classes: FAR = 0 (value 0), IN = 1 (value f kept, which
includes points exactly on Gamma), STRIP = 2 (0 < eta <= C k1, value
interpolated from V+_{B,C_r}).

Readings of the paper taken here (the paper leaves them open):
* Classification.  A grid point is first IN or FAR by the parity of the
  crossings of its grid column with a 16 B-vertex polygon of Gamma.  "Band"
  points -- outside points whose nearest boundary sample lies within
  C k1 + ds/2 and inside points within h + ds/2 (ds = k2 max|q'|, the largest
  sample spacing) -- then get a foot of the normal, and their signed normal
  distance eta decides IN (eta <= 0), STRIP (0 < eta <= C k1) or FAR
  (eta > C k1).  A point with eta <= 1e-13 (1 + |x| + |y|) is taken to lie
  on Gamma and is IN: this keeps grid points that sit exactly on Gamma (e.g.
  (1.3, 0) on the star) out of the rounding noise of eta.  Every point with 0 < eta <= C k1 is a band point, since its
  nearest sample is at most sqrt((C k1)^2 + (ds/2)^2) away.
* Proximity map.  The seed of every foot solve is the normal p of the
  nearest boundary point of V+_{B,C_r} (level q = 0) -- the index part of the
  proximity map of Sec. 3.3; the level index is not needed because the foot
  is refined to full precision.  ``proximity_map`` builds the literal map of
  Sec. 3.3 over all levels for checking seeds.
* Foot of the normal (Sec. 3.4).  Seed theta^(0) by interpolating
  theta = T(tau) over the M normals of S_{theta_p} at tau = 0 (eq. param_tau),
  then safeguarded Newton on g(theta) = (q(theta) - Q).q'(theta) inside a
  bracket around theta_p, to |d theta| <= 4e-16 * 2 pi or until the bracket
  is within 8 units in the last place.
* Matching stencils (Sec. 3.2, Fig. 3).  Candidate red stars are the
  crossings, at depth >= 0 and in order of depth, of the inward normal with
  the grid lines x = x_i (when |n_x| >= |n_y|) or y = y_j.  A star's nodes are
  the IN points of the run of IN points on its line that holds the star (at
  most M + 1 grid steps away) and the crossings of that line with Gamma that
  bound the run ("squares"); a square closer than h/2 to one of these IN
  nodes is dropped.  The red stars are the first M - 1 candidates offering at
  least M nodes (a line nearly tangent to Gamma next to a shallow star offers
  too few), and each uses the M nodes nearest to it.  Squares are listed once
  per use, in the order normal, star, node.  Values at the d - 1 interior
  matching points come from a degree-(M-1) interpolation along the normal over
  M nodes: the M - 1 stars and the point on Gamma itself (depth 0, the
  boundary sample), which also gives the matching point on Gamma.  Weights are
  formed in numpy.longdouble.
* Interior data only (Remark 3.1 II; ``interior_only=True``).  No squares: a
  star's nodes are IN points only, the along-normal interpolation uses M stars
  (no boundary sample to stand at depth 0), and the matching point on Gamma
  takes that interpolation too.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial import cKDTree

from .curves import boundary_grid, reach
from .interp import lagrange_weights

FAR, IN, STRIP = 0, 1, 2
LD = np.longdouble
TWO_PI = 2.0 * math.pi
EPS = 2.0 ** -52
ON_GAMMA_TOL = 1e-13
STAR_MIN_DEPTH = 0.05   # red stars closer to Gamma than this fraction of the star spacing are skipped


class GeometryError(Exception):
    pass


class Grid:
    def __init__(self, x0, y0, h, nx, ny):
        self.x0, self.y0, self.h, self.nx, self.ny = float(x0), float(y0), float(h), int(nx), int(ny)

    def xs(self):
        return self.x0 + np.arange(self.nx) * self.h

    def ys(self):
        return self.y0 + np.arange(self.ny) * self.h


# --------------------------------------------------------------------------
# foot of the normal (Sec. 3.4, eq. surround and eq. param_tau)
# --------------------------------------------------------------------------
def stencil_offsets(M):
    """Offsets -K_l..K_r of S_theta (eq. surround): K_l = K_r for odd M, K_r = K_l + 1 for even M."""
    kl = (M - 1) // 2
    kr = M // 2
    return np.arange(-kl, kr + 1)


def t_tau_seed(bd, X, Y, p, M):
    """theta^(0) = T(0) by Lagrange interpolation of (tau_j, theta_j) over S_{theta_p}."""
    B = bd["x"].size
    k2 = bd["k2"]
    j = p[:, None] + stencil_offsets(M)[None, :]
    jj = j % B
    tx = -bd["ny"][p][:, None]          # tangent direction of L_Q^perp (orthogonal to n(theta_p))
    ty = bd["nx"][p][:, None]
    ax = bd["nx"][jj]
    ay = bd["ny"][jj]
    wx = X[:, None] - bd["x"][jj]
    wy = Y[:, None] - bd["y"][jj]
    # q_j + sigma n_j = Q + tau t   <=>   sigma n_j - tau t = Q - q_j
    det = ax * (-ty) - (-tx) * ay
    tau = (ax * wy - wx * ay) / det
    theta_j = j * k2
    with np.errstate(all="ignore"):
        w = lagrange_weights(tau, np.zeros(len(p)))
        th0 = np.sum(w * theta_j, axis=1)
    return th0


def foot_solve(curve, bd, X, Y, p, M, tol=4e-16 * TWO_PI, maxit=60):
    """Foot parameter theta^Q in [0, 2pi) and signed distance eta for points (X, Y).

    p is the seed normal index.  Returns (theta, eta, iterations).
    """
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    p = np.asarray(p, dtype=np.int64)
    k2 = bd["k2"]
    thp = p * k2
    n = X.size
    if n == 0:
        return np.zeros(0), np.zeros(0), np.zeros(0, dtype=np.int64)

    def g_and_gp(th, idx=slice(None)):
        x, y, x1, y1, x2, y2 = curve.eval_vec(th)
        dx = x - X[idx]
        dy = y - Y[idx]
        return dx * x1 + dy * y1, x1 * x1 + y1 * y1 + dx * x2 + dy * y2

    # bracket [lo, hi] with g(lo) < 0 < g(hi), widened until it holds
    half = np.full(n, 2.0 * k2)
    lo = thp - half
    hi = thp + half
    for _ in range(6):
        glo, _ = g_and_gp(lo)
        ghi, _ = g_and_gp(hi)
        bad = ~((glo < 0) & (ghi > 0))
        if not bad.any():
            break
        half = np.where(bad, 2.0 * half, half)
        lo = np.where(bad, thp - half, lo)
        hi = np.where(bad, thp + half, hi)
    else:
        raise GeometryError("foot of the normal: no bracket")

    th = t_tau_seed(bd, X, Y, p, M)
    th = np.where(np.isfinite(th) & (th > lo) & (th < hi), th, thp)
    active = np.ones(n, dtype=bool)
    iters = np.zeros(n, dtype=np.int64)
    for _ in range(maxit):
        if not active.any():
            break
        idx = np.nonzero(active)[0]
        t = th[idx]
        g, gp = g_and_gp(t, idx)
        neg = g < 0
        lo[idx] = np.where(neg, t, lo[idx])
        hi[idx] = np.where(g > 0, t, hi[idx])
        new = t - g / gp
        outside = ~((new >= lo[idx]) & (new <= hi[idx]))     # also catches NaN
        new = np.where(outside, 0.5 * (lo[idx] + hi[idx]), new)
        new = np.where(g == 0, t, new)
        iters[idx] += 1
        th[idx] = new
        # converged: a step below tol, or the bracket around the root collapsed
        # to within tol (near the reach, rounding noise in g can exceed tol * g')
        done = (np.abs(new - t) <= tol) | (hi[idx] - lo[idx] <= 8 * EPS * np.maximum(1.0, np.abs(hi[idx])))
        active[idx[done]] = False
    else:
        if active.any():
            raise GeometryError("foot of the normal: Newton did not converge")
    th = np.fmod(th, TWO_PI)
    th = np.where(th < 0, th + TWO_PI, th)
    x, y, x1, y1, _, _ = curve.eval_vec(th)
    sp = np.sqrt(x1 * x1 + y1 * y1)
    eta = (X - x) * (y1 / sp) + (Y - y) * (-x1 / sp)
    return th, eta, iters


# --------------------------------------------------------------------------
# inside / outside by crossing parity (points away from Gamma)
# --------------------------------------------------------------------------
def column_parity_inside(curve, grid, nverts):
    """Boolean [nx, ny]: inside the polygon of nverts boundary points, by the
    parity of crossings of each grid column x = x_i below the point."""
    t = np.arange(nverts) * (TWO_PI / nverts)
    px, py, *_ = curve.eval_vec(t)
    ax, ay = px, py
    bx, by = np.roll(px, -1), np.roll(py, -1)
    # columns i with min(ax,bx) <= x_i < max(ax,bx) (half-open rule)
    xmin = np.minimum(ax, bx)
    xmax = np.maximum(ax, bx)
    i0 = np.ceil((xmin - grid.x0) / grid.h).astype(np.int64)
    i1 = np.ceil((xmax - grid.x0) / grid.h).astype(np.int64)  # exclusive
    cnt = np.maximum(i1 - i0, 0)
    e = np.repeat(np.arange(nverts), cnt)
    ii = np.concatenate([np.arange(a, b) for a, b in zip(i0, i1) if b > a]) if cnt.sum() else np.zeros(0, np.int64)
    xc = grid.x0 + ii * grid.h
    s = (xc - ax[e]) / (bx[e] - ax[e])
    yc = ay[e] + s * (by[e] - ay[e])
    inside = np.zeros((grid.nx, grid.ny), dtype=bool)
    ys = grid.ys()
    order = np.lexsort((yc, ii))
    ii = ii[order]
    yc = yc[order]
    starts = np.searchsorted(ii, np.arange(grid.nx))
    ends = np.searchsorted(ii, np.arange(grid.nx), side="right")
    for i in range(grid.nx):
        if ends[i] == starts[i] or i < 0:
            continue
        k = np.searchsorted(yc[starts[i]:ends[i]], ys)  # crossings strictly below y_j
        inside[i] = (k % 2) == 1
    return inside


# --------------------------------------------------------------------------
# the plan
# --------------------------------------------------------------------------
class Plan:
    pass


def make_plan(curve, grid, tables, B, k1=None, M=None, n_r=None, interior_only=False):
    """Geometrical Setup (Sec. 3.5 steps 1-4) plus the matching stencils of Sec. 3.2
    (from interior data only when ``interior_only``: Remark 3.1 II)."""
    d = tables["Q"].shape[0]
    C = tables["A"].shape[0]
    n_r = tables["Ar"].shape[0] // C if n_r is None else n_r
    Cr = C * n_r
    M = d + 3 if M is None else M
    h = grid.h
    k1 = h if k1 is None else float(k1)
    pl = Plan()
    pl.curve, pl.grid, pl.d, pl.C, pl.n_r, pl.Cr, pl.M, pl.k1, pl.B = curve, grid, d, C, n_r, Cr, M, k1, B
    pl.interior_only = bool(interior_only)
    pl.Q, pl.Ar = tables["Q"], tables["Ar"]

    # step 1: boundary discretisation and normals (eq. bdry_grid)
    bd = boundary_grid(curve, B)
    pl.bd = bd
    pl.k2 = bd["k2"]

    # admissibility: the exterior strip must stay within the exterior reach and inside the box
    r_ext, r_int = reach(curve, 16 * B)
    pl.reach_ext, pl.reach_int = r_ext, r_int
    if C * k1 > 0.9 * r_ext:
        raise GeometryError("C k1 = %.4g exceeds 0.9 x exterior reach %.4g" % (C * k1, r_ext))
    ox = bd["x"] + bd["nx"] * (C * k1)
    oy = bd["y"] + bd["ny"] * (C * k1)
    xlo, xhi = grid.x0, grid.x0 + (grid.nx - 1) * h
    ylo, yhi = grid.y0, grid.y0 + (grid.ny - 1) * h
    allx = np.concatenate([bd["x"], ox])
    ally = np.concatenate([bd["y"], oy])
    if allx.min() < xlo or allx.max() > xhi or ally.min() < ylo or ally.max() > yhi:
        raise GeometryError("Omega u V+ is not inside the box")

    # step 3: classification of H and proximity (nearest point of V+_{B,C_r} on level 0)
    sp = np.sqrt(bd["x1"] ** 2 + bd["y1"] ** 2)
    ds = pl.k2 * float(sp.max())                # largest spacing of the boundary samples
    tree = cKDTree(np.stack([bd["x"], bd["y"]], axis=1))
    pl.tree = tree
    XX, YY = np.meshgrid(grid.xs(), grid.ys(), indexing="ij")
    r_out = C * k1 + 0.5 * ds + 1e-12          # every point with 0 < eta <= C k1 is this close to a sample
    r_in = 0.5 * ds + h
    dist, near = tree.query(np.stack([XX.ravel(), YY.ravel()], axis=1), distance_upper_bound=r_out)
    inside = column_parity_inside(curve, grid, 16 * B).ravel()
    band = np.isfinite(dist) & np.where(inside, dist <= r_in, True)
    bidx = np.nonzero(band)[0]
    # step 4: foot of the normal for band points
    th, eta, iters = foot_solve(curve, bd, XX.ravel()[bidx], YY.ravel()[bidx], near[bidx], M)
    cls = np.where(inside, IN, FAR).astype(np.int8)
    # a point within rounding distance of Gamma counts as on Gamma, hence IN
    on_tol = ON_GAMMA_TOL * (1.0 + np.abs(XX.ravel()[bidx]) + np.abs(YY.ravel()[bidx]))
    bcls = np.where(eta <= on_tol, IN, np.where(eta <= C * k1, STRIP, FAR)).astype(np.int8)
    cls[bidx] = bcls
    pl.cls = cls.reshape(grid.nx, grid.ny)
    sel = bcls == STRIP
    pl.strip_idx = bidx[sel]                   # flat indices, ascending = row-major
    pl.strip_theta = th[sel]
    pl.strip_eta = eta[sel]
    pl.strip_seed = near[bidx][sel]
    pl.newton_iters = iters[sel]

    # matching stencils (Sec. 3.2)
    _matching_stencils(pl)
    return pl


def _bisect_crossing(pl, ax_is_x, a_line, b_in, b_out, nit=64):
    """Crossings with Gamma of segments {a = a_line, b in [b_in, b_out]} where the
    b_in end is inside (eta <= 0) and the b_out end outside (eta > 0): bisection
    on the sign of eta (one foot solve per step)."""
    lo = np.asarray(b_in, dtype=np.float64).copy()
    hi = np.asarray(b_out, dtype=np.float64).copy()
    a_line = np.asarray(a_line, dtype=np.float64)
    for _ in range(nit):
        mid = 0.5 * (lo + hi)
        if ax_is_x is None:
            raise AssertionError
        X = np.where(ax_is_x, a_line, mid)
        Y = np.where(ax_is_x, mid, a_line)
        _, near = pl.tree.query(np.stack([X, Y], axis=1))
        _, eta, _ = foot_solve(pl.curve, pl.bd, X, Y, near, pl.M)
        inside = eta <= 0
        lo = np.where(inside, mid, lo)
        hi = np.where(inside, hi, mid)
    return 0.5 * (lo + hi)


def _matching_stencils(pl):
    grid, bd, M, d, h = pl.grid, pl.bd, pl.M, pl.d, pl.grid.h
    B = pl.B
    cls = pl.cls
    # phase 1: candidate stars (up to 2M crossings per normal), their runs of IN
    # nodes and the segments holding a crossing of the star line with Gamma
    star_rec = []      # (p, vertical, line index, delta (LD), bstar (LD))
    runs = []          # [lower IN j's, upper IN j's, square_lo, square_hi]
    sq_req = []        # (record id, side, vertical, a_line, b_in, b_out)
    for p in range(B):
        nx, ny = bd["nx"][p], bd["ny"][p]
        vertical = abs(nx) >= abs(ny)
        if vertical:
            na, nb, qa, qb, a0, b0, Nb = nx, ny, bd["x"][p], bd["y"][p], grid.x0, grid.y0, grid.ny
        else:
            na, nb, qa, qb, a0, b0, Nb = ny, nx, bd["y"][p], bd["x"][p], grid.y0, grid.x0, grid.nx
        u = (qa - a0) / h
        if na > 0:
            i_first, step = math.floor(u), -1
        else:
            i_first, step = math.ceil(u), 1
        for s in range(2 * M):
            i_s = i_first + step * s
            a_s = a0 + i_s * h
            delta = (LD(qa) - LD(a_s)) / LD(na)
            bstar = LD(qb) - delta * LD(nb)
            jb = math.floor((float(bstar) - b0) / h)

            def c_at(j):
                if j < 0 or j >= Nb:
                    return FAR
                return cls[i_s, j] if vertical else cls[j, i_s]

            lower, upper = [], []
            if not pl.interior_only and delta < LD(STAR_MIN_DEPTH) * LD(h) / LD(abs(na)):
                # too close to the point on Gamma (itself a node along the normal)
                star_rec.append((p, vertical, i_s, delta, bstar))
                runs.append([[], [], None, None])
                continue
            j = jb
            while j >= jb - M and c_at(j) == IN:
                lower.append(j)
                j -= 1
            lo_stop = j if (j >= jb - M) else None
            j = jb + 1
            while j <= jb + 1 + M and c_at(j) == IN:
                upper.append(j)
                j += 1
            hi_stop = j if (j <= jb + 1 + M) else None
            rid = len(star_rec)
            star_rec.append((p, vertical, i_s, delta, bstar))
            runs.append([lower, upper, None, None])
            if pl.interior_only:
                continue          # no boundary samples: IN nodes only
            if lo_stop is not None:
                b_in = (b0 + (lo_stop + 1) * h) if lower else float(bstar)
                sq_req.append((rid, 0, vertical, a_s, b_in, b0 + lo_stop * h))
            if hi_stop is not None:
                b_in = (b0 + (hi_stop - 1) * h) if upper else float(bstar)
                sq_req.append((rid, 1, vertical, a_s, b_in, b0 + hi_stop * h))
    # phase 2: crossings with Gamma by bisection, all at once
    if sq_req:
        req = np.array([(r[2], r[3], r[4], r[5]) for r in sq_req], dtype=np.float64)
        bsq = _bisect_crossing(pl, req[:, 0] > 0.5, req[:, 1], req[:, 2], req[:, 3])
    else:
        bsq = np.zeros(0)
    for (rid, side, vertical, a_s, b_in, b_out), b in zip(sq_req, bsq):
        b0 = grid.y0 if vertical else grid.x0
        nodes = runs[rid][0] + runs[rid][1]
        if any(abs(b - (b0 + j * h)) < 0.5 * h for j in nodes):
            continue              # closer than h/2 to an IN node: dropped
        runs[rid][2 + side] = b
    # phase 3: per normal, the first M - 1 stars (M from interior data only)
    # whose line offers >= M nodes; the M nodes nearest each star; weights in
    # longdouble.  With boundary data, star slot M - 1 is the point on Gamma
    # (depth 0): its value is the boundary sample, its stencil unused.
    nstar = M if pl.interior_only else M - 1
    nref = np.zeros((B, M, M), dtype=np.int64)
    wv = np.zeros((B, M, M), dtype=LD)
    deltas = np.zeros((B, M), dtype=LD)
    pl.vertical = np.zeros(B, dtype=bool)
    sq_xy = []
    rid = 0
    for p in range(B):
        used = 0
        for s in range(2 * M):
            _, vertical, i_s, delta, bstar = star_rec[rid + s]
            lower, upper, sqlo, sqhi = runs[rid + s]
            if used == nstar or len(lower) + len(upper) + (sqlo is not None) + (sqhi is not None) < M:
                continue
            b0 = grid.y0 if vertical else grid.x0
            lo_list = [("g", j, b0 + j * h) for j in lower] + ([("s", None, sqlo)] if sqlo is not None else [])
            hi_list = [("g", j, b0 + j * h) for j in upper] + ([("s", None, sqhi)] if sqhi is not None else [])
            chosen = []
            a = b = 0
            bs = float(bstar)
            while len(chosen) < M:
                if a < len(lo_list) and b < len(hi_list):
                    dl = bs - lo_list[a][2]
                    du = hi_list[b][2] - bs
                    if dl < du or (dl == du and not (lo_list[a][0] == "s" and hi_list[b][0] == "g")):
                        chosen.append(lo_list[a]); a += 1
                    else:
                        chosen.append(hi_list[b]); b += 1
                elif a < len(lo_list):
                    chosen.append(lo_list[a]); a += 1
                else:
                    chosen.append(hi_list[b]); b += 1
            pos = np.array([LD(c[2]) for c in chosen], dtype=LD)
            wv[p, used] = lagrange_weights(pos, bstar)
            for k, c in enumerate(chosen):
                if c[0] == "g":
                    nref[p, used, k] = (i_s * grid.ny + c[1]) if vertical else (c[1] * grid.ny + i_s)
                else:
                    nref[p, used, k] = -(1 + len(sq_xy))
                    a_s = (grid.x0 if vertical else grid.y0) + i_s * h
                    sq_xy.append((a_s, c[2]) if vertical else (c[2], a_s))
            deltas[p, used] = delta
            used += 1
        if used < nstar:
            raise GeometryError("matching stencil: too few usable red stars at normal %d" % p)
        if nstar < M:        # the point on Gamma; placeholder stencil (star 0's nodes, zero weights)
            nref[p, M - 1] = nref[p, 0]
            deltas[p, M - 1] = 0
        pl.vertical[p] = vertical
        rid += 2 * M
    pl.squares = np.array(sq_xy, dtype=np.float64).reshape(-1, 2)
    nq = d if pl.interior_only else d - 1     # matching values interpolated along the normal
    depth = np.array([LD(d - 1 - q) * LD(pl.k1) for q in range(nq)], dtype=LD)
    wn = lagrange_weights(np.broadcast_to(deltas[:, None, :], (B, nq, M)).copy(),
                          np.broadcast_to(depth[None, :], (B, nq)).copy())
    pl.match_ref = nref
    pl.match_wv = wv
    pl.match_wn = wn
    pl.match_delta = deltas


def boundary_points(pl):
    """Ordered list of boundary points whose f values extension needs: the B
    feet q(theta_p) first, then the squares."""
    feet = np.stack([pl.bd["x"], pl.bd["y"]], axis=1)
    return np.concatenate([feet, pl.squares], axis=0)


def proximity_map(pl):
    """Literal proximity map of Sec. 3.3 over V+_{B,C_r}: every curvilinear
    point s_{p,q} is associated with its nearest Cartesian point; a Cartesian
    point claimed several times keeps the nearest curvilinear point (ties to
    the smallest (p, q)); STRIP points left without a partner take the nearest
    curvilinear partner of their 8 neighbours.  Returns p for each STRIP point
    (-1 if none)."""
    grid, bd = pl.grid, pl.bd
    q = np.arange(pl.Cr + 1)
    sx = bd["x"][:, None] + bd["nx"][:, None] * (q[None, :] * pl.k1 / pl.n_r)
    sy = bd["y"][:, None] + bd["ny"][:, None] * (q[None, :] * pl.k1 / pl.n_r)
    ii = np.rint((sx - grid.x0) / grid.h).astype(np.int64)
    jj = np.rint((sy - grid.y0) / grid.h).astype(np.int64)
    ok = (ii >= 0) & (ii < grid.nx) & (jj >= 0) & (jj < grid.ny)
    pp = np.broadcast_to(np.arange(pl.B)[:, None], sx.shape)
    qq = np.broadcast_to(q[None, :], sx.shape)
    d2 = (sx - (grid.x0 + ii * grid.h)) ** 2 + (sy - (grid.y0 + jj * grid.h)) ** 2
    flat = (ii * grid.ny + jj)[ok]
    order = np.lexsort((qq[ok], pp[ok], d2[ok], flat))
    flat_s = flat[order]
    first = np.ones(flat_s.size, dtype=bool)
    first[1:] = flat_s[1:] != flat_s[:-1]
    partner = np.full(grid.nx * grid.ny, -1, dtype=np.int64)
    partner_xy = np.zeros((grid.nx * grid.ny, 2))
    partner[flat_s[first]] = pp[ok][order][first]
    partner_xy[flat_s[first], 0] = sx[ok][order][first]
    partner_xy[flat_s[first], 1] = sy[ok][order][first]
    out = partner[pl.strip_idx].copy()
    for k in np.nonzero(out < 0)[0]:
        f = pl.strip_idx[k]
        i, j = divmod(int(f), grid.ny)
        X, Y = grid.x0 + i * grid.h, grid.y0 + j * grid.h
        best = None
        for di in (-1, 0, 1):
            for dj in (-1, 0, 1):
                a, b = i + di, j + dj
                if (di or dj) and 0 <= a < grid.nx and 0 <= b < grid.ny and partner[a * grid.ny + b] >= 0:
                    pq = partner[a * grid.ny + b]
                    for dp in (-1, 0, 1):
                        pp2 = (pq + dp) % pl.B
                        dd = (bd["x"][pp2] - X) ** 2 + (bd["y"][pp2] - Y) ** 2
                        if best is None or dd < best[0]:
                            best = (dd, pp2)
        out[k] = -1 if best is None else best[1]
    return out
