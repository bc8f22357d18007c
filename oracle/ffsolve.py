"""Fourier Forwarding solver of the wave equation (Sec. 4.2), oracle side.

Test infrastructure: plain NumPy in float64, written from the paper's
description; shares no code with the HIP library.

Problem (eq. wave_2d): u_tt = c^2 (u_xx + u_yy) in Omega, u = b(x, y, t) on
Gamma (Dirichlet data), u = f and u_t = g at t = 0.  One large step
[T_j, T_j + dT] of eq. ff_soln:

1. U_FC (eq. aux_sol): the 2D-FC extensions of u(T_j) and u_t(T_j) (the
   boundary samples taken from the Dirichlet data b and b_t at T_j), their
   FFTs, and every mode advanced in closed form (eq. wave_2d_ff).  U_FC is
   the solution wherever the disc of radius c (t - T_j) lies inside Omega.
2. U_B: on the grid points of the boundary region the solution is stepped
   with the small step dt (CFL 0.125, Sec. 4.2.1) from its own values at
   T_j, spatial derivatives by the 1D-FC of Sec. 2.3 (both blends) along
   grid lines; the Dirichlet condition enters at the grid points next to
   Gamma by interpolation along the grid line from the value at the
   crossing of that line with Gamma; values needed farther inside come from
   U_FC at the current time, evaluated directly (an inverse FFT of the
   propagated spectrum).
3. The combination (eq. ff_soln): U_B on the boundary region, U_FC elsewhere.

Readings (the paper sketches FF and defers its details to a later paper):

* Boundary region: IN grid points within Chebyshev grid distance n_B = n_c + 2
  of a non-IN grid point; dT = n_c h / c, so every other IN point lies at
  least c dT from Gamma (checked by the tests).  n_c = 6 as in Ex. 4.4.
* Small step: dt = dT / ceil(n_c / 0.125) (CFL 0.125).  The "second order
  Taylor series" update: u^{n+1} = u^n + dt v^n + dt^2 / 2 a^n,
  v^{n+1} = v^n + dt (a^n + a^{n+1}) / 2 (velocity form of the second-order
  Taylor step; a = c^2 Delta u).
* Boundary points of U_B: boundary-region points adjacent, along x or y, to
  a non-IN grid point.  Their u (and v) at each new time level is the
  degree-(M_b - 1) Lagrange interpolant along that grid line (the direction
  with the longer IN run when both qualify, x on ties) from the crossings of
  the line with Gamma that bound the run (data b, resp. b_t) and the stepped
  points of the run: the M_b nodes nearest the point (ties: lower position).
  M_b = 4 (a cubic closure).  The closure makes the stepper only
  conditionally useful: with the boundary points held at the exact solution
  the stepper is stable (unit disc, 512^2, 1600 small steps), with the
  interpolation closure its error grows, the faster the finer the grid; 2, 3,
  5 or more nodes, or nodes two grid steps apart, grow faster than 4.  The
  paper leaves its closure to a later paper.
* Stepped points: the other boundary-region points.  For each grid line the
  stepped points form sub-runs of the IN runs; the 1D-FC segment of a
  sub-run extends it by n_o = d points on each side, clipped to the IN run,
  and widened to at least 2 d points.  Values on a segment: stepped and
  boundary points from U_B, any other point from U_FC(t).  An IN run with
  fewer than 2 d points takes the second derivative of the Lagrange
  interpolant through its points and the two crossings bounding it (a
  crossing within h/2 of the run's end point is left out).
* 1D-FC second derivative of a segment of n equispaced values: the
  continuation (eq. fc_1d_cont) of length n + C with both blends, its DFT,
  the factor -(2 pi m / ((n + C) h))^2 per mode m in (-(n+C)/2, (n+C)/2],
  the inverse DFT, the first n values.
"""
from __future__ import annotations

import math

import numpy as np

from . import extend as E
from . import spectral as S
from .fc1d import fc1d_continuation
from .interp import lagrange_weights
from .plan import IN, _bisect_crossing, boundary_points


# ---------------------------------------------------------------------------
# derivative operators along one grid line
# ---------------------------------------------------------------------------
def fc1d_d2(vals, h, Q, A):
    """Second derivative of the 1D-FC trigonometric polynomial (Sec. 2.3) of
    equispaced vals (step h) at the data points."""
    pc = fc1d_continuation(np.asarray(vals, dtype=np.float64), Q, A)
    P = pc.size
    m = np.fft.fftfreq(P, d=1.0 / P)              # integer mode numbers
    if P % 2 == 0:
        m[P // 2] = P // 2                          # (-(P/2), P/2]: the Nyquist mode is +P/2
    k = 2.0 * math.pi * m / (P * h)
    return np.real(np.fft.ifft(-(k * k) * np.fft.fft(pc)))[: len(vals)]


def lagrange_d2_weights(nodes, x):
    """Weights w with sum_k w_k v_k = p''(x), p the interpolant of (nodes, v)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    n = nodes.size
    w = np.zeros(n)
    for k in range(n):
        others = np.delete(nodes, k)
        den = np.prod(nodes[k] - others)
        # second derivative of prod_{j != k} (x - x_j): sum over ordered pairs (a, b), a != b
        s = 0.0
        for a in range(n - 1):
            for b in range(n - 1):
                if a == b:
                    continue
                rest = [others[j] for j in range(n - 1) if j != a and j != b]
                s += np.prod([x - r for r in rest]) if rest else 1.0
        w[k] = s / den
    return w


# ---------------------------------------------------------------------------
# set-up: boundary region, crossings, boundary points, segments
# ---------------------------------------------------------------------------
class FFSetup:
    pass


def _runs(mask_line):
    """(start, end) inclusive index pairs of the True runs of a 1D boolean array."""
    idx = np.flatnonzero(mask_line)
    if idx.size == 0:
        return []
    br = np.flatnonzero(np.diff(idx) > 1)
    starts = np.concatenate([[idx[0]], idx[br + 1]])
    ends = np.concatenate([idx[br], [idx[-1]]])
    return list(zip(starts.tolist(), ends.tolist()))


def make_setup(pl, c=1.0, n_c=6, cfl=0.125, M_b=4, n_o=None):
    """Boundary region, crossings, interpolation and derivative stencils of
    the U_B solver on the plan's grid (pl from plan.make_plan)."""
    g = pl.grid
    nx, ny, h = g.nx, g.ny, g.h
    d = pl.d
    st = FFSetup()
    st.pl, st.c, st.n_c = pl, float(c), int(n_c)
    st.M_b = int(M_b)
    st.n_o = d if n_o is None else int(n_o)
    st.dT = n_c * h / c
    st.K = int(math.ceil(n_c / cfl - 1e-12))
    st.dt = st.dT / st.K
    inside = pl.cls == IN
    st.inside = inside
    # boundary region: Chebyshev grid distance <= n_B from a non-IN point
    n_B = n_c + 2
    st.n_B = n_B
    out = ~inside
    near = np.zeros_like(out)
    pad = np.pad(out, n_B, constant_values=True)
    for di in range(-n_B, n_B + 1):
        for dj in range(-n_B, n_B + 1):
            near |= pad[n_B + di: n_B + di + nx, n_B + dj: n_B + dj + ny]
    st.ub = inside & near
    # runs of IN points along x-lines (axis 0 index i varies, j fixed) and y-lines
    # line (ax, k): ax = 0 -> the line y = y_k (points (i, k)); ax = 1 -> x = x_k (points (k, j))
    st.runs = {0: [_runs(inside[:, j]) for j in range(ny)], 1: [_runs(inside[i, :]) for i in range(nx)]}
    # crossings bounding every run: [ax, line, pos (continuous index along the line)]
    cross = {}
    req = []
    for ax in (0, 1):
        for line, rl in enumerate(st.runs[ax]):
            for (a, b) in rl:
                for end, outn in ((a, a - 1), (b, b + 1)):
                    req.append((ax, line, end, outn))
    req = np.array(req, dtype=np.int64).reshape(-1, 4)
    if req.size:
        # crossing position by bisection on the sign of eta between the IN end and its outside neighbour
        ax_is_x = req[:, 0] == 1                      # ax = 1: x fixed at x_line, bisect in y
        a_line = np.where(ax_is_x, g.x0 + req[:, 1] * h, g.y0 + req[:, 1] * h)
        base = np.where(ax_is_x, g.y0, g.x0)
        pos = _bisect_crossing(pl, ax_is_x, a_line, base + req[:, 2] * h, base + req[:, 3] * h)
        for r, p in zip(req, pos):
            cross[(int(r[0]), int(r[1]), int(r[2]), int(r[3]))] = (float(p) - (g.y0 if r[0] == 1 else g.x0)) / h
    st.cross = cross                                   # (ax, line, end, out) -> crossing position / h
    st.cross_list = list(cross.keys())
    st.cross_index = {k: n for n, k in enumerate(st.cross_list)}
    cp = np.array([cross[k] for k in st.cross_list]) if cross else np.zeros(0)
    st.cross_xy = np.zeros((len(st.cross_list), 2))
    for n, (ax, line, end, outn) in enumerate(st.cross_list):
        if ax == 0:
            st.cross_xy[n] = (g.x0 + cp[n] * h, g.y0 + line * h)
        else:
            st.cross_xy[n] = (g.x0 + line * h, g.y0 + cp[n] * h)

    def run_of(ax, i, j):
        line, p = (j, i) if ax == 0 else (i, j)
        for (a, b) in st.runs[ax][line]:
            if a <= p <= b:
                return line, p, a, b
        raise AssertionError

    # boundary points of U_B and their interpolation direction
    bnd = np.zeros_like(inside)
    bdir = {}
    for i, j in zip(*np.nonzero(st.ub)):
        ends = []
        for ax in (0, 1):
            line, p, a, b = run_of(ax, i, j)
            if p == a or p == b:
                ends.append((b - a + 1, -ax, ax))
        if ends:
            bnd[i, j] = True
            bdir[(i, j)] = max(ends)[2]                # longer run first, x (ax = 0) on ties
    st.bnd = bnd
    st.stepped = st.ub & ~bnd
    # interpolation stencils of the boundary points
    st.bstencil = {}
    for (i, j), ax in bdir.items():
        line, p, a, b = run_of(ax, i, j)
        cand = [(float(q), ("grid", q)) for q in range(a, b + 1)
                if (st.stepped[q, line] if ax == 0 else st.stepped[line, q])]
        cand.append((st.cross[(ax, line, a, a - 1)], ("cross", st.cross_index[(ax, line, a, a - 1)])))
        cand.append((st.cross[(ax, line, b, b + 1)], ("cross", st.cross_index[(ax, line, b, b + 1)])))
        cand.sort(key=lambda t: (abs(t[0] - p), t[0]))
        nodes = cand[: st.M_b]
        wts = lagrange_weights(np.array([[t[0] for t in nodes]]), np.array([float(p)]))[0]
        refs = []
        for _, (kind, q) in nodes:
            if kind == "grid":
                refs.append(("grid", (q, line) if ax == 0 else (line, q)))
            else:
                refs.append(("cross", q))
        st.bstencil[(i, j)] = (refs, wts)
    # derivative segments of the stepped points
    st.segments = []     # (ax, line, lo, hi, kind): FC over [lo, hi], or Lagrange ('lag') over the run
    for ax in (0, 1):
        for line, rl in enumerate(st.runs[ax]):
            for (a, b) in rl:
                sel = [q for q in range(a, b + 1) if (st.stepped[q, line] if ax == 0 else st.stepped[line, q])]
                if not sel:
                    continue
                if b - a + 1 < 2 * d:
                    # Lagrange through the crossings and the run points
                    # (a crossing closer than h/2 to the run's end point is left out: the end
                    # point then lies on Gamma to within h/2 and its value stands for it)
                    xa = st.cross[(ax, line, a, a - 1)]
                    xb = st.cross[(ax, line, b, b + 1)]
                    ca = st.cross_index[(ax, line, a, a - 1)] if a - xa >= 0.5 else -1
                    cb = st.cross_index[(ax, line, b, b + 1)] if xb - b >= 0.5 else -1
                    nodes = np.concatenate([[xa] if ca >= 0 else [], np.arange(a, b + 1, dtype=np.float64),
                                            [xb] if cb >= 0 else []])
                    wl = {p: lagrange_d2_weights(nodes, float(p)) for p in sel}
                    st.segments.append((ax, line, a, b, "lag", (sel, wl, ca, cb)))
                    continue
                for (s0, s1) in _runs(np.isin(np.arange(a, b + 1), sel)):
                    s0 += a
                    s1 += a
                    lo, hi = max(a, s0 - st.n_o), min(b, s1 + st.n_o)
                    while hi - lo + 1 < 2 * d:
                        if lo > a:
                            lo -= 1
                        if hi - lo + 1 < 2 * d and hi < b:
                            hi += 1
                    st.segments.append((ax, line, lo, hi, "fc", list(range(s0, s1 + 1))))
    return st


# ---------------------------------------------------------------------------
# one large step
# ---------------------------------------------------------------------------
def _accel(st, u, bvals):
    """c^2 (u_xx + u_yy) at the stepped points (0 elsewhere); u holds valid
    values at every grid point a segment reads, bvals the data at the
    crossings (read by the Lagrange form of short runs)."""
    pl = st.pl
    h = pl.grid.h
    Q, A = pl.Q, _table_A(pl)
    a = np.zeros_like(u)
    for ax, line, lo, hi, kind, pts in st.segments:
        vals = u[lo:hi + 1, line] if ax == 0 else u[line, lo:hi + 1]
        if kind == "fc":
            d2 = fc1d_d2(vals, h, Q, A)
            for p in pts:
                if ax == 0:
                    a[p, line] += d2[p - lo]
                else:
                    a[line, p] += d2[p - lo]
        else:
            sel, wl, ca, cb = pts
            vv = np.concatenate([[bvals[ca]] if ca >= 0 else [], vals, [bvals[cb]] if cb >= 0 else []])
            for p in sel:
                val = float(wl[p] @ vv) / (h * h)
                if ax == 0:
                    a[p, line] += val
                else:
                    a[line, p] += val
    return (st.c ** 2) * a


def _table_A(pl):
    """The unrefined continuation matrix A (C x d): rows n_r, 2 n_r, ... of A_r."""
    return pl.Ar[pl.n_r - 1:: pl.n_r]


def _apply_bc(st, u, bvals):
    """Boundary points of U_B: interpolation along their grid line from the
    crossing values bvals [n_cross] and the stepped points."""
    for (i, j), (refs, wts) in st.bstencil.items():
        s = 0.0
        for (kind, r), w in zip(refs, wts):
            s += w * (u[r] if kind == "grid" else bvals[r])
        u[i, j] = s


def advance(st, u, ut, t0, bfun, btfun, nsmall=None):
    """One large step from T_j = t0: (u, u_t) on the grid (IN points) ->
    (u, u_t) at t0 + nsmall dt (nsmall = K small steps by default: the whole
    large step dT; eq. ff_soln holds at every time of the interval).
    bfun(x, y, t), btfun(x, y, t): Dirichlet data and its time derivative.
    Returns (u, ut); entries outside Omega are 0."""
    pl = st.pl
    g = pl.grid
    c = st.c
    bp = boundary_points(pl)
    U = S.fft2_forward(E.extend(pl, u, bfun(bp[:, 0], bp[:, 1], t0)))
    Ut = S.fft2_forward(E.extend(pl, ut, btfun(bp[:, 0], bp[:, 1], t0)))

    def ufc(t):
        a, at = S.ff_propagate(U, Ut, g.nx, g.ny, g.h, c, t - t0)
        return S.fft2_inverse(a, g.ny), S.fft2_inverse(at, g.ny)

    cx, cy = st.cross_xy[:, 0], st.cross_xy[:, 1]
    ub = st.ub
    uB = np.where(st.inside, u, 0.0)
    vB = np.where(st.inside, ut, 0.0)
    acc = _accel(st, uB, bfun(cx, cy, t0))                               # every IN value of u(T_j) is valid at t0
    dt = st.dt
    nsmall = st.K if nsmall is None else int(nsmall)
    for k in range(1, nsmall + 1):
        t = t0 + k * dt
        uF, _ = ufc(t)
        un = np.where(st.stepped, uB + dt * vB + 0.5 * dt * dt * acc, 0.0)
        # values read by the segments: U_B on the boundary region, U_FC elsewhere
        work = np.where(ub, un, np.where(st.inside, uF, 0.0))
        bv = bfun(cx, cy, t)
        _apply_bc(st, work, bv)
        acc_n = _accel(st, work, bv)
        vn = np.where(st.stepped, vB + 0.5 * dt * (acc + acc_n), 0.0)
        _apply_bc(st, vn, btfun(cx, cy, t))
        uB = np.where(ub, work, 0.0)
        vB = np.where(ub, vn, 0.0)
        acc = acc_n
    uF, utF = ufc(t0 + nsmall * dt)
    u_new = np.where(ub, uB, np.where(st.inside, uF, 0.0))
    ut_new = np.where(ub, vB, np.where(st.inside, utF, 0.0))
    return u_new, ut_new
