"""FC-Gram blending-to-zero tables (oracle side).

Follows Sec. 2.2 of Bruno & Paul (arXiv 2010.03901) and Remark 2.2:

* Gram polynomials on the d equispaced matching points x_j = j k (the tables
  do not depend on k, end of Sec. 2.3, so k = 1 here): QR factorisation
  P = Q R of the Vandermonde matrix P_ij = x_i^j (eq. pqr_factr) obtained by
  the stabilised (modified) Gram-Schmidt process, with R_ii > 0.
* Oversampled Gram values Q_os = P_os R^{-1} on the n_os(d-1)+1 points of
  step k/n_os in [0, (d-1)k] (eq. q_over).
* For each Gram column, a band-limited trigonometric polynomial of period
  (d + 2C + Z - 1) k (eq. auxi_trig_poly) fitted in the least-squares sense,
  by an SVD, to the oversampled Gram values and to zeros on the k/n_os-spaced
  points of the zero-matching interval [(d+C)k, (d+C+Z-1)k] (eq. min_prob).
* Continuation matrix A (C x d): the fitted polynomials at the C points
  x = d, ..., d+C-1 (eq. b_to_z).  Refined matrix A_r (C_r x d, C_r = n_r C):
  the fitted polynomials at the fine points (d-1) + l/n_r, l = 1..C_r, of
  ((d-1)k, (d+C-1)k] (Remark 2.2).

The band limit of the trigonometric basis is not given a value in the paper
(its letter clashes with the interpolation degree); it is the parameter
``mf`` here, recorded in the table file.  With mf = 20 the least-squares
matrix has a condition number near 4e15, so the fit is computed in mpmath
with 50 significant digits and only the final Q, A and A_r are rounded to
float64.
"""
from __future__ import annotations

import os

import mpmath as mp
import numpy as np

DATA_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")


def _gram_schmidt_qr(P):
    """Stabilised (modified) Gram-Schmidt QR of a square mpmath matrix, R_ii > 0."""
    n = P.rows
    V = P.copy()
    Q = mp.matrix(n, n)
    R = mp.matrix(n, n)
    for j in range(n):
        R[j, j] = mp.sqrt(mp.fsum(V[i, j] ** 2 for i in range(n)))
        for i in range(n):
            Q[i, j] = V[i, j] / R[j, j]
        for k in range(j + 1, n):
            R[j, k] = mp.fsum(Q[i, j] * V[i, k] for i in range(n))
            for i in range(n):
                V[i, k] -= R[j, k] * Q[i, j]
    return Q, R


def _trig_row(x, mf, period):
    """Real form of the basis of eq. auxi_trig_poly: 1, cos(2 pi m x / T), sin(2 pi m x / T)."""
    row = [mp.mpf(1)]
    for m in range(1, mf + 1):
        a = 2 * mp.pi * m * x / period
        row.append(mp.cos(a))
        row.append(mp.sin(a))
    return row


def compute_tables(d=5, C=27, Z=12, n_os=20, n_r=6, mf=20, dps=50):
    """Compute Q, A, A_r for the given FC-Gram parameters (slow: tens of seconds).

    Returns a dict with float64 arrays 'Q' (d x d), 'A' (C x d), 'Ar'
    (n_r C x d) and diagnostics.
    """
    with mp.workdps(dps):
        x = [mp.mpf(j) for j in range(d)]
        P = mp.matrix([[xi ** j for j in range(d)] for xi in x])
        Q, R = _gram_schmidt_qr(P)
        x_os = [mp.mpf(j) / n_os for j in range(n_os * (d - 1) + 1)]
        P_os = mp.matrix([[xi ** j for j in range(d)] for xi in x_os])
        Q_os = P_os * mp.inverse(R)
        x_zero = [mp.mpf(d + C) + mp.mpf(j) / n_os for j in range(n_os * (Z - 1) + 1)]
        period = mp.mpf(d + 2 * C + Z - 1)
        B_os = mp.matrix([_trig_row(xi, mf, period) for xi in x_os + x_zero])
        # SVD-based least squares (eq. min_prob): a = V^T diag(1/s) U^T rhs.
        U, S, V = mp.svd_r(B_os, full_matrices=False, compute_uv=True)
        ncoef = 2 * mf + 1
        x_A = [mp.mpf(j) for j in range(d, d + C)]
        x_Ar = [mp.mpf(d - 1) + mp.mpf(l) / n_r for l in range(1, C * n_r + 1)]
        E_A = mp.matrix([_trig_row(xi, mf, period) for xi in x_A])
        E_Ar = mp.matrix([_trig_row(xi, mf, period) for xi in x_Ar])
        A = np.zeros((C, d))
        Ar = np.zeros((C * n_r, d))
        resid = []
        for j in range(d):
            rhs = mp.matrix([Q_os[i, j] for i in range(len(x_os))] + [0] * len(x_zero))
            Ut_rhs = U.T * rhs
            a = V.T * mp.matrix([Ut_rhs[i] / S[i] for i in range(ncoef)])
            r = B_os * a - rhs
            resid.append(float(max(abs(v) for v in r)))
            A[:, j] = [float(v) for v in E_A * a]
            Ar[:, j] = [float(v) for v in E_Ar * a]
        Qf = np.array([[float(Q[i, j]) for j in range(d)] for i in range(d)])
        cond = float(max(S) / min(S))
    return {
        "d": d, "C": C, "Z": Z, "n_os": n_os, "n_r": n_r, "mf": mf, "dps": dps,
        "Q": Qf, "A": A, "Ar": Ar, "residuals": resid, "cond": cond,
    }


def table_path(d=5, C=27, Z=12, n_os=20, n_r=6, mf=20):
    return os.path.join(DATA_DIR, f"fcgram_d{d}_C{C}_Z{Z}_os{n_os}_r{n_r}_mf{mf}.txt")


def write_tables(t, path):
    with open(path, "w") as fh:
        fh.write("# FC-Gram tables written by oracle/make_tables.py (mpmath, %d digits)\n" % t["dps"])
        fh.write("# d C Z n_os n_r mf\n%d %d %d %d %d %d\n" % (t["d"], t["C"], t["Z"], t["n_os"], t["n_r"], t["mf"]))
        fh.write("# cond(B_os) %.3e ; max fit residual per Gram column: %s\n"
                 % (t["cond"], " ".join("%.3e" % r for r in t["residuals"])))
        for name in ("Q", "A", "Ar"):
            M = t[name]
            fh.write("# %s %d %d\n" % (name, M.shape[0], M.shape[1]))
            for row in M:
                fh.write(" ".join("%.17e" % v for v in row) + "\n")


def load_tables(d=5, C=27, Z=12, n_os=20, n_r=6, mf=20):
    """Load the stored tables; raises FileNotFoundError when they were never generated."""
    path = table_path(d, C, Z, n_os, n_r, mf)
    with open(path) as fh:
        lines = [ln.strip() for ln in fh if ln.strip()]
    out = {}
    i = 0
    while i < len(lines):
        ln = lines[i]
        if ln.startswith("# d C Z"):
            vals = [int(v) for v in lines[i + 1].split()]
            out.update(dict(zip(("d", "C", "Z", "n_os", "n_r", "mf"), vals)))
            i += 2
            continue
        if ln.startswith("# ") and ln.split()[1] in ("Q", "A", "Ar") and len(ln.split()) == 4:
            _, name, nr, nc = ln.split()
            nr, nc = int(nr), int(nc)
            out[name] = np.array([[float(v) for v in lines[i + 1 + r].split()] for r in range(nr)])
            assert out[name].shape == (nr, nc)
            i += 1 + nr
            continue
        i += 1
    return out
