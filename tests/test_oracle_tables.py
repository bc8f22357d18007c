"""Pins for the oracle's FC-Gram tables (Sec. 2.2, Remark 2.2) against what the
paper and the mathematics fix: orthonormal Gram values, polynomial structure,
fit quality, vanishing continuation and O(k^d) convergence of the 1D-FC."""
import numpy as np
import pytest

from oracle import fc1d, fcgram


@pytest.fixture(scope="module", params=[4, 5, 10, 12])
def tab(request):
    return fcgram.load_tables(d=request.param)


def test_gram_orthonormal_and_triangular(tab):
    Q = tab["Q"]
    d = Q.shape[0]
    # columns are orthonormal for the discrete scalar product on x_j = j
    assert np.allclose(Q.T @ Q, np.eye(d), atol=1e-14)
    # P = Q R with R upper triangular and R_ii > 0 (eq. pqr_factr, Gram-Schmidt order)
    P = np.vander(np.arange(d, dtype=float), d, increasing=True)
    R = Q.T @ P
    assert np.allclose(np.tril(R, -1), 0.0, atol=1e-11 * np.abs(R).max())
    assert np.all(np.diag(R) > 0)
    assert np.allclose(Q @ R, P, atol=1e-12 * np.abs(P).max())


def test_gram_columns_are_polynomials(tab):
    """Column j holds the values of a degree-j polynomial: its (j+1)-th finite
    difference vanishes."""
    Q = tab["Q"]
    for j in range(Q.shape[0] - 1):
        assert np.abs(np.diff(Q[:, j], n=j + 1)).max() < 1e-13


def test_table_file_metadata():
    t = fcgram.load_tables(d=5)
    assert (t["d"], t["C"], t["Z"], t["n_os"], t["n_r"], t["mf"]) == (5, 27, 12, 20, 6, 20)
    assert t["A"].shape == (27, 5) and t["Ar"].shape == (162, 5)


def test_refined_matrix_contains_unrefined(tab):
    """A_r at the fine points (d-1) + l/n_r includes the unrefined points d..d+C-1
    (l = n_r, 2 n_r, ...): those rows must equal A (Remark 2.2)."""
    A, Ar = tab["A"], tab["Ar"]
    n_r = Ar.shape[0] // A.shape[0]
    assert np.allclose(Ar[n_r - 1::n_r], A, rtol=0, atol=1e-12 * np.abs(A).max())


def test_continuation_of_constants_blends_to_zero(tab):
    """A constant vector blends smoothly to (nearly) zero at the end of the
    continuation interval (Sec. 3.1: vanishing at q = C_r)."""
    Q, Ar = tab["Q"], tab["Ar"]
    d = Q.shape[0]
    F = Ar @ (Q.T @ np.ones(d))
    assert abs(F[0] - 1.0) < 0.2          # first fine point next to the data
    # last continuation point: it lies before the zero-matching interval, so it
    # is small by smoothness, not fitted to zero (1.3e-9 measured at d = 12)
    assert abs(F[-1]) < (1e-9 if d <= 5 else 1e-8)


def test_continuation_matches_polynomials_near_boundary(tab):
    """Data of a polynomial of degree < d is continued by its trigonometric fit:
    just past the matching interval the continuation stays close to the polynomial."""
    Q, Ar = tab["Q"], tab["Ar"]
    d = Q.shape[0]
    n_r = Ar.shape[0] // tab["A"].shape[0]
    x = np.arange(d, dtype=float)
    for deg in range(d):
        phi = (x / (d - 1)) ** deg
        F = Ar @ (Q.T @ phi)
        # one fine step past the last matching point
        xe = (d - 1) + 1.0 / n_r
        assert abs(F[0] - (xe / (d - 1)) ** deg) < 0.05


def _phi(x):
    return np.exp(np.sin(5.4 * np.pi * x - 2.7 * np.pi) - np.cos(2 * np.pi * x)) - np.sin(2.5 * np.pi * x) + 1.0


def test_fc1d_converges_at_order_d(tab):
    """1D-FC of Fig. 1's function converges as O(k^d) (Sec. 2.3)."""
    Q, A = tab["Q"], tab["A"]
    d = Q.shape[0]
    xe = np.linspace(0.0, 1.0, 2001)
    errs = []
    Ns = [101, 201, 401]
    for N in Ns:
        x = np.linspace(0.0, 1.0, N)
        v = fc1d.fc1d_eval(_phi(x), Q, A, xe)
        errs.append(np.abs(v - _phi(xe)).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < 1e-5
    # order d over each halving, unless the error has reached the rounding
    # floor (d = 10, 12 reach about 1e-13 at N = 401)
    assert orders[0] > d - 0.8, (errs, orders)
    assert orders[-1] > d - 0.8 or errs[-1] < 1e-11, (errs, orders)


def test_fc1d_interpolates_data(tab):
    Q, A = tab["Q"], tab["A"]
    x = np.linspace(0.0, 1.0, 101)
    v = fc1d.fc1d_eval(_phi(x), Q, A, x)
    assert np.abs(v - _phi(x)).max() < 1e-12
