// FC-Gram blending-to-zero tables in binary128 (__float128) arithmetic.
//
// Sec. 2.2 and Remark 2.2 of Bruno & Paul (arXiv 2010.03901):
//   * Gram polynomials on the d matching points x_j = j (the tables do not
//     depend on the step k): P = Q R, P_ij = x_i^j, by modified (stabilised)
//     Gram-Schmidt with R_ii > 0 (eq. pqr_factr);
//   * oversampled values Q_os = P_os R^{-1} on x = j / n_os (eq. q_over);
//   * per Gram column, the least-squares trigonometric polynomial of period
//     d + 2C + Z - 1 matching Q_os on [0, d-1] and 0 on the k/n_os points of
//     [d+C, d+C+Z-1] (eq. auxi_trig_poly, eq. min_prob).  The paper solves it by
//     an SVD; the problem has full column rank, so the Householder-QR solution
//     used here is the same minimiser;
//   * A: the fit at x = d .. d+C-1 (eq. b_to_z); A_r: the fit at the refined
//     points (d-1) + l/n_r, l = 1..n_r C (Remark 2.2).
// The least-squares matrix has condition number ~4e15 at band limit 20, so the
// fit is done with a 113-bit significand and only the results are rounded to
// double.
#include <quadmath.h>

#include <cstdlib>
#include <cstring>
#include <vector>

#include "internal.h"

namespace fc2d {

typedef __float128 q128;

static void mgs_qr(int d, std::vector<q128>& P, std::vector<q128>& Q, std::vector<q128>& R) {
    // column-major d x d
    std::vector<q128> V = P;
    Q.assign(d * d, 0);
    R.assign(d * d, 0);
    for (int j = 0; j < d; ++j) {
        q128 s = 0;
        for (int i = 0; i < d; ++i) s += V[i + j * d] * V[i + j * d];
        R[j + j * d] = sqrtq(s);
        for (int i = 0; i < d; ++i) Q[i + j * d] = V[i + j * d] / R[j + j * d];
        for (int k = j + 1; k < d; ++k) {
            q128 r = 0;
            for (int i = 0; i < d; ++i) r += Q[i + j * d] * V[i + k * d];
            R[j + k * d] = r;
            for (int i = 0; i < d; ++i) V[i + k * d] -= r * Q[i + j * d];
        }
    }
}

// trigonometric basis row at x = num / den (exact rational), period T (integer)
static void trig_row(long num, long den, long T, int mf, q128* row) {
    row[0] = 1;
    for (int m = 1; m <= mf; ++m) {
        // angle = 2 pi m num / (den T), reduced modulo 2 pi exactly in integers
        long long period = (long long)den * T;
        long long r = ((long long)m * num) % period;
        if (r < 0) r += period;
        q128 a = 2 * M_PIq * (q128)r / (q128)period;
        row[2 * m - 1] = cosq(a);
        row[2 * m] = sinq(a);
    }
}

int gram_tables(int d, int C, int Z, int n_os, int n_r, int mf, double* Qout, double* Aout,
                double* Arout) {
    if (d < 2 || d > 16 || C < 1 || Z < 2 || n_os < 1 || n_r < 1 || mf < 1) return -1;
    const int nc = 2 * mf + 1;
    const long T = d + 2 * C + Z - 1;
    // Gram basis
    std::vector<q128> P(d * d), Q, R;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            q128 v = 1;
            for (int e = 0; e < j; ++e) v *= i;
            P[i + j * d] = v;
        }
    mgs_qr(d, P, Q, R);
    // oversampled Gram values: row-vector solve q_os R = p_os
    const int nos_pts = n_os * (d - 1) + 1;
    const int nz_pts = n_os * (Z - 1) + 1;
    const int nrow = nos_pts + nz_pts;
    if (nrow < nc) return -1;
    std::vector<q128> Qos(nos_pts * d);
    for (int r = 0; r < nos_pts; ++r) {
        q128 x = (q128)r / n_os;
        q128 p[16];
        q128 v = 1;
        for (int j = 0; j < d; ++j) { p[j] = v; v *= x; }
        for (int j = 0; j < d; ++j) {
            q128 s = p[j];
            for (int k = 0; k < j; ++k) s -= Qos[r * d + k] * R[k + j * d];
            Qos[r * d + j] = s / R[j + j * d];
        }
    }
    // least-squares matrix (column-major nrow x nc)
    std::vector<q128> Bm(nrow * nc);
    std::vector<q128> row(nc);
    for (int r = 0; r < nrow; ++r) {
        long num, den = n_os;
        if (r < nos_pts) num = r;
        else num = (long)(d + C) * n_os + (r - nos_pts);
        trig_row(num, den, T, mf, row.data());
        for (int c = 0; c < nc; ++c) Bm[r + c * nrow] = row[c];
    }
    // Householder QR of Bm, applied to the d right-hand sides
    std::vector<q128> rhs(nrow * d, 0);
    for (int j = 0; j < d; ++j)
        for (int r = 0; r < nos_pts; ++r) rhs[r + j * nrow] = Qos[r * d + j];
    std::vector<q128> v(nrow);
    for (int k = 0; k < nc; ++k) {
        q128 nrm = 0;
        for (int i = k; i < nrow; ++i) nrm += Bm[i + k * nrow] * Bm[i + k * nrow];
        nrm = sqrtq(nrm);
        if (nrm == 0) return -1;
        q128 alpha = Bm[k + k * nrow] > 0 ? -nrm : nrm;
        for (int i = 0; i < nrow; ++i) v[i] = (i < k) ? 0 : Bm[i + k * nrow];
        v[k] -= alpha;
        q128 vv = 0;
        for (int i = k; i < nrow; ++i) vv += v[i] * v[i];
        if (vv == 0) continue;
        for (int c = k; c < nc; ++c) {
            q128 s = 0;
            for (int i = k; i < nrow; ++i) s += v[i] * Bm[i + c * nrow];
            s = 2 * s / vv;
            for (int i = k; i < nrow; ++i) Bm[i + c * nrow] -= s * v[i];
        }
        for (int c = 0; c < d; ++c) {
            q128 s = 0;
            for (int i = k; i < nrow; ++i) s += v[i] * rhs[i + c * nrow];
            s = 2 * s / vv;
            for (int i = k; i < nrow; ++i) rhs[i + c * nrow] -= s * v[i];
        }
    }
    // back substitution R a = (Q^T rhs)[0:nc]
    std::vector<q128> coef(nc * d);
    for (int c = 0; c < d; ++c)
        for (int i = nc - 1; i >= 0; --i) {
            q128 s = rhs[i + c * nrow];
            for (int k = i + 1; k < nc; ++k) s -= Bm[i + k * nrow] * coef[k + c * nc];
            coef[i + c * nc] = s / Bm[i + i * nrow];
        }
    // continuation matrices
    for (int l = 0; l < C; ++l) {
        trig_row((long)(d + l) * n_os, n_os, T, mf, row.data());
        for (int j = 0; j < d; ++j) {
            q128 s = 0;
            for (int c = 0; c < nc; ++c) s += row[c] * coef[c + j * nc];
            Aout[l * d + j] = (double)s;
        }
    }
    const int Cr = C * n_r;
    for (int l = 1; l <= Cr; ++l) {
        trig_row((long)(d - 1) * n_r + l, n_r, T, mf, row.data());
        for (int j = 0; j < d; ++j) {
            q128 s = 0;
            for (int c = 0; c < nc; ++c) s += row[c] * coef[c + j * nc];
            Arout[(l - 1) * d + j] = (double)s;
        }
    }
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) Qout[i * d + j] = (double)Q[i + j * d];
    return 0;
}

}  // namespace fc2d
