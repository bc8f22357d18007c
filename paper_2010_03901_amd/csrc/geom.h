// Boundary curves and the foot of the normal, shared by the host plan code
// and the device plan kernels (FC2D_HD = __host__ __device__ under hipcc).
//
// Curves (Sec. 3.1, eq. param) are counter-clockwise Fourier series:
//   polar      q = r(t) (cos t, sin t),  r(t) = a0 + sum_m (a_{2m-1} cos mt + a_{2m} sin mt)
//   cartesian  x(t) = series a, y(t) = series b
// Outward normal n = (y', -x') / |q'|.
//
// Foot of the normal (Sec. 3.4): seed theta^(0) by Lagrange interpolation of
// theta = T(tau) over the M normals of S_{theta_p} (eq. surround, eq. param_tau),
// then safeguarded Newton on g(theta) = (q(theta) - Q) . q'(theta),
// g' = |q'|^2 + (q - Q) . q'', bracketed around theta_p.
#pragma once

#include <math.h>

#if defined(__HIPCC__)
#define FC2D_HD __host__ __device__
#else
#define FC2D_HD
#endif

namespace fc2d {

constexpr int kMaxModes = 16;
constexpr double kTwoPi = 6.283185307179586476925286766559;

struct CurveC {
    int kind;     // 1 polar, 2 cartesian
    int nmodes;
    double a[1 + 2 * kMaxModes];
    double b[1 + 2 * kMaxModes];
};

// value, first and second derivative of a0 + sum (a_{2m-1} cos mt + a_{2m} sin mt)
FC2D_HD inline void series3(const double* c, int n, double t, double* v, double* d1, double* d2) {
    double s = c[0], s1 = 0.0, s2 = 0.0;
    for (int m = 1; m <= n; ++m) {
        const double a = c[2 * m - 1];
        const double b = c[2 * m];
        const double mt = m * t;
        const double cm = cos(mt);
        const double sm = sin(mt);
        s += a * cm + b * sm;
        s1 += m * (b * cm - a * sm);
        s2 -= (double)(m * m) * (a * cm + b * sm);
    }
    *v = s;
    *d1 = s1;
    *d2 = s2;
}

// (x, y, x', y', x'', y'') at t
FC2D_HD inline void curve_eval(const CurveC& cv, double t, double* o) {
    if (cv.kind == 1) {
        double r, r1, r2;
        series3(cv.a, cv.nmodes, t, &r, &r1, &r2);
        const double ct = cos(t), st = sin(t);
        o[0] = r * ct;
        o[1] = r * st;
        o[2] = r1 * ct - r * st;
        o[3] = r1 * st + r * ct;
        o[4] = r2 * ct - 2.0 * r1 * st - r * ct;
        o[5] = r2 * st + 2.0 * r1 * ct - r * st;
    } else {
        series3(cv.a, cv.nmodes, t, &o[0], &o[2], &o[4]);
        series3(cv.b, cv.nmodes, t, &o[1], &o[3], &o[5]);
    }
}

// Boundary samples used to seed foot solves.
struct BndView {
    const double* x;
    const double* y;
    const double* nx;
    const double* ny;
    int B;
    double k2;
};

FC2D_HD inline int imod(int a, int b) {
    int r = a % b;
    return r < 0 ? r + b : r;
}

enum { FOOT_OK = 0, FOOT_NO_BRACKET = 1, FOOT_NO_CONVERGENCE = 2 };

// Foot of the normal through (X, Y) seeded by normal p; M = size of S_theta.
// Returns FOOT_*; theta in [0, 2 pi), eta signed distance (> 0 outside).
template <int M>
FC2D_HD inline int foot_solve(const CurveC& cv, const BndView& bd, double X, double Y, int p,
                              int maxit, double* theta_out, double* eta_out, int* iters_out) {
    const double k2 = bd.k2;
    const double thp = p * k2;
    double o[6];
    // bracket [lo, hi] around theta_p with g(lo) < 0 < g(hi), widened as needed
    double half = 2.0 * k2, lo = 0.0, hi = 0.0;
    bool ok = false;
    for (int e = 0; e < 6; ++e) {
        lo = thp - half;
        hi = thp + half;
        curve_eval(cv, lo, o);
        const double glo = (o[0] - X) * o[2] + (o[1] - Y) * o[3];
        curve_eval(cv, hi, o);
        const double ghi = (o[0] - X) * o[2] + (o[1] - Y) * o[3];
        if (glo < 0 && ghi > 0) {
            ok = true;
            break;
        }
        half *= 2.0;
    }
    if (!ok) return FOOT_NO_BRACKET;
    // T(tau) seed: intersections of the normals of S_{theta_p} with L_Q^perp
    constexpr int kl = (M - 1) / 2;
    const double tx = -bd.ny[p], ty = bd.nx[p];
    double tau[M], thj[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int j = p - kl + m;
        const int jj = imod(j, bd.B);
        const double ax = bd.nx[jj], ay = bd.ny[jj];
        const double wx = X - bd.x[jj], wy = Y - bd.y[jj];
        const double det = ax * (-ty) - (-tx) * ay;
        tau[m] = (ax * wy - wx * ay) / det;
        thj[m] = j * k2;
    }
    double th = 0.0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        double w = 1.0;
#pragma unroll
        for (int k = 0; k < M; ++k)
            if (k != m) w *= (0.0 - tau[k]) / (tau[m] - tau[k]);
        th += w * thj[m];
    }
    if (!(th > lo && th < hi)) th = thp;   // also rejects NaN
    const double tol = 4e-16 * kTwoPi;
    int it = 0;
    bool conv = false;
    while (it < maxit) {
        curve_eval(cv, th, o);
        const double dx = o[0] - X, dy = o[1] - Y;
        const double g = dx * o[2] + dy * o[3];
        const double gp = o[2] * o[2] + o[3] * o[3] + dx * o[4] + dy * o[5];
        if (g < 0) lo = th;
        if (g > 0) hi = th;
        double nw = th - g / gp;
        if (!(nw >= lo && nw <= hi)) nw = 0.5 * (lo + hi);
        if (g == 0) nw = th;
        ++it;
        // converged: a step below tol, or the bracket collapsed to 8 ulps
        // (near the reach, rounding noise in g can exceed tol * g')
        const bool done = fabs(nw - th) <= tol || hi - lo <= 8.0 * 0x1p-52 * fmax(1.0, fabs(hi));
        th = nw;
        if (done) {
            conv = true;
            break;
        }
    }
    if (!conv) return FOOT_NO_CONVERGENCE;
    th = fmod(th, kTwoPi);
    if (th < 0) th += kTwoPi;
    curve_eval(cv, th, o);
    const double sp = sqrt(o[2] * o[2] + o[3] * o[3]);
    *theta_out = th;
    *eta_out = (X - o[0]) * (o[3] / sp) + (Y - o[1]) * (-o[2] / sp);
    *iters_out = it;
    return FOOT_OK;
}

}  // namespace fc2d
