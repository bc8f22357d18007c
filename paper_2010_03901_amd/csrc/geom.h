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
// g' = |q'|^2 + (q - Q) . q'', bracketed around theta_p.  foot_from_seed runs
// the same safeguarded Newton from any seed parameter (the polar angle of Q, or
// a learned guess) with a bracket grown around it.
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

// (x, y, x', y', x'', y'') at t of the polar curve q = r(t) (cos t, sin t), r = series a
FC2D_HD inline void polar_eval(const double* a, int n, double t, double* o) {
    double r, r1, r2;
    series3(a, n, t, &r, &r1, &r2);
    const double ct = cos(t), st = sin(t);
    o[0] = r * ct;
    o[1] = r * st;
    o[2] = r1 * ct - r * st;
    o[3] = r1 * st + r * ct;
    o[4] = r2 * ct - 2.0 * r1 * st - r * ct;
    o[5] = r2 * st + 2.0 * r1 * ct - r * st;
}

// (x, y, x', y', x'', y'') at t
FC2D_HD inline void curve_eval(const CurveC& cv, double t, double* o) {
    if (cv.kind == 1) {
        polar_eval(cv.a, cv.nmodes, t, o);
    } else {
        series3(cv.a, cv.nmodes, t, &o[0], &o[2], &o[4]);
        series3(cv.b, cv.nmodes, t, &o[1], &o[3], &o[5]);
    }
}

// A polar curve held by reference (coefficient rows of a device array).
struct PolarRef {
    const double* a;
    int nmodes;
};

FC2D_HD inline void curve_eval(const PolarRef& cv, double t, double* o) { polar_eval(cv.a, cv.nmodes, t, o); }

// r^(k)(t), k = 0..5, of r = a0 + sum_m (a_{2m-1} cos mt + a_{2m} sin mt):
// with P_m = a cos mt + b sin mt and S_m = b cos mt - a sin mt, P' = m S and S' = -m P.
FC2D_HD inline void polar_derivs(const double* a, int n, double t, double* R) {
    R[0] = a[0];
    R[1] = R[2] = R[3] = R[4] = R[5] = 0.0;
    for (int m = 1; m <= n; ++m) {
        const double mt = m * t;
        const double cm = cos(mt), sm = sin(mt);
        const double P = a[2 * m - 1] * cm + a[2 * m] * sm;
        const double S = a[2 * m] * cm - a[2 * m - 1] * sm;
        const double m2 = (double)m * m;
        R[0] += P;
        R[1] += m * S;
        R[2] -= m2 * P;
        R[3] -= m2 * m * S;
        R[4] += m2 * m2 * P;
        R[5] += m2 * m2 * m * S;
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

// Safeguarded Newton on g in [lo, hi] (g(lo) < 0 < g(hi)) from *th: a step
// leaving the bracket is replaced by bisection; converged when a step is below
// 4e-16 * 2 pi or the bracket has collapsed to 8 ulps (near the reach, rounding
// noise in g can exceed tol * g').  Returns false when maxit steps do not converge.
template <class CV>
FC2D_HD inline bool newton_bracketed(const CV& cv, double X, double Y, double* th_io, double lo, double hi,
                                     int maxit, int* it_out) {
    const double tol = 4e-16 * kTwoPi;
    double o[6];
    double th = *th_io;
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
        const bool done = fabs(nw - th) <= tol || hi - lo <= 8.0 * 0x1p-52 * fmax(1.0, fabs(hi));
        th = nw;
        if (done) {
            conv = true;
            break;
        }
    }
    *th_io = th;
    *it_out = it;
    return conv;
}

// theta wrapped to [0, 2 pi) and the signed distance of (X, Y) along the outward normal
template <class CV>
FC2D_HD inline void foot_finish(const CV& cv, double X, double Y, double th, double* theta_out, double* eta_out) {
    double o[6];
    th = fmod(th, kTwoPi);
    if (th < 0) th += kTwoPi;
    curve_eval(cv, th, o);
    const double sp = sqrt(o[2] * o[2] + o[3] * o[3]);
    *theta_out = th;
    *eta_out = (X - o[0]) * (o[3] / sp) + (Y - o[1]) * (-o[2] / sp);
}

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
    int it = 0;
    if (!newton_bracketed(cv, X, Y, &th, lo, hi, maxit, &it)) return FOOT_NO_CONVERGENCE;
    foot_finish(cv, X, Y, th, theta_out, eta_out);
    *iters_out = it;
    return FOOT_OK;
}

// Foot of the normal through (X, Y) from the seed parameter th0: bracket
// [th0 - half, th0 + half] with g(lo) < 0 < g(hi), half = half0 doubled up to
// 10 times, then the safeguarded Newton from th0.
template <class CV>
FC2D_HD inline int foot_from_seed(const CV& cv, double X, double Y, double th0, double half0, int maxit,
                                  double* theta_out, double* eta_out, int* iters_out) {
    double o[6];
    double half = half0, lo = 0.0, hi = 0.0;
    bool ok = false;
    for (int e = 0; e < 11; ++e) {
        lo = th0 - half;
        hi = th0 + half;
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
    double th = th0;
    int it = 0;
    if (!newton_bracketed(cv, X, Y, &th, lo, hi, maxit, &it)) return FOOT_NO_CONVERGENCE;
    foot_finish(cv, X, Y, th, theta_out, eta_out);
    *iters_out = it;
    return FOOT_OK;
}

}  // namespace fc2d
