// Full 2D-FC Poisson solve (Sec. 4.1): Delta u = f in Omega, u = g on Gamma,
// as u = u_p + v (eq. total_soln).  Kernels for
//  * the mean term of the particular solution (eq. poisson_ps): the spectrum's
//    mean f_00 and u_p += f_00 (x^2 + y^2) / 4 (sign read so that Delta u_p = f);
//  * g_hom = g - u_p at the Nystrom nodes q(2 pi j / nb) (eq. laplace_bc),
//    u_p there by degree-(M-1) tensor interpolation from the grid;
//  * the Nystrom matrix I - 2K of the double-layer equation phi - 2 K phi =
//    -2 g_hom (trapezoidal rule; smooth kernel with the curvature limit on the
//    diagonal), stored column-major, and the GMRES building blocks;
//  * the density's trigonometric interpolant on R nb nodes (Dirichlet kernel);
//  * v = double-layer potential at the IN grid points: the nb-node trapezoidal
//    sum where every node is at least 7 node spacings away, the R nb-node sum
//    otherwise; points whose nearest fine node is closer than h are listed,
//    and those within h/2 of Gamma (foot of the normal, Sec. 3.4) take v from
//    the foot value g_hom(theta) and the fine sums at M - 1 points h/2, h, ...
//    inward along the normal, interpolated in the distance with degree M - 1.
#include <hip/hip_runtime.h>

#include <math.h>

#include <algorithm>
#include <string>

#include "internal.h"
#include "lagrange_dev.h"

namespace fc2d {

__global__ void k_pois_mean(const double2* __restrict__ spec, double inv_n, double* __restrict__ mean) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *mean = spec[0].x * inv_n;
}

__global__ void k_pois_quad(double* __restrict__ u, int nx, int ny, double x0, double y0, double h,
                            const double* __restrict__ mean) {
    const int64_t n = (int64_t)nx * ny;
    const double m4 = 0.25 * *mean;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / ny), j = (int)(e - (int64_t)i * ny);
        const double x = x0 + i * h, y = y0 + j * h;
        u[e] += m4 * (x * x + y * y);
    }
}

template <int M>
__global__ void k_pois_ghom(const double* __restrict__ up, int nx, int ny, double x0, double y0, double h,
                            const double* __restrict__ qd, int nb, const double* __restrict__ g,
                            double* __restrict__ ghom) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nb) return;
    ghom[j] = g[j] - bval_one<M>(up, nx, ny, x0, y0, h, qd[6 * j], qd[6 * j + 1]);
}

// A[j nb + i] = delta_ij - 2 K(t_i, t_j) 2 pi / nb, with K(t, tau) =
// (q(t) - q(tau)) . (y'(tau), -x'(tau)) / (2 pi |q(t) - q(tau)|^2) and the
// diagonal limit -(x' y'' - y' x'') / (4 pi |q'|^2).  qd: (x, y, x', y', x'', y'') per node.
__global__ void k_nystrom(const double* __restrict__ qd, int nb, double* __restrict__ A) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nb * nb) return;
    const int j = (int)(e / nb), i = (int)(e - (int64_t)j * nb);
    const double* a = qd + 6 * i;
    const double* b = qd + 6 * j;
    double K;
    if (i == j) {
        K = -(a[2] * a[5] - a[3] * a[4]) / (4.0 * M_PI * (a[2] * a[2] + a[3] * a[3]));
    } else {
        const double dx = a[0] - b[0], dy = a[1] - b[1];
        K = (dx * b[3] - dy * b[2]) / ((dx * dx + dy * dy) * (2.0 * M_PI));
    }
    A[e] = (i == j ? 1.0 : 0.0) - 2.0 * K * (2.0 * M_PI / nb);
}

// ---- GMRES building blocks (vectors of length n; V holds basis vectors of stride n)
__global__ void k_matvec_cm(const double* __restrict__ A, const double* __restrict__ x, int n,
                            double* __restrict__ y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += A[(int64_t)k * n + i] * x[k];
    y[i] = s;
}

// out[b] = <V_b, w> for b < nv (one block per vector)
__global__ __launch_bounds__(256) void k_dots(const double* __restrict__ V, int nv, const double* __restrict__ w,
                                              int n, double* __restrict__ out) {
    __shared__ double red[256];
    const int b = blockIdx.x;
    if (b >= nv) return;
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += V[(int64_t)b * n + i] * w[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[b] = red[0];
}

// w -= sum_b c[b] V_b, b < nv
__global__ void k_sub(const double* __restrict__ V, int nv, const double* __restrict__ c, int n,
                      double* __restrict__ w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = w[i];
    for (int b = 0; b < nv; ++b) s -= c[b] * V[(int64_t)b * n + i];
    w[i] = s;
}

// y = a x + b z
__global__ void k_axpbz(double a, const double* __restrict__ x, double b, const double* __restrict__ z, int n,
                        double* __restrict__ y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i] + b * z[i];
}

// density on R nb equispaced nodes: phif[i] = sum_j phi_j D(tau_i - t_j)
__global__ void k_trig_up(const double* __restrict__ phi, int nb, int R, double* __restrict__ phif) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nf = nb * R;
    if (i >= nf) return;
    if (i % R == 0) {
        phif[i] = phi[i / R];
        return;
    }
    const double tau = 2.0 * M_PI * (double)i / (double)nf;
    double s = 0.0;
    for (int j = 0; j < nb; ++j) {
        const double d = tau - 2.0 * M_PI * (double)j / (double)nb;
        const double sh = sin(0.5 * d);
        double w = sin(0.5 * nb * d) / (nb * sh);
        if ((nb & 1) == 0) w *= cos(0.5 * d);
        s += w * phi[j];
    }
    phif[i] = s;
}

// trigonometric interpolant of the nb samples at parameter th (as k_trig_up)
__device__ inline double trig_at(const double* __restrict__ vals, int nb, double th) {
    double s = 0.0;
    for (int j = 0; j < nb; ++j) {
        const double d = th - 2.0 * M_PI * (double)j / (double)nb;
        const double sh = sin(0.5 * d);
        if (sh == 0.0) return vals[j];
        double w = sin(0.5 * nb * d) / (nb * sh);
        if ((nb & 1) == 0) w *= cos(0.5 * d);
        s += w * vals[j];
    }
    return s;
}

// trapezoidal double-layer sum at (X, Y) over n nodes: qd as in k_nystrom
// (only x, y, x', y' read), density phi; also the smallest squared node distance
__device__ inline double dl_sum(const double* __restrict__ qd, const double* __restrict__ phi, int n, double X,
                                double Y, double* dmin2) {
    double s = 0.0, dm = 1e300;
    for (int j = 0; j < n; ++j) {
        const double* b = qd + 6 * j;
        const double dx = X - b[0], dy = Y - b[1];
        const double r2 = dx * dx + dy * dy;
        dm = fmin(dm, r2);
        s += phi[j] * (dx * b[3] - dy * b[2]) / r2;
    }
    *dmin2 = dm;
    return s / n;   // (1 / 2 pi) x (2 pi / n)
}

// v at every IN point; u = u_p + v there, 0 elsewhere.  Points whose nearest
// fine node is closer than h are appended to cand (count in *ncand).
__global__ void k_dl_grid(const int8_t* __restrict__ cls, const double* __restrict__ up, int nx, int ny,
                          double x0, double y0, double h, const double* __restrict__ qc,
                          const double* __restrict__ phic, int nb, const double* __restrict__ qf,
                          const double* __restrict__ phif, int nbf, double far2, double* __restrict__ u,
                          int32_t* __restrict__ cand, int* __restrict__ ncand) {
    const int64_t n = (int64_t)nx * ny;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        if (cls[e] != 1) {
            u[e] = 0.0;
            continue;
        }
        const int i = (int)(e / ny), j = (int)(e - (int64_t)i * ny);
        const double X = x0 + i * h, Y = y0 + j * h;
        double d2;
        double v = dl_sum(qc, phic, nb, X, Y, &d2);
        if (d2 < far2) {
            v = dl_sum(qf, phif, nbf, X, Y, &d2);
            if (d2 < h * h) {
                const int k = atomicAdd(ncand, 1);
                cand[k] = (int32_t)e;
            }
        }
        u[e] = up[e] + v;
    }
}

// the listed points within h/2 of Gamma: foot (theta, eta); v from the foot
// value and the fine sums at M - 1 points inward along the normal, degree
// M - 1 in the distance; plan boundary samples (bx, by, bnx, bny) seed the foot
template <int M>
__global__ void k_dl_near(const int32_t* __restrict__ cand, const int* __restrict__ ncand, CurveC cv, BndView bd,
                          int maxit, const double* __restrict__ up, int ny, double x0, double y0, double h,
                          const double* __restrict__ ghom, int nb, const double* __restrict__ qf,
                          const double* __restrict__ phif, int nbf, double* __restrict__ u,
                          int* __restrict__ nfail) {
    const int nc = *ncand;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nc; e += gridDim.x * blockDim.x) {
        const int64_t idx = cand[e];
        const int i = (int)(idx / ny), j = (int)(idx - (int64_t)i * ny);
        const double X = x0 + i * h, Y = y0 + j * h;
        int p = 0;
        double best = 1e300;
        for (int r = 0; r < bd.B; ++r) {
            const double dx = bd.x[r] - X, dy = bd.y[r] - Y;
            const double d2 = dx * dx + dy * dy;
            if (d2 < best) { best = d2; p = r; }
        }
        double th, eta;
        int it;
        if (foot_solve<M>(cv, bd, X, Y, p, maxit, &th, &eta, &it) != FOOT_OK) {
            atomicAdd(nfail, 1);
            continue;
        }
        if (!(fabs(eta) < 0.5 * h)) continue;
        double o[6];
        curve_eval(cv, th, o);
        const double sp = sqrt(o[2] * o[2] + o[3] * o[3]);
        const double ix = -o[3] / sp, iy = o[2] / sp;   // inward normal
        double vals[M];
        vals[0] = trig_at(ghom, nb, th);
        for (int m = 1; m < M; ++m) {
            const double s = 0.5 * h * m;
            double d2;
            vals[m] = dl_sum(qf, phif, nbf, o[0] + s * ix, o[1] + s * iy, &d2);
        }
        // Lagrange weights on the nodes s_m = m h / 2 at s = -eta
        const double x = -eta / (0.5 * h);
        double w[M];
        equi_weights<M>(x, w);
        double v = 0.0;
        for (int m = 0; m < M; ++m) v += w[m] * vals[m];
        u[idx] = up[idx] + v;
    }
}

// ---- launchers -------------------------------------------------------------
static int pois_check(const char* what, hipStream_t s) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string(what) + ": " + hipGetErrorString(e));
        return FC2D_E_HIP;
    }
    trace_point(what, s);
    return FC2D_OK;
}

static unsigned blocks_for(int64_t n, int64_t cap = 1 << 16) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, cap));
}

int pois_mean(const fc2d_grid* g, const double* spec, double* mean, hipStream_t s) {
    k_pois_mean<<<1, 64, 0, s>>>((const double2*)spec, 1.0 / ((double)g->nx * g->ny), mean);
    return pois_check("k_pois_mean", s);
}

int pois_add_quad(const fc2d_grid* g, const double* mean, double* up, hipStream_t s) {
    k_pois_quad<<<blocks_for((int64_t)g->nx * g->ny), 256, 0, s>>>(up, g->nx, g->ny, g->x0, g->y0, g->h, mean);
    return pois_check("k_pois_quad", s);
}

int pois_ghom(int M, const fc2d_grid* g, const double* up, const double* qd, int nb, const double* gv,
              double* ghom, hipStream_t s) {
    const unsigned nbk = (unsigned)((nb + 255) / 256);
    switch (M) {
#define FC2D_GH(MM) \
        case MM: k_pois_ghom<MM><<<nbk, 256, 0, s>>>(up, g->nx, g->ny, g->x0, g->y0, g->h, qd, nb, gv, ghom); break;
        FC2D_GH(4) FC2D_GH(5) FC2D_GH(6) FC2D_GH(7) FC2D_GH(8) FC2D_GH(13) FC2D_GH(15)
#undef FC2D_GH
        default: set_error("unsupported M"); return FC2D_E_ARG;
    }
    return pois_check("k_pois_ghom", s);
}

int pois_nystrom(const double* qd, int nb, double* A, hipStream_t s) {
    k_nystrom<<<blocks_for((int64_t)nb * nb, (int64_t)1 << 30), 256, 0, s>>>(qd, nb, A);
    return pois_check("k_nystrom", s);
}

int pois_matvec(const double* A, const double* x, int n, double* y, hipStream_t s) {
    k_matvec_cm<<<(unsigned)((n + 127) / 128), 128, 0, s>>>(A, x, n, y);
    return pois_check("k_matvec", s);
}

int pois_dots(const double* V, int nv, const double* w, int n, double* out, hipStream_t s) {
    k_dots<<<(unsigned)nv, 256, 0, s>>>(V, nv, w, n, out);
    return pois_check("k_dots", s);
}

int pois_sub(const double* V, int nv, const double* c, int n, double* w, hipStream_t s) {
    k_sub<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(V, nv, c, n, w);
    return pois_check("k_sub", s);
}

int pois_axpbz(double a, const double* x, double b, const double* z, int n, double* y, hipStream_t s) {
    k_axpbz<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(a, x, b, z, n, y);
    return pois_check("k_axpbz", s);
}

int pois_trig_up(const double* phi, int nb, int R, double* phif, hipStream_t s) {
    k_trig_up<<<(unsigned)(((int64_t)nb * R + 255) / 256), 256, 0, s>>>(phi, nb, R, phif);
    return pois_check("k_trig_up", s);
}

int pois_dl_grid(const fc2d_grid* g, const int8_t* cls, const double* up, const double* qc, const double* phic,
                 int nb, const double* qf, const double* phif, int nbf, double far2, double* u, int32_t* cand,
                 int* ncand, hipStream_t s) {
    k_dl_grid<<<blocks_for((int64_t)g->nx * g->ny, 8192), 256, 0, s>>>(cls, up, g->nx, g->ny, g->x0, g->y0, g->h,
                                                                       qc, phic, nb, qf, phif, nbf, far2, u, cand,
                                                                       ncand);
    return pois_check("k_dl_grid", s);
}

int pois_dl_near(int M, const int32_t* cand, const int* ncand, int64_t cap, const CurveC& cv, const BndView& bd,
                 int maxit, const fc2d_grid* g, const double* up, const double* ghom, int nb, const double* qf,
                 const double* phif, int nbf, double* u, int* nfail, hipStream_t s) {
    const unsigned nbk = blocks_for(cap, 4096);
    switch (M) {
#define FC2D_NEAR(MM) \
        case MM: k_dl_near<MM><<<nbk, 256, 0, s>>>(cand, ncand, cv, bd, maxit, up, g->ny, g->x0, g->y0, g->h, ghom, nb, qf, phif, nbf, u, nfail); break;
        FC2D_NEAR(4) FC2D_NEAR(5) FC2D_NEAR(6) FC2D_NEAR(7) FC2D_NEAR(8) FC2D_NEAR(13) FC2D_NEAR(15)
#undef FC2D_NEAR
        default: set_error("unsupported M"); return FC2D_E_ARG;
    }
    return pois_check("k_dl_near", s);
}

}  // namespace fc2d
