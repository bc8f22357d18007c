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
//    sum where every node is at least 7 node spacings away, otherwise the sum
//    on a refined level (2, 4, ..., 32 nb nodes) with spacing at most a seventh
//    of the distance; points whose nearest node is closer than h are listed,
//    and those within h/2 of Gamma (foot of the normal, Sec. 3.4) take v from
//    the foot value g_hom(theta) and the 32 nb-node sums at M - 1 points h/2,
//    h, ... inward along the normal, interpolated in the distance with degree
//    M - 1.
#include <hip/hip_runtime.h>

#include <math.h>

#include <algorithm>
#include <string>

#include "internal.h"
#include "poisson_int.h"
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

__global__ void k_pois_nodes(CurveC cv, int nb, double* __restrict__ qc, double* __restrict__ geo) {
    const int top = kPoisLevels - 1;
    const int64_t nall = (int64_t)nb * ((2 << top) - 1);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb + nall) return;
    const double nf = (double)nb * (double)(1 << top);
    double o[6];
    if (i < nb) {
        curve_eval(cv, 2.0 * M_PI * (double)(i << top) / nf, o);
        for (int c = 0; c < 6; ++c) qc[6 * i + c] = o[c];
        return;
    }
    const int64_t e = i - nb;
    int L = 0;
    while (e >= (int64_t)nb * ((2 << L) - 1)) ++L;
    const int64_t k = e - (int64_t)nb * ((1 << L) - 1);
    curve_eval(cv, 2.0 * M_PI * (double)(k << (top - L)) / nf, o);
    reinterpret_cast<double4*>(geo)[e] = make_double4(o[0], o[1], o[2], o[3]);
}

// chords of the nb-node polygon: seg[j] = (x_j, y_j, x_{j+1} - x_j, y_{j+1} - y_j)
// and sinv[j] = 1 / |chord|^2, from the level-0 node data
__global__ void k_pois_segments(const double4* __restrict__ geo, int nb, double4* __restrict__ seg,
                                double* __restrict__ sinv) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nb) return;
    const double4 a = geo[j], b = geo[j + 1 < nb ? j + 1 : 0];
    const double sx = b.x - a.x, sy = b.y - a.y;
    seg[j] = make_double4(a.x, a.y, sx, sy);
    sinv[j] = 1.0 / (sx * sx + sy * sy);
}

// one block per grid row; runs (start, end, class) cover the row in order
__global__ void k_pois_classes(const int32_t* __restrict__ run_ptr, const int32_t* __restrict__ run, int ny,
                               int8_t* __restrict__ cls) {
    const int i = blockIdx.x;
    const int r0 = run_ptr[i], r1 = run_ptr[i + 1];
    for (int j = threadIdx.x; j < ny; j += blockDim.x) {
        int8_t c = 0;
        for (int r = r0; r < r1; ++r)
            if (j >= run[3 * r] && j < run[3 * r + 1]) c = (int8_t)run[3 * r + 2];
        cls[(int64_t)i * ny + j] = c;
    }
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
// part[c n + i] = sum over the columns k of split c of A[k n + i] x[k]
// (A column-major; grid: row blocks of 256 x column splits)
// (NF right-hand sides x_f at stride xs; A read once for all of them:
// part[(c NF + f) n + i])
template <int NF>
__global__ __launch_bounds__(256) void k_matvec_part(const double* __restrict__ A, const double* __restrict__ x,
                                                     int64_t xs, int n, int splits, double* __restrict__ part) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    const int k0 = (int)((int64_t)n * c / splits), k1 = (int)((int64_t)n * (c + 1) / splits);
    if (i >= n) return;
    double s0[NF], s1[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) s0[f] = s1[f] = 0.0;
    int k = k0;
    for (; k + 2 <= k1; k += 2) {
        const double a0 = A[(int64_t)k * n + i], a1 = A[(int64_t)(k + 1) * n + i];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            s0[f] += a0 * x[f * xs + k];
            s1[f] += a1 * x[f * xs + k + 1];
        }
    }
    if (k < k1) {
        const double a0 = A[(int64_t)k * n + i];
#pragma unroll
        for (int f = 0; f < NF; ++f) s0[f] += a0 * x[f * xs + k];
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) part[((int64_t)c * NF + f) * n + i] = s0[f] + s1[f];
}

// y[i] = sum of the splits' partial sums: block of 32 rows x 8 groups, group
// g adding splits g, g + 8, ... in order, then the groups in order through LDS
__global__ __launch_bounds__(256) void k_matvec_sum(const double* __restrict__ part, int n, int splits,
                                                    double* __restrict__ y) {
    __shared__ double red[8][32];
    const int r = threadIdx.x & 31, g = threadIdx.x >> 5;
    const int i = blockIdx.x * 32 + r;
    double s = 0.0;
    if (i < n)
        for (int c = g; c < splits; c += 8) s += part[(int64_t)c * n + i];
    red[g][r] = s;
    __syncthreads();
    if (g == 0 && i < n) {
        double t = 0.0;
        for (int q = 0; q < 8; ++q) t += red[q][r];
        y[i] = t;
    }
}

// out[b] = <V_b, w> for b < nv (one block per vector); field blockIdx.y takes
// V, w and out at its strides
__global__ __launch_bounds__(256) void k_dots(const double* __restrict__ V, int64_t vs, int nv,
                                              const double* __restrict__ w, int64_t ws, int n,
                                              double* __restrict__ out, int64_t os) {
    __shared__ double red[256];
    const int b = blockIdx.x;
    if (b >= nv) return;
    V += vs * blockIdx.y;
    w += ws * blockIdx.y;
    out += os * blockIdx.y;
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

// w -= sum_b c[b] V_b, b < nv; field blockIdx.y at its strides
__global__ void k_sub(const double* __restrict__ V, int64_t vs, int nv, const double* __restrict__ c, int64_t cs,
                      int n, double* __restrict__ w, int64_t ws) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    V += vs * blockIdx.y;
    c += cs * blockIdx.y;
    w += ws * blockIdx.y;
    double s = w[i];
    for (int b = 0; b < nv; ++b) s -= c[b] * V[(int64_t)b * n + i];
    w[i] = s;
}

// y_f = a_f x_f for the fields f = blockIdx.y (at most kPoisChunk)
struct Scal4 {
    double a[kPoisChunk];
};
__global__ void k_scale(Scal4 a, const double* __restrict__ x, int64_t xs, int n, double* __restrict__ y,
                        int64_t ys) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[ys * blockIdx.y + i] = a.a[blockIdx.y] * x[xs * blockIdx.y + i];
}

// y_f = x_f / sqrt(h_f) with h_f = hn[f hs] read on the device (zeros when h_f
// is not positive): the next Arnoldi vector without a trip to the host
__global__ void k_normalize(const double* __restrict__ x, int64_t xs, int n, const double* __restrict__ hn,
                            int64_t hs, double* __restrict__ y, int64_t ys) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double hv = hn[hs * blockIdx.y];
    const double sc = hv > 0.0 ? 1.0 / sqrt(hv) : 0.0;
    y[ys * blockIdx.y + i] = sc * x[xs * blockIdx.y + i];
}

// y = a x + b z
__global__ void k_axpbz(double a, const double* __restrict__ x, double b, const double* __restrict__ z, int n,
                        double* __restrict__ y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i] + b * z[i];
}

// Trigonometric interpolation of the nb samples phi_j (nodes t_j = 2 pi j / nb)
// at the R nb nodes tau_i = 2 pi i / (R nb) through the Dirichlet kernel
// D(s) = sin(nb s / 2) / (nb sin(s / 2)), times cos(s / 2) for even nb.  With
// i = R m + r, tau_i - t_j = 2 pi (k + r / R) / nb, k = m - j (mod nb; D has
// period 2 pi), so residue r is a circulant convolution of phi with
// W_r[k] = D(2 pi (k + r / R) / nb) = (-1)^k sin(pi r / R) c(pi x) / nb, where
// x = (k R + r) / (R nb) and c = cot (even nb) or 1 / sin (odd nb).
// W[(r - 1) nb + k], r = 1 .. R - 1; x is a ratio of integers, so sinpi / cospi
// take it with relative rounding only.
__global__ void k_trig_weights(int nb, int R, double* __restrict__ W) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)(R - 1) * nb) return;
    const int r = (int)(e / nb) + 1, k = (int)(e - (int64_t)(r - 1) * nb);
    const double x = (double)((int64_t)k * R + r) / ((double)R * nb);
    double sx, cx;
    sincospi(x, &sx, &cx);
    const double c = (nb & 1) ? 1.0 / sx : cx / sx;
    W[e] = ((k & 1) ? -1.0 : 1.0) * sinpi((double)r / R) * c / nb;
}

// phif[R m + r] = sum_j phi_j W_r[(m - j) mod nb] for r >= 1, phif[R m] = phi_m.
// Block: 256 consecutive m of one r (blockIdx.y); phi and the window of W_r
// that a chunk of 1024 j needs are staged in LDS.
__global__ __launch_bounds__(256) void k_trig_conv(const double* __restrict__ phi, int nb, int R,
                                                   const double* __restrict__ W, double* __restrict__ phif) {
    constexpr int CJ = 1024;
    __shared__ double ph[CJ], win[CJ + 256];
    const int r = blockIdx.y, m0 = blockIdx.x * 256, ml = threadIdx.x, m = m0 + ml;
    if (r == 0) {
        if (m < nb) phif[(int64_t)R * m] = phi[m];
        return;
    }
    const double* Wr = W + (int64_t)(r - 1) * nb;
    double s = 0.0;
    for (int j0 = 0; j0 < nb; j0 += CJ) {
        const int nj = min(CJ, nb - j0);
        // window: win[t] = W_r[(m0 - j0 - (CJ - 1) + t) mod nb], t < CJ + 255
        int kb = (m0 - j0 - (CJ - 1)) % nb;
        if (kb < 0) kb += nb;
        for (int t = ml; t < CJ + 255; t += 256) {
            int k = kb + t;
            while (k >= nb) k -= nb;
            win[t] = Wr[k];
        }
        for (int t = ml; t < nj; t += 256) ph[t] = phi[j0 + t];
        __syncthreads();
        if (m < nb)
            for (int jj = 0; jj < nj; ++jj) s += ph[jj] * win[ml - jj + CJ - 1];
        __syncthreads();
    }
    if (m < nb) phif[(int64_t)R * m + r] = s;
}

// Node records of the double-layer sums for NF fields: (x, y) and, per field
// f, (phi_f y', phi_f x'), phi_f the field's density at the node (NF = 1: the
// 32-byte record (x, y, phi y', phi x')).  Level L node k sits at record
// nb (2^L - 1) + k; its density is finest-level node k 2^(kPoisLevels - 1 - L).
template <int NF>
struct DlRec {
    double x, y;
    double ab[2 * NF];
};

template <int NF>
__global__ void k_records(const double4* __restrict__ geo, const double* __restrict__ phif, int nb,
                          DlRec<NF>* __restrict__ rec) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int top = kPoisLevels - 1;
    if (i >= (int64_t)nb * ((2 << top) - 1)) return;
    int L = 0;
    while (i >= (int64_t)nb * ((2 << L) - 1)) ++L;
    const int64_t k = i - (int64_t)nb * ((1 << L) - 1);
    const double4 g = geo[i];   // x, y, x', y'
    DlRec<NF> r;
    r.x = g.x;
    r.y = g.y;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const double ph = phif[((int64_t)f * nb << top) + (k << (top - L))];
        r.ab[2 * f] = ph * g.w;
        r.ab[2 * f + 1] = ph * g.z;
    }
    rec[i] = r;
}

// 1 / r2 from the hardware reciprocal r and its residual e = 1 - r2 r:
// 1 / r2 = r / (1 - e) = r (1 + e + e^2) up to e^3 relative (|e| < 2^-24, so
// rounding dominates: as accurate as two Newton steps, one instruction fewer;
// the squared distances here are normal numbers far from the range limits)
__device__ inline double inv_r2(double r2) {
    const double r = __builtin_amdgcn_rcp(r2);
    const double e = fma(-r2, r, 1.0);
    return fma(r, fma(e, e, e), r);
}

// trapezoidal double-layer terms of the node records [j0, j1) at (X, Y) for NF
// fields, not yet divided by the node count: sum[f].  The records come through
// the scalar cache (wave-uniform addresses), 8 / NF per wait, their
// reciprocals formed side by side; distance and reciprocal are shared by the
// fields, and for one or two fields four terms share one reciprocal (of the
// product of their squared distances, at most about 1e8 and at least about
// 1e-40 here: normal numbers).  With MIN also a lower bound of the smallest squared node distance:
// the minimum of the high words, low word zero (relative error below 2^-20,
// rounded down; it only steers the level choice and the candidate test).
template <bool MIN, int NF>
__device__ inline void dl_partial(const DlRec<NF>* __restrict__ rec, int j0, int j1, double X, double Y,
                                  double* sum, double* dmin2) {
    constexpr int U = NF == 1 ? 8 : (NF == 2 ? 4 : 2);
    double s0[NF], s1[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) s0[f] = s1[f] = 0.0;
    unsigned dmh = 0xffffffffu;
    int j = j0;
    for (; j + U <= j1; j += U) {
        DlRec<NF> b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) b[u] = rec[j + u];
        double dx[U], dy[U], r2[U], rv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            dx[u] = X - b[u].x;
            dy[u] = Y - b[u].y;
            r2[u] = dx[u] * dx[u] + dy[u] * dy[u];
            if (MIN) dmh = min(dmh, (unsigned)(__double_as_longlong(r2[u]) >> 32));
        }
        if constexpr (NF <= 2) {
            // four terms over one reciprocal: with p01 = n0 r1 + n1 r0, d01 = r0 r1
            // (and p23, d23 alike), n0/r0 + n1/r1 + n2/r2 + n3/r3 = (p01 d23 + p23 d01) / (d01 d23)
            double d01[U / 4], d23[U / 4];
#pragma unroll
            for (int v = 0; v < U / 4; ++v) {
                d01[v] = r2[4 * v] * r2[4 * v + 1];
                d23[v] = r2[4 * v + 2] * r2[4 * v + 3];
                rv[v] = inv_r2(d01[v] * d23[v]);
            }
#pragma unroll
            for (int v = 0; v < U / 4; ++v)
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const int u = 4 * v;
                    double n[4];
#pragma unroll
                    for (int m = 0; m < 4; ++m) n[m] = dx[u + m] * b[u + m].ab[2 * f] - dy[u + m] * b[u + m].ab[2 * f + 1];
                    const double p01 = fma(n[0], r2[u + 1], n[1] * r2[u]);
                    const double p23 = fma(n[2], r2[u + 3], n[3] * r2[u + 2]);
                    const double t = fma(p01, d23[v], p23 * d01[v]) * rv[v];
                    if (v & 1) s1[f] += t;
                    else s0[f] += t;
                }
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) rv[u] = inv_r2(r2[u]);
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const double t = (dx[u] * b[u].ab[2 * f] - dy[u] * b[u].ab[2 * f + 1]) * rv[u];
                    if (u & 1) s1[f] += t;
                    else s0[f] += t;
                }
        }
    }
    for (; j < j1; ++j) {
        const DlRec<NF> b = rec[j];
        const double dx = X - b.x, dy = Y - b.y;
        const double r2 = dx * dx + dy * dy;
        if (MIN) dmh = min(dmh, (unsigned)(__double_as_longlong(r2) >> 32));
        const double rv = inv_r2(r2);
#pragma unroll
        for (int f = 0; f < NF; ++f) s0[f] += (dx * b.ab[2 * f] - dy * b.ab[2 * f + 1]) * rv;
    }
    if (MIN) *dmin2 = __longlong_as_double((long long)((unsigned long long)dmh << 32));
#pragma unroll
    for (int f = 0; f < NF; ++f) sum[f] = s0[f] + s1[f];
}

// squared distance from (X, Y) to the nb-node polygon (wave-uniform chords
// through the scalar cache, four per wait), as a lower bound from the high word
__device__ inline double poly_dist2(const double4* __restrict__ seg, const double* __restrict__ sinv, int nb,
                                   double X, double Y) {
    unsigned dmh = 0xffffffffu;
    int j = 0;
    for (; j + 4 <= nb; j += 4) {
        double4 c[4];
        double iv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            c[u] = seg[j + u];
            iv[u] = sinv[j + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double vx = X - c[u].x, vy = Y - c[u].y;
            const double t = fmin(fmax((vx * c[u].z + vy * c[u].w) * iv[u], 0.0), 1.0);
            const double dx = vx - t * c[u].z, dy = vy - t * c[u].w;
            dmh = min(dmh, (unsigned)(__double_as_longlong(dx * dx + dy * dy) >> 32));
        }
    }
    for (; j < nb; ++j) {
        const double4 c = seg[j];
        const double vx = X - c.x, vy = Y - c.y;
        const double t = fmin(fmax((vx * c.z + vy * c.w) * sinv[j], 0.0), 1.0);
        const double dx = vx - t * c.z, dy = vy - t * c.w;
        dmh = min(dmh, (unsigned)(__double_as_longlong(dx * dx + dy * dy) >> 32));
    }
    return __longlong_as_double((long long)((unsigned long long)dmh << 32));
}

// blocks that share the nodes of a level of n nodes (1024 nodes per wave of a
// 16-wave block at least): the finest levels carry few points, and splitting
// their nodes over blocks keeps the chip busy
__host__ __device__ inline int dl_chunks(int n) { return n >= (16 << 14) ? 16 : (n >= (1 << 14) ? n >> 14 : 1); }

// the coarsest level whose node spacing (at most dsmax 2^-L) is a seventh of
// the distance dist to Gamma or less; the finest level when none is
__device__ inline int dl_level(double dist, double dsmax) {
    int L = 0;
    while (L < kPoisLevels - 1 && 7.0 * dsmax > dist * (double)(1 << L)) ++L;
    return L;
}

// v at every IN point from the nb-node sum (trapezoidal weight 2 pi / nb, the
// 1 / (2 pi) of the kernel folded in); u = u_p + v there, 0 elsewhere.  The
// distance to Gamma is bounded from below by the larger of (nearest node
// distance - dsmax / 2, dsmax the largest spacing of the nb nodes) and (the
// distance to the nb-node polygon - sag, sag bounding how far an arc leaves
// its chord).  Points whose bound is below h/2 go to cand (the foot of the
// normal decides there); other points closer than 7 dsmax go to the list of
// the level dl_level picks, bl[L cap ...], count bcnt[L].  NF fields: up and u
// hold them npts apart.
template <int NF>
__global__ __launch_bounds__(256) void k_dl_grid(const int8_t* __restrict__ cls, const double* __restrict__ up,
                                                 int nx, int ny, int64_t npts, double x0, double y0, double h,
                                                 const DlRec<NF>* __restrict__ rec, int nb, double dsmax,
                                                 const double4* __restrict__ seg, const double* __restrict__ sinv,
                                                 double sag, double* __restrict__ u, int32_t* __restrict__ bl,
                                                 int64_t cap,
                                                 int* __restrict__ bcnt, int32_t* __restrict__ cand,
                                                 int* __restrict__ ncand) {
    // one 8 x 8 tile of points per wave
    const int tj = (ny + 7) >> 3;
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
    const int i0 = (tile / tj) * 8, jt0 = (tile % tj) * 8;
    const int i = i0 + (l >> 3), j = jt0 + (l & 7);
    const int64_t e = (int64_t)i * ny + j;
    const bool in = i < nx && j < ny && cls[e] == 1;
    if (i < nx && j < ny && !in) {
#pragma unroll
        for (int f = 0; f < NF; ++f) u[f * npts + e] = 0.0;
    }
    if (__ballot(in) == 0) return;   // wave-uniform: every lane is still active here
    // far tile: its centre's distance to the nb-node polygon (the lanes split
    // the chords), less the tile's half-diagonal and sag, clears the listing
    // threshold max(7 dsmax, h/2) + dsmax / 2 for every point: no nearest-node
    // minimum needed
    double cm = 1e300;
    {
        const double cx = x0 + (i0 + 3.5) * h, cy = y0 + (jt0 + 3.5) * h;
        for (int q = l; q < nb; q += 64) {
            const double4 c = seg[q];
            const double vx = cx - c.x, vy = cy - c.y;
            const double t = fmin(fmax((vx * c.z + vy * c.w) * sinv[q], 0.0), 1.0);
            const double dx = vx - t * c.z, dy = vy - t * c.w;
            cm = fmin(cm, dx * dx + dy * dy);
        }
#pragma unroll
        for (int of = 32; of > 0; of >>= 1) cm = fmin(cm, __shfl_xor(cm, of, 64));
    }
    const bool far = sqrt(cm) - 3.5 * M_SQRT2 * h - sag > (fmax(7.0 * dsmax, 0.5 * h) + 0.5 * dsmax) * (1.0 + 1e-12);
    if (!in) return;
    const double X = x0 + i * h, Y = y0 + j * h;
    double d2, sum[NF];
    if (far) {
        dl_partial<false, NF>(rec, 0, nb, X, Y, sum, &d2);
#pragma unroll
        for (int f = 0; f < NF; ++f) u[f * npts + e] = up[f * npts + e] + sum[f] / nb;
        return;
    }
    dl_partial<true, NF>(rec, 0, nb, X, Y, sum, &d2);
#pragma unroll
    for (int f = 0; f < NF; ++f) u[f * npts + e] = up[f * npts + e] + sum[f] / nb;
    const double dn = sqrt(d2) - 0.5 * dsmax;
    if (dn < fmax(7.0 * dsmax, 0.5 * h)) {
        const double dest = fmax(dn, sqrt(poly_dist2(seg, sinv, nb, X, Y)) - sag);
        if (dest < 0.5 * h) {
            const int k = atomicAdd(ncand, 1);
            cand[k] = (int32_t)e;
        } else if (dest < 7.0 * dsmax) {
            const int L = dl_level(dest, dsmax);
            const int k = atomicAdd(bcnt + L, 1);
            bl[L * cap + k] = (int32_t)e;
        }
    }
}

// the listed points of one level (n = 2^L nb nodes), 64 per block: the nodes
// split into gridDim.y chunks (blockIdx.y) and each chunk over the block's W
// waves, the partial sums added in wave order.  One chunk: u = u_p + v.  More:
// the chunk's sum / n to part[(c capl + k) NF + f] for list entry k < capl
// (k_band_fin adds them), more entries than capl counted in *over
template <int W, int NF>
__global__ __launch_bounds__(64 * W) void k_dl_band(const int32_t* __restrict__ bl, const int* __restrict__ bcnt,
                                                    const double* __restrict__ up, int ny, int64_t npts, double x0,
                                                    double y0, double h, const DlRec<NF>* __restrict__ rec, int n,
                                                    double* __restrict__ u, double* __restrict__ part, int capl,
                                                    int* __restrict__ over) {
    __shared__ double ps[W][NF][64];
    const int C = gridDim.y, c = blockIdx.y;
    int cnt = *bcnt;
    if (C > 1 && cnt > capl) {
        if (blockIdx.x == 0 && c == 0 && threadIdx.x == 0) atomicAdd(over, 1);
        cnt = capl;
    }
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), l = threadIdx.x & 63;
    const int64_t c0 = (int64_t)n * c / C, cl = (int64_t)n * (c + 1) / C - c0;
    const int j0 = (int)(c0 + cl * w / W), j1 = (int)(c0 + cl * (w + 1) / W);
    for (int g = blockIdx.x; g * 64 < cnt; g += gridDim.x) {
        const int k = g * 64 + l;
        const int64_t e = bl[k < cnt ? k : g * 64];   // idle lanes repeat the group's first point
        const int i = (int)(e / ny), jj = (int)(e - (int64_t)i * ny);
        double dm, sum[NF];
        dl_partial<false, NF>(rec, j0, j1, x0 + i * h, y0 + jj * h, sum, &dm);
#pragma unroll
        for (int f = 0; f < NF; ++f) ps[w][f][l] = sum[f];
        __syncthreads();
        if (w == 0 && k < cnt) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                double s = 0.0;
                for (int q = 0; q < W; ++q) s += ps[q][f][l];
                if (C == 1) u[f * npts + e] = up[f * npts + e] + s / n;
                else part[((int64_t)c * capl + k) * NF + f] = s / n;
            }
        }
        __syncthreads();
    }
}

// u = u_p + the C chunk sums of each listed point (chunk order), NF fields
template <int NF>
__global__ void k_band_fin(const int32_t* __restrict__ bl, const int* __restrict__ bcnt, int C,
                           const double* __restrict__ part, int capl, const double* __restrict__ up, int64_t npts,
                           double* __restrict__ u) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= min(*bcnt, capl)) return;
    const int64_t e = bl[k];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        double s = 0.0;
        for (int c = 0; c < C; ++c) s += part[((int64_t)c * capl + k) * NF + f];
        u[f * npts + e] = up[f * npts + e] + s;
    }
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// the candidate points, one 64-lane block each: foot (theta, eta) seeded by
// the nearest plan boundary sample (lane reduction, smallest index among
// equals).  A point with |eta| >= h/2 is no near point: it joins the band list
// of the level its distance |eta| needs (none when level 0, already summed,
// will do).  A near point takes g_hom(theta) from the lanes, the degree-(M - 1)
// Lagrange weights in the distance on the nodes s_m = m h / 2 at s = -eta, and
// the M - 1 points P_m = foot + s_m (inward normal), m >= 1, whose sums
// k_dl_samples forms: sample k (M - 1) + m - 1 joins the list of the level its
// polygon distance bound needs, sl[L scap ...], count scnt[L].  Near point k:
// nidx[k], nw[k M + m], nv0[k NF + f] = g_hom of field f at theta (ghom: NF
// rows of nb), samp[k (M - 1) + m - 1] = P_m and slev[...] its level; count
// cnt[0], beyond capn counted in cnt[1].
template <int M, int NF>
__global__ __launch_bounds__(64) void k_near_prep(const int32_t* __restrict__ cand, const int* __restrict__ ncand,
                                                  CurveC cv, BndView bd, int maxit, int ny, double x0, double y0,
                                                  double h, const double* __restrict__ ghom, int nb, double dsmax,
                                                  const double4* __restrict__ seg, const double* __restrict__ sinv,
                                                  double sag, int32_t* __restrict__ bl, int64_t cap,
                                                  int* __restrict__ bcnt, int capn, int32_t* __restrict__ nidx,
                                                  double* __restrict__ nw, double* __restrict__ nv0,
                                                  double2* __restrict__ samp, int32_t* __restrict__ sl,
                                                  int8_t* __restrict__ slev, int64_t scap,
                                                  int* __restrict__ scnt, int* __restrict__ cnt,
                                                  int* __restrict__ nfail) {
    const int nc = *ncand;
    const int lane = threadIdx.x;
    for (int e = blockIdx.x; e < nc; e += gridDim.x) {
        const int64_t idx = cand[e];
        const int i = (int)(idx / ny), j = (int)(idx - (int64_t)i * ny);
        const double X = x0 + i * h, Y = y0 + j * h;
        double best = 1e300;
        int p = 0x7fffffff;
        for (int r = lane; r < bd.B; r += 64) {
            const double dx = bd.x[r] - X, dy = bd.y[r] - Y;
            const double d2 = dx * dx + dy * dy;
            if (d2 < best) { best = d2; p = r; }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double ob = __shfl_xor(best, o, 64);
            const int op = __shfl_xor(p, o, 64);
            if (ob < best || (ob == best && op < p)) { best = ob; p = op; }
        }
        double th, eta;
        int it;
        const int fst = foot_solve<M>(cv, bd, X, Y, p, maxit, &th, &eta, &it);   // every lane, same result
        if (fst != FOOT_OK) {
            if (lane == 0) atomicAdd(nfail, 1);
            continue;
        }
        if (!(fabs(eta) < 0.5 * h)) {
            if (lane == 0 && fabs(eta) < 7.0 * dsmax) {
                const int L = dl_level(fabs(eta), dsmax);
                const int q = atomicAdd(bcnt + L, 1);
                bl[L * cap + q] = (int32_t)idx;
            }
            continue;
        }
        // trigonometric interpolant of each field's g_hom at theta
        double sv[NF], hv[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) sv[f] = hv[f] = 0.0;
        bool hit = false;
        for (int k = lane; k < nb; k += 64) {
            const double d = th - 2.0 * M_PI * (double)k / (double)nb;
            const double sh = sin(0.5 * d);
            if (sh == 0.0) {
                hit = true;
#pragma unroll
                for (int f = 0; f < NF; ++f) hv[f] = ghom[f * nb + k];
                continue;
            }
            double w = sin(0.5 * nb * d) / (nb * sh);
            if ((nb & 1) == 0) w *= cos(0.5 * d);
#pragma unroll
            for (int f = 0; f < NF; ++f) sv[f] += w * ghom[f * nb + k];
        }
        const double any = wave_sum(hit ? 1.0 : 0.0);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            sv[f] = wave_sum(sv[f]);
            hv[f] = wave_sum(hit ? hv[f] : 0.0);
        }
        int k = 0;
        if (lane == 0) k = atomicAdd(cnt, 1);
        k = __shfl(k, 0, 64);
        if (k >= capn) {
            if (lane == 0) atomicAdd(cnt + 1, 1);
            continue;
        }
        double o[6];
        curve_eval(cv, th, o);
        const double sp = sqrt(o[2] * o[2] + o[3] * o[3]);
        const double ix = -o[3] / sp, iy = o[2] / sp;   // inward normal
        if (lane == 0) {
            double w[M];
            equi_weights<M>(-eta / (0.5 * h), w);
            nidx[k] = (int32_t)idx;
#pragma unroll
            for (int f = 0; f < NF; ++f) nv0[(int64_t)k * NF + f] = any > 0.0 ? hv[f] : sv[f];
            for (int m = 0; m < M; ++m) nw[(int64_t)k * M + m] = w[m];
        }
        // squared distances of the M - 1 samples to the nb-node polygon: the
        // lanes split the chords, then a wave minimum
        double sm[M - 1];
#pragma unroll
        for (int m = 0; m < M - 1; ++m) sm[m] = 1e300;
        for (int j = lane; j < nb; j += 64) {
            const double4 c = seg[j];
            const double iv = sinv[j];
#pragma unroll
            for (int m = 0; m < M - 1; ++m) {
                const double sh = 0.5 * h * (m + 1);
                const double vx = o[0] + sh * ix - c.x, vy = o[1] + sh * iy - c.y;
                const double t = fmin(fmax((vx * c.z + vy * c.w) * iv, 0.0), 1.0);
                const double dx = vx - t * c.z, dy = vy - t * c.w;
                sm[m] = fmin(sm[m], dx * dx + dy * dy);
            }
        }
        double mine = 0.0;
#pragma unroll
        for (int m = 0; m < M - 1; ++m) {
#pragma unroll
            for (int of = 32; of > 0; of >>= 1) sm[m] = fmin(sm[m], __shfl_xor(sm[m], of, 64));
            if (m == lane - 1) mine = sm[m];
        }
        if (lane >= 1 && lane < M) {
            const double sh = 0.5 * h * lane;
            const double px = o[0] + sh * ix, py = o[1] + sh * iy;
            const double dsb = sqrt(mine) - sag;
            const int64_t si = (int64_t)k * (M - 1) + lane - 1;
            samp[si] = make_double2(px, py);
            const int L = dsb >= 7.0 * dsmax ? 0 : dl_level(dsb, dsmax);
            slev[si] = (int8_t)L;
            const int q = atomicAdd(scnt + L, 1);
            sl[L * scap + q] = (int32_t)si;
        }
    }
}

// double-layer sums over one level's n nodes at the sample points listed for
// it (sl, count *scnt), 64 per block: the nodes split into gridDim.y chunks
// (blockIdx.y, dl_chunks(n) of them) and each chunk over the block's W waves,
// the partials added in wave order; sval[(c scap + k) NF + f] = chunk c's sum
// of field f / n for sample k
template <int W, int NF>
__global__ __launch_bounds__(64 * W) void k_dl_samples(const double2* __restrict__ samp,
                                                       const int32_t* __restrict__ sl, const int* __restrict__ scnt,
                                                       const DlRec<NF>* __restrict__ rec, int n, int64_t scap,
                                                       double* __restrict__ sval) {
    __shared__ double ps[W][NF][64];
    const int cnt = *scnt;
    const int C = gridDim.y, c = blockIdx.y;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), l = threadIdx.x & 63;
    const int64_t c0 = (int64_t)n * c / C, cl = (int64_t)n * (c + 1) / C - c0;
    const int j0 = (int)(c0 + cl * w / W), j1 = (int)(c0 + cl * (w + 1) / W);
    for (int g = blockIdx.x; g * 64 < cnt; g += gridDim.x) {
        const int k = g * 64 + l;
        const int64_t si = sl[k < cnt ? k : g * 64];   // idle lanes repeat the group's first sample
        const double2 P = samp[si];
        double dm, sum[NF];
        dl_partial<false, NF>(rec, j0, j1, P.x, P.y, sum, &dm);
#pragma unroll
        for (int f = 0; f < NF; ++f) ps[w][f][l] = sum[f];
        __syncthreads();
        if (w == 0 && k < cnt) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                double s = 0.0;
                for (int q = 0; q < W; ++q) s += ps[q][f][l];
                sval[(c * scap + si) * NF + f] = s / n;
            }
        }
        __syncthreads();
    }
}

// u = u_p + sum_m w_m v_m at the near points (v_0 = g_hom(theta), v_m the
// sample sums: the chunk sums of the sample's level added in chunk order),
// per field (up and u hold the NF fields npts apart)
template <int M, int NF>
__global__ void k_near_fin(const int32_t* __restrict__ nidx, const int* __restrict__ nnear, int capn,
                           const double* __restrict__ nw, const double* __restrict__ nv0,
                           const double* __restrict__ sval, const int8_t* __restrict__ slev, int nb,
                           const double* __restrict__ up, int64_t npts, double* __restrict__ u) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= min(*nnear, capn)) return;
    const int64_t scap = (int64_t)capn * (M - 1);
    const double* w = nw + (int64_t)k * M;
    const int64_t e = nidx[k];
    double v[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) v[f] = w[0] * nv0[(int64_t)k * NF + f];
    for (int m = 1; m < M; ++m) {
        const int64_t si = (int64_t)k * (M - 1) + m - 1;
        const int C = dl_chunks(nb << slev[si]);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            double s = 0.0;
            for (int c = 0; c < C; ++c) s += sval[(c * scap + si) * NF + f];
            v[f] += w[m] * s;
        }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) u[f * npts + e] = up[f * npts + e] + v[f];
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

int pois_nodes(const CurveC& cv, int nb, double* qc, double* geo, double* seg, double* sinv, hipStream_t s) {
    const int64_t n = (int64_t)nb * (2 << (kPoisLevels - 1));   // nb + all levels
    k_pois_nodes<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(cv, nb, qc, geo);
    k_pois_segments<<<(unsigned)((nb + 255) / 256), 256, 0, s>>>((const double4*)geo, nb, (double4*)seg, sinv);
    return pois_check("k_pois_nodes", s);
}

int pois_classes(const int32_t* run_ptr, const int32_t* run, int nx, int ny, int8_t* cls, hipStream_t s) {
    k_pois_classes<<<(unsigned)nx, 256, 0, s>>>(run_ptr, run, ny, cls);
    return pois_check("k_pois_classes", s);
}

int pois_nystrom(const double* qd, int nb, double* A, hipStream_t s) {
    k_nystrom<<<blocks_for((int64_t)nb * nb, (int64_t)1 << 30), 256, 0, s>>>(qd, nb, A);
    return pois_check("k_nystrom", s);
}

int pois_matvec_splits(int n) { return std::max(1, std::min(64, n / 32)); }

int pois_matvec(const double* A, const double* x, int64_t xs, int n, int nfc, double* part, double* y,
                hipStream_t s) {
    const int sp = pois_matvec_splits(n);
    const dim3 grid((unsigned)((n + 255) / 256), (unsigned)sp);
    switch (nfc) {
        case 1: k_matvec_part<1><<<grid, 256, 0, s>>>(A, x, xs, n, sp, part); break;
        case 2: k_matvec_part<2><<<grid, 256, 0, s>>>(A, x, xs, n, sp, part); break;
        case 4: k_matvec_part<4><<<grid, 256, 0, s>>>(A, x, xs, n, sp, part); break;
        default: set_error("Poisson: unsupported field chunk"); return FC2D_E_ARG;
    }
    // the splits' partials of the nfc outputs: one sum over nfc n entries (y holds them n apart)
    k_matvec_sum<<<(unsigned)(((int64_t)nfc * n + 31) / 32), 256, 0, s>>>(part, nfc * n, sp, y);
    return pois_check("k_matvec", s);
}

int pois_dots(const double* V, int64_t vs, int nv, const double* w, int64_t ws, int n, int nfc, double* out,
              int64_t os, hipStream_t s) {
    k_dots<<<dim3((unsigned)nv, (unsigned)nfc), 256, 0, s>>>(V, vs, nv, w, ws, n, out, os);
    return pois_check("k_dots", s);
}

int pois_sub(const double* V, int64_t vs, int nv, const double* c, int64_t cs, int n, int nfc, double* w,
             int64_t ws, hipStream_t s) {
    k_sub<<<dim3((unsigned)((n + 255) / 256), (unsigned)nfc), 256, 0, s>>>(V, vs, nv, c, cs, n, w, ws);
    return pois_check("k_sub", s);
}

int pois_scale(const double* a, const double* x, int64_t xs, int n, int nfc, double* y, int64_t ys,
               hipStream_t s) {
    Scal4 sc{};
    for (int f = 0; f < nfc && f < kPoisChunk; ++f) sc.a[f] = a[f];
    k_scale<<<dim3((unsigned)((n + 255) / 256), (unsigned)nfc), 256, 0, s>>>(sc, x, xs, n, y, ys);
    return pois_check("k_scale", s);
}

int pois_normalize(const double* x, int64_t xs, int n, int nfc, const double* hn, int64_t hs, double* y, int64_t ys,
                   hipStream_t s) {
    k_normalize<<<dim3((unsigned)((n + 255) / 256), (unsigned)nfc), 256, 0, s>>>(x, xs, n, hn, hs, y, ys);
    return pois_check("k_normalize", s);
}

int pois_axpbz(double a, const double* x, double b, const double* z, int n, double* y, hipStream_t s) {
    k_axpbz<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(a, x, b, z, n, y);
    return pois_check("k_axpbz", s);
}

int pois_records(const double* phi, int nb, int nfc, const double* geo, double* wtab, double* phif, double* rec,
                 hipStream_t s) {
    const int top = kPoisLevels - 1, R = 1 << top;
    k_trig_weights<<<(unsigned)(((int64_t)(R - 1) * nb + 255) / 256), 256, 0, s>>>(nb, R, wtab);
    for (int f = 0; f < nfc; ++f)
        k_trig_conv<<<dim3((unsigned)((nb + 255) / 256), (unsigned)R), 256, 0, s>>>(
            phi + (int64_t)f * nb, nb, R, wtab, phif + (int64_t)f * nb * R);
    int st = pois_check("k_trig_up", s);
    if (st) return st;
    const int64_t nall = (int64_t)nb * ((2 << top) - 1);
    const unsigned blk = (unsigned)((nall + 255) / 256);
    switch (nfc) {
        case 1: k_records<1><<<blk, 256, 0, s>>>((const double4*)geo, phif, nb, (DlRec<1>*)rec); break;
        case 2: k_records<2><<<blk, 256, 0, s>>>((const double4*)geo, phif, nb, (DlRec<2>*)rec); break;
        case 4: k_records<4><<<blk, 256, 0, s>>>((const double4*)geo, phif, nb, (DlRec<4>*)rec); break;
        default: set_error("Poisson: unsupported field chunk"); return FC2D_E_ARG;
    }
    return pois_check("k_records", s);
}

// the band kernel of one level with W waves per block
template <int W, int NF>
static void band_launch(const PoisDl& a, unsigned bx, int C, int L, const DlRec<NF>* rl, int* bcnt, int* over,
                        hipStream_t s) {
    const fc2d_grid* g = a.g;
    const int64_t npts = (int64_t)g->nx * g->ny;
    k_dl_band<W, NF><<<dim3(bx, C), 64 * W, 0, s>>>(a.bl + L * a.cap, bcnt + L, a.up, g->ny, npts, g->x0, g->y0, g->h,
                                                   rl, a.nb << L, a.u, a.bpart, a.capb, over);
}

template <int W, int NF>
static void samples_launch(const PoisDl& a, unsigned bx, int C, int L, int64_t scap, const DlRec<NF>* rl,
                           int* scnt, hipStream_t s) {
    k_dl_samples<W, NF><<<dim3(bx, C), 64 * W, 0, s>>>((const double2*)a.samp, a.sl + L * scap, scnt + L, rl,
                                                      a.nb << L, scap, a.sval);
}

template <int M, int NF>
static int dl_eval_mnf(const PoisDl& a, hipStream_t s) {
    const fc2d_grid* g = a.g;
    const int nb = a.nb;
    const int64_t npts = (int64_t)g->nx * g->ny;
    const int64_t tiles = (int64_t)((g->nx + 7) / 8) * ((g->ny + 7) / 8);
    const int64_t scap = (int64_t)a.capn * (M - 1);
    const DlRec<NF>* r = (const DlRec<NF>*)a.rec;
    int* ncand = a.cnt;
    int* nfail = a.cnt + 1;
    int* bcnt = a.cnt + 2;
    int* ncnt = a.cnt + 2 + kPoisLevels;
    int* scnt = a.cnt + 4 + kPoisLevels;
    int* over = a.cnt + 3 + kPoisLevels;
    // level 0 everywhere, band lists and candidates
    k_dl_grid<NF><<<(unsigned)((tiles + 3) / 4), 256, 0, s>>>(a.cls, a.up, g->nx, g->ny, npts, g->x0, g->y0, g->h, r,
                                                              nb, a.dsmax, (const double4*)a.seg, a.sinv, a.sag, a.u,
                                                              a.bl, a.cap, bcnt, a.cand, ncand);
    int st = pois_check("k_dl_grid", s);
    if (st) return st;
    // feet of the candidates: near points and their samples; the others join the band lists
    const unsigned nbk = (unsigned)std::max<int64_t>(1, std::min<int64_t>(a.cap, 16384));
    k_near_prep<M, NF><<<nbk, 64, 0, s>>>(a.cand, ncand, a.cv, a.bd, a.maxit, g->ny, g->x0, g->y0, g->h, a.ghom, nb,
                                          a.dsmax, (const double4*)a.seg, a.sinv, a.sag, a.bl, a.cap, bcnt, a.capn,
                                          a.nidx, a.nw, a.nv0, (double2*)a.samp, a.sl, a.slev, scap, scnt, ncnt,
                                          nfail);
    if ((st = pois_check("k_near_prep", s))) return st;
    // band levels 1 .. kPoisLevels - 1, up to 16 waves per group of 64 points
    for (int L = 1; L < kPoisLevels; ++L) {
        const DlRec<NF>* rl = r + (int64_t)nb * ((1 << L) - 1);
        const int C = dl_chunks(nb << L);
        const unsigned bx =
            (unsigned)std::max<int64_t>(1, std::min<int64_t>(((C > 1 ? a.capb : a.cap) + 63) / 64, 2048 / C));
        switch (L) {
            case 1: band_launch<2, NF>(a, bx, C, L, rl, bcnt, over, s); break;
            case 2: band_launch<4, NF>(a, bx, C, L, rl, bcnt, over, s); break;
            case 3: band_launch<8, NF>(a, bx, C, L, rl, bcnt, over, s); break;
            default: band_launch<16, NF>(a, bx, C, L, rl, bcnt, over, s); break;
        }
        if ((st = pois_check("k_dl_band", s))) return st;
        if (C > 1) {
            k_band_fin<NF><<<(unsigned)std::max(1, (a.capb + 255) / 256), 256, 0, s>>>(
                a.bl + L * a.cap, bcnt + L, C, a.bpart, a.capb, a.up, npts, a.u);
            if ((st = pois_check("k_band_fin", s))) return st;
        }
    }
    // sample sums by level
    for (int L = 0; L < kPoisLevels; ++L) {
        const DlRec<NF>* rl = r + (int64_t)nb * ((1 << L) - 1);
        const int C = dl_chunks(nb << L);
        const unsigned bx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((scap + 63) / 64, 2048 / C));
        switch (L) {
            case 0: samples_launch<1, NF>(a, bx, C, L, scap, rl, scnt, s); break;
            case 1: samples_launch<2, NF>(a, bx, C, L, scap, rl, scnt, s); break;
            case 2: samples_launch<4, NF>(a, bx, C, L, scap, rl, scnt, s); break;
            case 3: samples_launch<8, NF>(a, bx, C, L, scap, rl, scnt, s); break;
            default: samples_launch<16, NF>(a, bx, C, L, scap, rl, scnt, s); break;
        }
        if ((st = pois_check("k_dl_samples", s))) return st;
    }
    const unsigned fbk = (unsigned)std::max(1, (a.capn + 255) / 256);
    k_near_fin<M, NF><<<fbk, 256, 0, s>>>(a.nidx, ncnt, a.capn, a.nw, a.nv0, a.sval, a.slev, nb, a.up, npts, a.u);
    return pois_check("k_near_fin", s);
}

template <int M>
static int dl_eval_m(const PoisDl& a, hipStream_t s) {
    switch (a.nfc) {
        case 1: return dl_eval_mnf<M, 1>(a, s);
        case 2: return dl_eval_mnf<M, 2>(a, s);
        case 4: return dl_eval_mnf<M, 4>(a, s);
        default: set_error("Poisson: unsupported field chunk"); return FC2D_E_ARG;
    }
}

int pois_dl_eval(const PoisDl& a, hipStream_t s) {
    switch (a.M) {
#define FC2D_NEAR(MM) \
        case MM: return dl_eval_m<MM>(a, s);
        FC2D_NEAR(4) FC2D_NEAR(5) FC2D_NEAR(6) FC2D_NEAR(7) FC2D_NEAR(8) FC2D_NEAR(13) FC2D_NEAR(15)
#undef FC2D_NEAR
        default: set_error("unsupported M"); return FC2D_E_ARG;
    }
}

}  // namespace fc2d
