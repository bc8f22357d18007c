// Equispaced Lagrange interpolation on the device: the weights of degree M - 1
// and the tensor-product interpolation of a periodic grid field at a point.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fc2d {

// 1 / prod_{q != m} (m - q) = 1 / ((-1)^(M-1-m) m! (M-1-m)!): the denominators of the
// Lagrange weights on the nodes 0, 1, ..., M-1
template <int M>
__host__ __device__ constexpr double equi_inv_den(int m) {
    double d = 1.0;
    for (int q = 0; q < M; ++q)
        if (q != m) d *= (double)(m - q);
    return 1.0 / d;
}

// Lagrange weights of degree M-1 on the equispaced nodes 0..M-1 at x:
// w_m = prod_{q < m}(x - q) prod_{q > m}(x - q) / prod_{q != m}(m - q), the
// numerators from prefix and suffix products (no division at run time).
template <int M>
__device__ __forceinline__ void equi_weights(double x, double* w) {
    double pre[M], suf[M];
    pre[0] = 1.0;
#pragma unroll
    for (int m = 1; m < M; ++m) pre[m] = pre[m - 1] * (x - (double)(m - 1));
    suf[M - 1] = 1.0;
#pragma unroll
    for (int m = M - 2; m >= 0; --m) suf[m] = suf[m + 1] * (x - (double)(m + 1));
#pragma unroll
    for (int m = 0; m < M; ++m) w[m] = pre[m] * suf[m] * equi_inv_den<M>(m);
}

// Degree-(M-1) tensor-product Lagrange interpolation of the full-box field u
// [nx][ny] on the centred M x M block of nodes around (X, Y) (grid indices
// periodic).
template <int M>
__device__ __forceinline__ double bval_one(const double* __restrict__ u, int nx, int ny, double x0, double y0,
                                           double h, double X, double Y) {
    const int i0 = (int)floor((X - x0) / h) - M / 2 + 1;
    const int j0 = (int)floor((Y - y0) / h) - M / 2 + 1;
    double wx[M], wy[M];
    equi_weights<M>((X - (x0 + (double)i0 * h)) / h, wx);
    equi_weights<M>((Y - (y0 + (double)j0 * h)) / h, wy);
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < M; ++a) {
        int ii = (i0 + a) % nx;
        ii = ii < 0 ? ii + nx : ii;
        const double* rowp = u + (int64_t)ii * ny;
        double r = 0.0;
#pragma unroll
        for (int b = 0; b < M; ++b) {
            int jj = (j0 + b) % ny;
            jj = jj < 0 ? jj + ny : jj;
            r += wy[b] * rowp[jj];
        }
        acc += wx[a] * r;
    }
    return acc;
}

}  // namespace fc2d
