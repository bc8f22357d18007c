// Cartesian Evaluation kernels (Sec. 3.5 steps 5-6).
//
//  k_match   one wave per (normal p, field): lane (s, k) multiplies the k-th
//            grid-line node of red star s by its weight, the wave reduces to
//            the M star values, then along the normal to f_{D_p} (Sec. 3.2),
//            then c_p = Q^T f_{D_p} -- all in double-double, rounded once.
//  k_strip   one thread per STRIP point and field: interpolation onto H n V+
//            (Sec. 3.4).  Because every normal carries the same level weights
//            v(eta_Q), the continuation values never need to be formed:
//                ext(Q) = sum_j w_j(theta^Q) [ v_0 f_{D_j}[d-1] + u . c_j ],
//                u = sum_{l >= 1} v_l A_r[l-1, :]
//            which equals the normal-then-tangential interpolation of the
//            blended values F = A_r c (eq. b_to_z, Remark 2.2) up to rounding.
//  k_mask    per grid row: FAR runs written with 0, IN runs copied when the
//            output is a different buffer (in place, IN entries are untouched).
//  k_blend   materialises F[l][p] (checking only).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dd.h"
#include "internal.h"

namespace fc2d {

template <int M>
__global__ __launch_bounds__(64) void k_match(const int32_t* __restrict__ mref, const double* __restrict__ mwv,
                                              const double* __restrict__ mwn, const double* __restrict__ Q, int D,
                                              int B, const double* __restrict__ fg, int64_t npts,
                                              const double* __restrict__ fb, int64_t nbdry, double* __restrict__ c_out,
                                              double* __restrict__ fD_out) {
    const int p = blockIdx.x;
    const int f = blockIdx.y;
    const int lane = threadIdx.x;
    const int s = lane >> 3;
    const int k = lane & 7;
    const double* g = fg + (int64_t)f * npts;
    const double* bv = fb + (int64_t)f * nbdry;
    dd prod = {0.0, 0.0};
    if (s < M && k < M) {
        const int64_t o = ((int64_t)p * M + s) * M + k;
        const int32_t r = mref[o];
        const double val = r >= 0 ? g[r] : bv[B + (-r - 1)];
        prod = dd_mul_d(dd{mwv[2 * o], mwv[2 * o + 1]}, val);
    }
    // star values: reduce over k within the 8-lane group of star s
    prod = dd_add(prod, dd_shfl_xor(prod, 1));
    prod = dd_add(prod, dd_shfl_xor(prod, 2));
    prod = dd_add(prod, dd_shfl_xor(prod, 4));
    // along the normal: lane (s, q) forms wn[q][s] * star_s, reduce over s
    dd t = {0.0, 0.0};
    if (s < M && k < D - 1) {
        const int64_t o = ((int64_t)p * (D - 1) + k) * M + s;
        t = dd_mul(dd{mwn[2 * o], mwn[2 * o + 1]}, prod);
    }
    t = dd_add(t, dd_shfl_xor(t, 8));
    t = dd_add(t, dd_shfl_xor(t, 16));
    t = dd_add(t, dd_shfl_xor(t, 32));
    // lanes 0..D-2 now hold f_D[p][lane]; f_D[p][D-1] is the boundary sample
    const double fb_p = bv[p];
    dd fq[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) fq[q] = dd_shfl(t, q < 8 ? q : 0);
    if (lane < D) {
        dd acc = {0.0, 0.0};
        for (int q = 0; q < D; ++q) {
            const dd v = (q < D - 1) ? fq[q] : dd{fb_p, 0.0};
            acc = dd_add(acc, dd_mul_d(v, Q[q * D + lane]));
        }
        c_out[((int64_t)f * B + p) * D + lane] = acc.hi;
        if (fD_out) fD_out[((int64_t)f * B + p) * D + lane] = (lane < D - 1) ? t.hi : fb_p;
    }
}

__global__ void k_blend(const double* __restrict__ c, const double* __restrict__ fb, int64_t nbdry,
                        const double* __restrict__ Ar, int D, int B, int Cr, double* __restrict__ F) {
    const int64_t n = (int64_t)(Cr + 1) * B;
    const int f = blockIdx.y;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int l = (int)(k / B);
        const int p = (int)(k - (int64_t)l * B);
        double v;
        if (l == 0) {
            v = fb[(int64_t)f * nbdry + p];
        } else {
            v = 0.0;
            for (int j = 0; j < D; ++j) v += Ar[(l - 1) * D + j] * c[((int64_t)f * B + p) * D + j];
        }
        F[(int64_t)f * n + k] = v;
    }
}

template <int M>
__global__ __launch_bounds__(256) void k_strip(const int32_t* __restrict__ sidx, const double* __restrict__ sth,
                                               const double* __restrict__ seta, int64_t S, const double* __restrict__ Ar,
                                               int D, int Cr, int B, double k2, double lev_scale,
                                               const double* __restrict__ c, const double* __restrict__ fb,
                                               int64_t nbdry, double* __restrict__ out, int64_t npts) {
    extern __shared__ double sAr[];
    for (int k = threadIdx.x; k < Cr * D; k += blockDim.x) sAr[k] = Ar[k];
    __syncthreads();
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= S) return;
    const int f = blockIdx.y;
    const double th = sth[k];
    const double eta = seta[k];
    constexpr int kl = (M - 1) / 2;
    const int p0 = (M % 2 == 0) ? (int)floor(th / k2) : (int)rint(th / k2);
    double tn[M], w[M];
#pragma unroll
    for (int m = 0; m < M; ++m) tn[m] = (double)(p0 - kl + m) * k2;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        double v = 1.0;
#pragma unroll
        for (int q = 0; q < M; ++q)
            if (q != m) v *= (th - tn[q]) / (tn[m] - tn[q]);
        w[m] = v;
    }
    const double s = eta * lev_scale;
    int l0 = (int)floor(s) - M / 2 + 1;
    l0 = l0 < 0 ? 0 : (l0 > Cr - M + 1 ? Cr - M + 1 : l0);
    double v[M];
#pragma unroll
    for (int l = 0; l < M; ++l) {
        double a = 1.0;
#pragma unroll
        for (int q = 0; q < M; ++q)
            if (q != l) a *= (s - (double)(l0 + q)) / ((double)(l0 + l) - (double)(l0 + q));
        v[l] = a;
    }
    double u[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) u[j] = 0.0;
#pragma unroll
    for (int l = 0; l < M; ++l) {
        const int lev = l0 + l;
        if (lev >= 1) {
#pragma unroll
            for (int j = 0; j < 9; ++j)
                if (j < D) u[j] += v[l] * sAr[(lev - 1) * D + j];
        }
    }
    const double v0 = (l0 == 0) ? v[0] : 0.0;
    const double* cf = c + (int64_t)f * B * D;
    const double* bv = fb + (int64_t)f * nbdry;
    double ext = 0.0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        int pj = (p0 - kl + m) % B;
        pj = pj < 0 ? pj + B : pj;
        double gsum = v0 * bv[pj];
#pragma unroll
        for (int j = 0; j < 9; ++j)
            if (j < D) gsum += u[j] * cf[(int64_t)pj * D + j];
        ext += w[m] * gsum;
    }
    out[(int64_t)f * npts + sidx[k]] = ext;
}

__global__ void k_mask(const int32_t* __restrict__ run_ptr, const int32_t* __restrict__ runs, int ny,
                       const double* in, double* out, int64_t npts, int copy_in) {
    const int i = blockIdx.x;
    const int f = blockIdx.y;
    const double* src = in + (int64_t)f * npts + (int64_t)i * ny;
    double* dst = out + (int64_t)f * npts + (int64_t)i * ny;
    for (int r = run_ptr[i]; r < run_ptr[i + 1]; ++r) {
        const int a = runs[3 * r], b = runs[3 * r + 1], cl = runs[3 * r + 2];
        if (cl == 0) {
            for (int j = a + threadIdx.x; j < b; j += blockDim.x) dst[j] = 0.0;
        } else if (cl == 1 && copy_in) {
            for (int j = a + threadIdx.x; j < b; j += blockDim.x) dst[j] = src[j];
        }
    }
}

static int launch_check(const char* what, hipStream_t s) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string(what) + ": " + hipGetErrorString(e));
        return FC2D_E_HIP;
    }
    trace_point(what, s);
    return FC2D_OK;
}

int launch_match(const fc2d_plan* pl, const double* f_grid, const double* f_bdry, int64_t nbdry, double* c_out,
                 double* fD_out, int nf, hipStream_t s) {
    const int64_t npts = (int64_t)pl->grid.nx * pl->grid.ny;
    dim3 grid(pl->B, nf);
    switch (pl->M) {
        case 4: k_match<4><<<grid, 64, 0, s>>>(pl->d_mref, pl->d_mwv, pl->d_mwn, pl->d_Q, pl->d, pl->B, f_grid, npts, f_bdry, nbdry, c_out, fD_out); break;
        case 5: k_match<5><<<grid, 64, 0, s>>>(pl->d_mref, pl->d_mwv, pl->d_mwn, pl->d_Q, pl->d, pl->B, f_grid, npts, f_bdry, nbdry, c_out, fD_out); break;
        case 6: k_match<6><<<grid, 64, 0, s>>>(pl->d_mref, pl->d_mwv, pl->d_mwn, pl->d_Q, pl->d, pl->B, f_grid, npts, f_bdry, nbdry, c_out, fD_out); break;
        case 7: k_match<7><<<grid, 64, 0, s>>>(pl->d_mref, pl->d_mwv, pl->d_mwn, pl->d_Q, pl->d, pl->B, f_grid, npts, f_bdry, nbdry, c_out, fD_out); break;
        case 8: k_match<8><<<grid, 64, 0, s>>>(pl->d_mref, pl->d_mwv, pl->d_mwn, pl->d_Q, pl->d, pl->B, f_grid, npts, f_bdry, nbdry, c_out, fD_out); break;
        default: set_error("unsupported M"); return FC2D_E_ARG;
    }
    return launch_check("k_match", s);
}

int launch_blend(const fc2d_plan* pl, const double* c, const double* f_bdry, int64_t nbdry, double* F, int nf,
                 hipStream_t s) {
    const int64_t n = (int64_t)(pl->Cr + 1) * pl->B;
    dim3 grid((unsigned)std::min<int64_t>((n + 255) / 256, 4096), nf);
    k_blend<<<grid, 256, 0, s>>>(c, f_bdry, nbdry, pl->d_Ar, pl->d, pl->B, pl->Cr, F);
    return launch_check("k_blend", s);
}

int launch_strip(const fc2d_plan* pl, const double* c, const double* f_bdry, int64_t nbdry, double* out, int nf,
                 hipStream_t s) {
    const int64_t S = (int64_t)pl->strip_idx.size();
    if (S == 0) return FC2D_OK;
    const int64_t npts = (int64_t)pl->grid.nx * pl->grid.ny;
    dim3 grid((unsigned)((S + 255) / 256), nf);
    const size_t lds = (size_t)pl->Cr * pl->d * sizeof(double);
    const double lev_scale = pl->n_r / pl->k1;
    switch (pl->M) {
        case 4: k_strip<4><<<grid, 256, lds, s>>>(pl->d_sidx, pl->d_sth, pl->d_seta, S, pl->d_Ar, pl->d, pl->Cr, pl->B, pl->k2, lev_scale, c, f_bdry, nbdry, out, npts); break;
        case 5: k_strip<5><<<grid, 256, lds, s>>>(pl->d_sidx, pl->d_sth, pl->d_seta, S, pl->d_Ar, pl->d, pl->Cr, pl->B, pl->k2, lev_scale, c, f_bdry, nbdry, out, npts); break;
        case 6: k_strip<6><<<grid, 256, lds, s>>>(pl->d_sidx, pl->d_sth, pl->d_seta, S, pl->d_Ar, pl->d, pl->Cr, pl->B, pl->k2, lev_scale, c, f_bdry, nbdry, out, npts); break;
        case 7: k_strip<7><<<grid, 256, lds, s>>>(pl->d_sidx, pl->d_sth, pl->d_seta, S, pl->d_Ar, pl->d, pl->Cr, pl->B, pl->k2, lev_scale, c, f_bdry, nbdry, out, npts); break;
        case 8: k_strip<8><<<grid, 256, lds, s>>>(pl->d_sidx, pl->d_sth, pl->d_seta, S, pl->d_Ar, pl->d, pl->Cr, pl->B, pl->k2, lev_scale, c, f_bdry, nbdry, out, npts); break;
        default: set_error("unsupported M"); return FC2D_E_ARG;
    }
    return launch_check("k_strip", s);
}

int launch_mask(const fc2d_plan* pl, const double* f_grid, double* out, int nf, hipStream_t s) {
    const int64_t npts = (int64_t)pl->grid.nx * pl->grid.ny;
    dim3 grid(pl->grid.nx, nf);
    k_mask<<<grid, 256, 0, s>>>(pl->d_run_ptr, pl->d_run, pl->grid.ny, f_grid, out, npts, f_grid != out);
    return launch_check("k_mask", s);
}

}  // namespace fc2d
