// Cartesian Evaluation kernels (Sec. 3.5 steps 5-6).
//
//  k_match   one thread per (normal p, field): the red-star values along the
//            grid lines, the matching values along the normal (Sec. 3.2) and
//            c_p = Q^T f_{D_p}, each a compensated dot product with
//            double-double weights (rounded once); the normal's weights are
//            uniform over the wave.
//  k_strip   one thread per STRIP point looping over a chunk of fields:
//            interpolation onto H n V+
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

// Compensated dot product (Ogita, Rump & Oishi, "Accurate sum and dot product",
// SIAM J. Sci. Comput. 26, 2005: Dot2) with a double-double left factor and
// either a double or a double-double right factor.  Accumulates (s, e) with
// s + e accurate as if computed in twice the working precision.
struct Acc2 {
    double s = 0.0, e = 0.0;
    __device__ __forceinline__ void add(dd w, double v) {
#pragma clang fp contract(off)
        const double p = w.hi * v;
        const double ep = fma(w.hi, v, -p);
        const double t = s + p;
        const double bb = t - s;
        const double es = (s - (t - bb)) + (p - bb);
        s = t;
        e += ep + es + w.lo * v;
    }
    __device__ __forceinline__ void add(dd w, dd v) {
#pragma clang fp contract(off)
        const double p = w.hi * v.hi;
        const double ep = fma(w.hi, v.hi, -p);
        const double t = s + p;
        const double bb = t - s;
        const double es = (s - (t - bb)) + (p - bb);
        s = t;
        e += ep + es + (w.hi * v.lo + w.lo * v.hi);
    }
    __device__ __forceinline__ dd result() const {
#pragma clang fp contract(off)
        const double hi = s + e;
        return dd{hi, e - (hi - s)};
    }
};

// One thread per (normal p, field f): the weights of normal p are uniform
// across the wave (scalar loads), each lane gathers its own field's values.
template <int M>
__global__ __launch_bounds__(64) void k_match(const int32_t* __restrict__ mref, const double* __restrict__ mwv,
                                              const double* __restrict__ mwn, const double* __restrict__ Q, int D,
                                              int B, const double* __restrict__ fg, int64_t npts,
                                              const double* __restrict__ fb, int64_t nbdry, int nf,
                                              double* __restrict__ c_out, double* __restrict__ fD_out) {
    // consecutive normals share grid lines: give each XCD (blocks are dealt
    // round-robin to the 8 XCDs) a contiguous range of normals so they share an L2
    const int per_xcd = (B + 7) / 8;
    const int p = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    const int f = blockIdx.y * 64 + threadIdx.x;
    if (p >= B || f >= nf) return;
    const double* g = fg + (int64_t)f * npts;
    const double* bv = fb + (int64_t)f * nbdry;
    const int32_t* ref = mref + (int64_t)p * M * M;
    const double* wv = mwv + (int64_t)p * M * M * 2;
    const double* wn = mwn + (int64_t)p * (D - 1) * M * 2;
    // red-star values along the grid lines (Sec. 3.2, first interpolation)
    dd star[M];
#pragma unroll
    for (int s = 0; s < M; ++s) {
        Acc2 a;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int o = s * M + k;
            const int32_t r = ref[o];
            const double val = r >= 0 ? g[r] : bv[B + (-r - 1)];
            a.add(dd{wv[2 * o], wv[2 * o + 1]}, val);
        }
        star[s] = a.result();
    }
    // matching values along the normal (second interpolation), then Q^T f_D
    const double fbp = bv[p];
    dd fD[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        if (q < D - 1) {
            Acc2 a;
#pragma unroll
            for (int s = 0; s < M; ++s) {
                const int o = q * M + s;
                a.add(dd{wn[2 * o], wn[2 * o + 1]}, star[s]);
            }
            fD[q] = a.result();
        } else {
            fD[q] = dd{fbp, 0.0};
        }
    }
    // c_p = Q^T f_{D_p}, stored with the boundary value appended: [c_0..c_{d-1}, f_{D_p}[d-1], 0 pad]
    const int DP = (D + 2) & ~1;
    double* co = c_out + ((int64_t)f * B + p) * DP;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        if (j < D) {
            Acc2 a;
#pragma unroll
            for (int q = 0; q < 9; ++q)
                if (q < D) a.add(fD[q], Q[q * D + j]);
            co[j] = a.result().hi;
        }
    }
    co[D] = fbp;
    if (DP > D + 1) co[D + 1] = 0.0;
    if (fD_out) {
        double* fo = fD_out + ((int64_t)f * B + p) * D;
#pragma unroll
        for (int q = 0; q < 9; ++q)
            if (q < D) fo[q] = fD[q].hi;
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
            const int DP = (D + 2) & ~1;
            for (int j = 0; j < D; ++j) v += Ar[(l - 1) * D + j] * c[((int64_t)f * B + p) * DP + j];
        }
        F[(int64_t)f * n + k] = v;
    }
}

template <int M>
__global__ __launch_bounds__(256) void k_strip(const int32_t* __restrict__ sidx, const double* __restrict__ sth,
                                               const double* __restrict__ seta, int64_t S, const double* __restrict__ Ar,
                                               int D, int Cr, int B, double k2, double lev_scale,
                                               const double* __restrict__ c, const double* __restrict__ fb,
                                               int64_t nbdry, double* __restrict__ out, int64_t npts, int nf, int fpt) {
    extern __shared__ double sAr[];
    for (int k = threadIdx.x; k < Cr * D; k += blockDim.x) sAr[k] = Ar[k];
    __syncthreads();
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= S) return;
    const double th = sth[k];
    const double eta = seta[k];
    const int32_t idx = sidx[k];
    constexpr int kl = (M - 1) / 2;
    const int p0 = (M % 2 == 0) ? (int)floor(th / k2) : (int)rint(th / k2);
    // theta weights over S_{theta^Q}
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
    // level weights at s = eta n_r / k1 and u = A_r^T v (factored blend)
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
    double u[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) u[j] = 0.0;
#pragma unroll
    for (int l = 0; l < M; ++l) {
        const int lev = l0 + l;
        if (lev >= 1) {
#pragma unroll
            for (int j = 0; j < 9; ++j)
                if (j < D) u[j] += v[l] * sAr[(lev - 1) * D + j];
        }
    }
    // slot D of each normal's record holds its boundary value: weight v_0 when l0 = 0
    u[D] = (l0 == 0) ? v[0] : 0.0;
    const int DP = (D + 2) & ~1;
    int pj[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        int q = (p0 - kl + m) % B;
        pj[m] = q < 0 ? q + B : q;
    }
    const int f0 = blockIdx.y * fpt;
    const int f1 = min(nf, f0 + fpt);
#pragma unroll 2
    for (int f = f0; f < f1; ++f) {
        const double* cf = c + (int64_t)f * B * DP;
        double ext = 0.0;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const double2* rec = (const double2*)(cf + (int64_t)pj[m] * DP);
            double gsum = 0.0;
#pragma unroll
            for (int j2 = 0; j2 < 5; ++j2) {
                if (2 * j2 < DP) {
                    const double2 cc = rec[j2];
                    gsum += u[2 * j2] * cc.x + u[2 * j2 + 1] * cc.y;
                }
            }
            ext += w[m] * gsum;
        }
        out[(int64_t)f * npts + idx] = ext;
    }
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

// fields per thread in k_strip (0 = automatic); set by the autotuner
static int g_strip_fpt = 0;
int strip_fpt_get() { return g_strip_fpt; }
int strip_fpt_set(int v) {
    if (v < 0 || v > 128) return FC2D_E_ARG;
    g_strip_fpt = v;
    return FC2D_OK;
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
    dim3 grid(((pl->B + 7) / 8) * 8, (nf + 63) / 64);
    switch (pl->M) {
#define FC2D_MATCH(MM) \
        case MM: k_match<MM><<<grid, 64, 0, s>>>(pl->d_mref, pl->d_mwv, pl->d_mwn, pl->d_Q, pl->d, pl->B, f_grid, npts, f_bdry, nbdry, nf, c_out, fD_out); break;
        FC2D_MATCH(4) FC2D_MATCH(5) FC2D_MATCH(6) FC2D_MATCH(7) FC2D_MATCH(8)
#undef FC2D_MATCH
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
    // fields per thread: enough blocks to fill the chip, weights amortised over the rest
    const int64_t pblocks = (S + 255) / 256;
    int fpt = g_strip_fpt > 0 ? g_strip_fpt
                              : (int)std::max<int64_t>(1, std::min<int64_t>(16, (int64_t)nf * pblocks / 2048));
    fpt = std::max(1, std::min(fpt, nf));
    dim3 grid((unsigned)pblocks, (nf + fpt - 1) / fpt);
    const size_t lds = (size_t)pl->Cr * pl->d * sizeof(double);
    const double lev_scale = pl->n_r / pl->k1;
    switch (pl->M) {
#define FC2D_STRIP(MM) \
        case MM: k_strip<MM><<<grid, 256, lds, s>>>(pl->d_sidx, pl->d_sth, pl->d_seta, S, pl->d_Ar, pl->d, pl->Cr, pl->B, pl->k2, lev_scale, c, f_bdry, nbdry, out, npts, nf, fpt); break;
        FC2D_STRIP(4) FC2D_STRIP(5) FC2D_STRIP(6) FC2D_STRIP(7) FC2D_STRIP(8)
#undef FC2D_STRIP
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
