// 2D FFT of the extended grid (Sec. 3.5 step 7) and the spectral consumers
// (Poisson particular solution, Sec. 4.1; Fourier-Forwarding propagation,
// Sec. 4.2), float64 on gfx950.
//
// Forward real-to-complex transform, two passes over HBM:
//   pass R (rows):    each row of N_y reals is read as N_y/2 complex numbers
//                     z_n = u_{2n} + i u_{2n+1}, transformed in LDS by a
//                     radix-8/4 Stockham FFT, and split into the N_y/2 + 1
//                     bins of the real transform (X_k = E_k + W^k O_k);
//   pass C (columns): tiles of T adjacent columns (T x 16 B contiguous per row)
//                     are transformed along x in LDS and written back in place.
// The inverse runs pass C (inverse) in place on the spectrum, then pass R'
// which rebuilds z from the half spectrum, inverse-transforms and writes reals
// scaled by 1/(N_x N_y).
// Twiddles come from a per-length table exp(-2 pi i k / N) computed on the
// host in extended precision.
#include <hip/hip_runtime.h>
#include <math.h>

#include <map>
#include <mutex>
#include <vector>

#include "internal.h"

namespace fc2d {

struct RadixPlan {
    int nst;
    int r[16];
};

static RadixPlan radix_plan(int L) {
    RadixPlan p{};
    int n = L;
    std::vector<int> rs;
    while (n % 8 == 0 && n > 1) { rs.push_back(8); n /= 8; }
    if (n == 4) rs.push_back(4);
    else if (n == 2) {
        // replace one radix 8 by 4 x 4
        if (!rs.empty()) { rs.pop_back(); rs.push_back(4); rs.push_back(4); }
        else rs.push_back(2);
    }
    p.nst = (int)rs.size();
    for (int i = 0; i < p.nst; ++i) p.r[i] = rs[i];
    return p;
}

// ---------------------------------------------------------------------------
// twiddle tables, cached per (device, N)
// ---------------------------------------------------------------------------
static std::mutex g_tw_mu;
static std::map<std::pair<int, int>, double2*> g_tw;

static const double2* twiddles(int N) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_tw_mu);
    auto it = g_tw.find({dev, N});
    if (it != g_tw.end()) return it->second;
    std::vector<double2> h(N);
    for (int k = 0; k < N; ++k) {
        const long double a = -2.0L * 3.14159265358979323846264338327950288L * (long double)k / (long double)N;
        h[k] = make_double2((double)cosl(a), (double)sinl(a));
    }
    double2* d = nullptr;
    if (hipMalloc((void**)&d, N * sizeof(double2)) != hipSuccess) return nullptr;
    if (hipMemcpy(d, h.data(), N * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return nullptr;
    }
    g_tw[{dev, N}] = d;
    return d;
}

// ---------------------------------------------------------------------------
// complex helpers and small DFTs
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ double2 cmul_mi(double2 a) {
    return INV ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

template <bool INV>
__device__ __forceinline__ void dft2(double2& a, double2& b) {
    const double2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <bool INV>
__device__ __forceinline__ void dft4(double2& a0, double2& a1, double2& a2, double2& a3) {
    const double2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
    const double2 t2 = cadd(a1, a3), t3 = cmul_mi<INV>(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

template <bool INV>
__device__ __forceinline__ void dft8(double2* v) {
    double2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    double2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<INV>(e0, e1, e2, e3);
    dft4<INV>(o0, o1, o2, o3);
    const double c = 0.70710678118654752440084436210485;
    // w8^k, forward w8 = exp(-i pi/4)
    const double2 w1 = INV ? make_double2(c, c) : make_double2(c, -c);
    const double2 w3 = INV ? make_double2(-c, c) : make_double2(-c, -c);
    o1 = cmul(o1, w1);
    o2 = cmul_mi<INV>(o2);
    o3 = cmul(o3, w3);
    v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

// In-LDS Stockham FFT of nseq sequences of length L, element (q, n) at
// buf[q * qs + n * ns].  Twiddle table of length NT (a multiple of L).
// All threads of the block must call it.
constexpr int kBPT = 4;   // butterflies per thread per stage (upper bound)

template <int R, bool INV>
__device__ __forceinline__ void lds_stage(double2* buf, int L, int nseq, int qs, int ns, int Ns,
                                          const double2* __restrict__ tw, int NT) {
    const int nthr = blockDim.x;
    const int nb = nseq * (L / R);
    const int tstep = NT / (Ns * R);
    double2 v[kBPT][R];
#pragma unroll
    for (int i = 0; i < kBPT; ++i) {
        const int b = threadIdx.x + i * nthr;
        if (b < nb) {
            const int q = b % nseq;
            const int t = b / nseq;
            const int j = t % Ns;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double2 x = buf[q * qs + (t + r * (L / R)) * ns];
                if (r > 0 && j > 0) {
                    double2 w = tw[j * r * tstep];
                    if (INV) w = cconj(w);
                    x = cmul(x, w);
                }
                v[i][r] = x;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kBPT; ++i) {
        const int b = threadIdx.x + i * nthr;
        if (b < nb) {
            const int q = b % nseq;
            const int t = b / nseq;
            const int j = t % Ns;
            if constexpr (R == 8) dft8<INV>(v[i]);
            else if constexpr (R == 4) dft4<INV>(v[i][0], v[i][1], v[i][2], v[i][3]);
            else dft2<INV>(v[i][0], v[i][1]);
            const int idxD = (t / Ns) * Ns * R + j;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[q * qs + (idxD + r * Ns) * ns] = v[i][r];
        }
    }
    __syncthreads();
}

template <bool INV>
__device__ void lds_fft(double2* buf, int L, int nseq, int qs, int ns, const RadixPlan& rp,
                        const double2* __restrict__ tw, int NT) {
    int Ns = 1;
    for (int st = 0; st < rp.nst; ++st) {
        const int R = rp.r[st];
        if (R == 8) lds_stage<8, INV>(buf, L, nseq, qs, ns, Ns, tw, NT);
        else if (R == 4) lds_stage<4, INV>(buf, L, nseq, qs, ns, Ns, tw, NT);
        else lds_stage<2, INV>(buf, L, nseq, qs, ns, Ns, tw, NT);
        Ns *= R;
    }
}

// ---------------------------------------------------------------------------
// pass R: real rows -> half-spectrum rows
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_rows_r2c(const double* __restrict__ in, double2* __restrict__ out, int nx,
                                                  int ny, int rpb, RadixPlan rp, const double2* __restrict__ tw) {
    extern __shared__ double2 sbuf[];
    const int L = ny / 2;
    const int f = blockIdx.y;
    const int row0 = blockIdx.x * rpb;
    const int nrows = min(rpb, nx - row0);
    const double2* src = (const double2*)(in + ((int64_t)f * nx + row0) * ny);
    for (int e = threadIdx.x; e < nrows * L; e += blockDim.x) sbuf[e] = src[e];
    __syncthreads();
    lds_fft<false>(sbuf, L, nrows, L, 1, rp, tw, ny);
    double2* dst = out + ((int64_t)f * nx + row0) * (L + 1);
    for (int e = threadIdx.x; e < nrows * (L + 1); e += blockDim.x) {
        const int q = e / (L + 1);
        const int k = e - q * (L + 1);
        const double2 zk = sbuf[q * L + (k == L ? 0 : k)];
        const double2 zc = cconj(sbuf[q * L + (k == 0 ? 0 : L - k)]);
        const double2 E = make_double2(0.5 * (zk.x + zc.x), 0.5 * (zk.y + zc.y));
        const double2 D = make_double2(0.5 * (zk.x - zc.x), 0.5 * (zk.y - zc.y));
        // O = D / i = -i D
        const double2 O = make_double2(D.y, -D.x);
        const double2 w = tw[k % ny];
        dst[e] = cadd(E, cmul(w, O));
    }
}

// pass R': half-spectrum rows -> real rows (scaled)
__global__ __launch_bounds__(256) void k_rows_c2r(const double2* __restrict__ in, double* __restrict__ out, int nx,
                                                  int ny, int rpb, RadixPlan rp, const double2* __restrict__ tw,
                                                  double scale) {
    extern __shared__ double2 sbuf[];
    const int L = ny / 2;
    const int f = blockIdx.y;
    const int row0 = blockIdx.x * rpb;
    const int nrows = min(rpb, nx - row0);
    const double2* src = in + ((int64_t)f * nx + row0) * (L + 1);
    for (int e = threadIdx.x; e < nrows * L; e += blockDim.x) {
        const int q = e / L;
        const int k = e - q * L;
        const double2 xk = src[q * (L + 1) + k];
        const double2 xc = cconj(src[q * (L + 1) + (L - k)]);
        const double2 S = cadd(xk, xc);
        const double2 D = csub(xk, xc);
        const double2 w = cconj(tw[k]);   // exp(+2 pi i k / ny)
        const double2 Dw = cmul(D, w);
        // Z' = S + i Dw
        sbuf[e] = make_double2(S.x - Dw.y, S.y + Dw.x);
    }
    __syncthreads();
    lds_fft<true>(sbuf, L, nrows, L, 1, rp, tw, ny);
    double2* dst = (double2*)(out + ((int64_t)f * nx + row0) * ny);
    for (int e = threadIdx.x; e < nrows * L; e += blockDim.x) {
        const double2 z = sbuf[e];
        dst[e] = make_double2(z.x * scale, z.y * scale);
    }
}

// ---------------------------------------------------------------------------
// pass C: complex transform along x of T adjacent columns, in place
// ---------------------------------------------------------------------------
template <bool INV>
__global__ __launch_bounds__(256) void k_cols(double2* __restrict__ data, int nx, int ncol, int T, RadixPlan rp,
                                              const double2* __restrict__ tw) {
    extern __shared__ double2 sbuf[];
    const int f = blockIdx.y;
    const int c0 = blockIdx.x * T;
    double2* base = data + (int64_t)f * nx * ncol;
    for (int e = threadIdx.x; e < nx * T; e += blockDim.x) {
        const int n = e / T;
        const int q = e - n * T;
        sbuf[e] = (c0 + q < ncol) ? base[(int64_t)n * ncol + c0 + q] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    lds_fft<INV>(sbuf, nx, T, 1, T, rp, tw, nx);
    for (int e = threadIdx.x; e < nx * T; e += blockDim.x) {
        const int n = e / T;
        const int q = e - n * T;
        if (c0 + q < ncol) base[(int64_t)n * ncol + c0 + q] = sbuf[e];
    }
}

static int check(const char* what, hipStream_t s) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string(what) + ": " + hipGetErrorString(e));
        return FC2D_E_HIP;
    }
    trace_point(what, s);
    return FC2D_OK;
}

static int col_tile(int nx) { return nx >= 4096 ? 1 : (nx >= 2048 ? 2 : 4); }
static int rows_per_block(int ny) { return ny / 2 >= 256 ? 1 : 256 / (ny / 2); }
static int nthreads_for(int elems) { return std::max(64, std::min(256, elems / 4)); }

int fft2_r2c(const fc2d_grid* g, const double* in, double* out, int nf, hipStream_t s) {
    const int nx = g->nx, ny = g->ny, L = ny / 2;
    if (nx > 4096 || ny > 8192) { set_error("fc2d_fft: sizes above 4096 x 8192 are not supported"); return FC2D_E_ARG; }
    const double2* twy = twiddles(ny);
    const double2* twx = twiddles(nx);
    if (!twy || !twx) { set_error("twiddle table allocation failed"); return FC2D_E_NOMEM; }
    const int rpb = rows_per_block(ny);
    const RadixPlan rpy = radix_plan(L);
    dim3 gr((nx + rpb - 1) / rpb, nf);
    k_rows_r2c<<<gr, nthreads_for(rpb * L), rpb * L * sizeof(double2), s>>>(in, (double2*)out, nx, ny, rpb, rpy, twy);
    int st = check("k_rows_r2c", s);
    if (st) return st;
    const int T = col_tile(nx);
    const RadixPlan rpx = radix_plan(nx);
    dim3 gc((L + 1 + T - 1) / T, nf);
    k_cols<false><<<gc, nthreads_for(nx * T), nx * T * sizeof(double2), s>>>((double2*)out, nx, L + 1, T, rpx, twx);
    return check("k_cols", s);
}

int fft2_c2r(const fc2d_grid* g, double* in, double* out, int nf, hipStream_t s) {
    const int nx = g->nx, ny = g->ny, L = ny / 2;
    if (nx > 4096 || ny > 8192) { set_error("fc2d_fft: sizes above 4096 x 8192 are not supported"); return FC2D_E_ARG; }
    const double2* twy = twiddles(ny);
    const double2* twx = twiddles(nx);
    if (!twy || !twx) { set_error("twiddle table allocation failed"); return FC2D_E_NOMEM; }
    const int T = col_tile(nx);
    const RadixPlan rpx = radix_plan(nx);
    dim3 gc((L + 1 + T - 1) / T, nf);
    k_cols<true><<<gc, nthreads_for(nx * T), nx * T * sizeof(double2), s>>>((double2*)in, nx, L + 1, T, rpx, twx);
    int st = check("k_cols", s);
    if (st) return st;
    const int rpb = rows_per_block(ny);
    const RadixPlan rpy = radix_plan(L);
    dim3 gr((nx + rpb - 1) / rpb, nf);
    k_rows_c2r<<<gr, nthreads_for(rpb * L), rpb * L * sizeof(double2), s>>>((const double2*)in, out, nx, ny, rpb, rpy,
                                                                           twy, 1.0 / ((double)nx * (double)ny));
    return check("k_rows_c2r", s);
}

// ---------------------------------------------------------------------------
// pointwise spectral operators
// ---------------------------------------------------------------------------
__device__ __forceinline__ void mode_of(int64_t e, int nx, int ncol, int* i, int* j) {
    const int64_t r = e / ncol;
    *j = (int)(e - r * ncol);
    *i = (int)(r % nx);
}

__global__ void k_spectral(const double2* in, double2* out, int64_t n, int nx, int ny, double h, int op) {
    const int ncol = ny / 2 + 1;
    const double Lx = nx * h, Ly = ny * h;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        int i, j;
        mode_of(e, nx, ncol, &i, &j);
        const double l = (i <= nx / 2) ? (double)i : (double)(i - nx);
        const double m = (double)j;
        const double kx = 2.0 * M_PI * l / Lx;
        const double ky = 2.0 * M_PI * m / Ly;
        const double2 v = in[e];
        double2 r;
        if (op == FC2D_LAPLACE_INV) {
            const double k2 = kx * kx + ky * ky;
            r = k2 > 0 ? make_double2(-v.x / k2, -v.y / k2) : make_double2(0.0, 0.0);
        } else {
            double k = (op == FC2D_DX) ? kx : ky;
            if (op == FC2D_DX && (nx % 2 == 0) && i == nx / 2) k = 0.0;
            if (op == FC2D_DY && (ny % 2 == 0) && j == ny / 2) k = 0.0;
            r = make_double2(-k * v.y, k * v.x);
        }
        out[e] = r;
    }
}

int spectral_apply(const fc2d_grid* g, int op, const double* in, double* out, int nf, hipStream_t s) {
    const int64_t n = (int64_t)nf * g->nx * (g->ny / 2 + 1);
    const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    k_spectral<<<nb, 256, 0, s>>>((const double2*)in, (double2*)out, n, g->nx, g->ny, g->h, op);
    return check("k_spectral", s);
}

__global__ void k_ff(const double2* u0, const double2* u1, double2* uh, double2* uth, int64_t n, int nx, int ny,
                     double h, double c, double t) {
    const int ncol = ny / 2 + 1;
    const double Lx = nx * h, Ly = ny * h;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        int i, j;
        mode_of(e, nx, ncol, &i, &j);
        const double l = (i <= nx / 2) ? (double)i : (double)(i - nx);
        const double m = (double)j;
        const double a = l / Lx, b = m / Ly;
        const double w = 2.0 * M_PI * c * sqrt(a * a + b * b);
        const double2 f0 = u0[e], f1 = u1[e];
        double2 ra, rt;
        if (i == 0 && j == 0) {
            ra = make_double2(f0.x + t * f1.x, f0.y + t * f1.y);
            rt = f1;
        } else {
            double sw, cw;
            sincos(w * t, &sw, &cw);
            const double sinc = w > 0 ? sw / w : t;
            ra = make_double2(cw * f0.x + sinc * f1.x, cw * f0.y + sinc * f1.y);
            const double mw = -w * sw;
            rt = make_double2(mw * f0.x + cw * f1.x, mw * f0.y + cw * f1.y);
        }
        uh[e] = ra;
        uth[e] = rt;
    }
}

int ff_apply(const fc2d_grid* g, double c, double t, const double* u0, const double* u1, double* uh, double* uth,
             int nf, hipStream_t s) {
    const int64_t n = (int64_t)nf * g->nx * (g->ny / 2 + 1);
    const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    k_ff<<<nb, 256, 0, s>>>((const double2*)u0, (const double2*)u1, (double2*)uh, (double2*)uth, n, g->nx, g->ny, g->h,
                            c, t);
    return check("k_ff", s);
}

}  // namespace fc2d
