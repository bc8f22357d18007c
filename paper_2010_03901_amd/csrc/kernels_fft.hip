// 2D FFT of the extended grid (Sec. 3.5 step 7) and the spectral consumers
// (Poisson particular solution, Sec. 4.1; Fourier-Forwarding propagation,
// Sec. 4.2), float64 on gfx950.
//
// Forward real-to-complex transform, two passes over HBM:
//   pass R (rows):    each row of N_y reals is read as N_y/2 complex numbers
//                     z_n = u_{2n} + i u_{2n+1}, transformed by a Stockham FFT
//                     held in registers (radices 16, 8, 4, 2; the elements
//                     change threads through LDS between stages), and split
//                     into the N_y/2 + 1 bins of the real transform
//                     (X_k = E_k + W^k O_k);
//   pass C (columns): tiles of T adjacent columns (T x 16 B contiguous per row)
//                     are transformed along x the same way and written back in
//                     place.
// The inverse runs pass C (inverse) in place on the spectrum, then pass R'
// which rebuilds z from the half spectrum, inverse-transforms and writes reals
// scaled by 1/(N_x N_y).
// The Stockham stages compute their twiddles in registers (sincospi of an
// exact ratio, powers by a product tree); only the real split of the row
// passes reads a per-length table exp(-2 pi i k / N), computed on the host in
// extended precision and cached per device.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"

namespace fc2d {

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

template <bool INV>
__device__ __forceinline__ double2 cmul_w(double2 a, double c, double s) {
    // a * (c + i s) forward, a * (c - i s) inverse (s given for the forward sign)
    return INV ? make_double2(a.x * c + a.y * s, a.y * c - a.x * s) : make_double2(a.x * c - a.y * s, a.x * s + a.y * c);
}

template <bool INV>
__device__ __forceinline__ void dft16(double2* v) {
    // 16 = 4 x 4: DFT4 over n1 for each n2, twiddle W16^(n2 k1), DFT4 over n2, transpose
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4<INV>(v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]);
    const double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173, c2 = 0.70710678118654752440;
    // forward W16^m = cos(2 pi m/16) - i sin(2 pi m/16)
    v[1 + 4] = cmul_w<INV>(v[1 + 4], c1, -s1);    // m = 1
    v[1 + 8] = cmul_w<INV>(v[1 + 8], c2, -c2);    // m = 2
    v[1 + 12] = cmul_w<INV>(v[1 + 12], s1, -c1);  // m = 3
    v[2 + 4] = cmul_w<INV>(v[2 + 4], c2, -c2);    // m = 2
    v[2 + 8] = cmul_mi<INV>(v[2 + 8]);            // m = 4
    v[2 + 12] = cmul_w<INV>(v[2 + 12], -c2, -c2); // m = 6
    v[3 + 4] = cmul_w<INV>(v[3 + 4], s1, -c1);    // m = 3
    v[3 + 8] = cmul_w<INV>(v[3 + 8], -c2, -c2);   // m = 6
    v[3 + 12] = cmul_w<INV>(v[3 + 12], -c1, s1);  // m = 9
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4<INV>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    double2 o[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) o[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = o[k];
}

template <int R, bool INV>
__device__ __forceinline__ void dftR(double2* v) {
    if constexpr (R == 16) dft16<INV>(v);
    else if constexpr (R == 8) dft8<INV>(v);
    else if constexpr (R == 4) dft4<INV>(v[0], v[1], v[2], v[3]);
    else dft2<INV>(v[0], v[1]);
}

// largest radix in {16, 8, 4, 2} not above E that divides rem
constexpr int pick_radix(int rem, int E) {
    int r = 16;
    while (r > E || rem % r != 0) r >>= 1;
    return r;
}

// LDS slot of element x: the low 3 bits XORed with the next 3, so a wave
// writing with a stride of 4, 8 or 16 elements (16-byte complex values)
// spreads over the banks; a bijection on every aligned block of 64 elements.
__device__ __forceinline__ int swz(int x) { return x ^ ((x >> 3) & 7); }

// x, hidden from the optimiser (an empty asm that claims to change it): keeps
// the twiddles of a later transform from being merged with an earlier one's
// and held in registers in between
__device__ __forceinline__ int opaque(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

// exp(-2 pi i a / n) for 0 <= a < n, n a power of two (2a/n is exact)
__device__ __forceinline__ double2 unit_root(int a, int n) {
    double sn, cs;
    sincospi(2.0 * (double)a / (double)n, &sn, &cs);
    return make_double2(cs, -sn);
}

// w[r] = w1^r for r = 1..R-1 (R a power of two <= 16) by a product tree of
// depth log2 R, so each power carries a few rounding errors at most
template <int R>
__device__ __forceinline__ void root_powers(double2 w1, double2* w) {
    w[1] = w1;
    if constexpr (R > 2) {
        w[2] = cmul(w1, w1);
        w[3] = cmul(w[2], w1);
    }
    if constexpr (R > 4) {
        w[4] = cmul(w[2], w[2]);
#pragma unroll
        for (int r = 5; r < 8; ++r) w[r] = cmul(w[4], w[r - 4]);
    }
    if constexpr (R > 8) {
        w[8] = cmul(w[4], w[4]);
#pragma unroll
        for (int r = 9; r < 16; ++r) w[r] = cmul(w[8], w[r - 8]);
    }
}

// Register-resident Stockham FFT of length L, E elements per thread
// (P = L / E threads per sequence).  Thread t owns butterflies b_i = t + i P;
// v[i R + r] holds element b_i + r L/R of the current stage.  On entry v holds
// the input in the first stage's read pattern (loaded by the caller); on exit
// v[i R + r] = X[b_i + r L/R] for the last stage's radix R.  Intermediate
// exchanges go through LDS at lds[n * NS + q * QS].
template <int L, int E, int Ns, bool INV>
struct StockhamFrom {
    static constexpr int R = pick_radix(L / Ns, E);
    static constexpr int NB = E / R;   // butterflies per thread
    static constexpr int P = L / E;
    static constexpr bool LAST = Ns * R == L;

    __device__ static void run(double2* v, double2* lds, int QS, int NS, int q, int t,
                               const double2* __restrict__ tw, int NT) {
        if constexpr (Ns > 1) {
            // read this stage's inputs from LDS
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const int b = t + i * P;
#pragma unroll
                for (int r = 0; r < R; ++r) v[i * R + r] = lds[swz((b + r * (L / R)) * NS + q * QS)];
            }
            // twiddles W_{Ns R}^{j r}, computed (no table reads on the critical path)
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const int b = t + i * P;
                const int j = b % Ns;
                double2 w[R];
                root_powers<R>(unit_root(opaque(j), Ns * R), w);
#pragma unroll
                for (int r = 1; r < R; ++r) v[i * R + r] = cmul(v[i * R + r], INV ? cconj(w[r]) : w[r]);
            }
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) dftR<R, INV>(v + i * R);
        if constexpr (!LAST) {
            __syncthreads();   // every thread has read this stage's inputs
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const int b = t + i * P;
                const int j = b % Ns;
                const int base = (b / Ns) * Ns * R + j;
#pragma unroll
                for (int r = 0; r < R; ++r) lds[swz((base + r * Ns) * NS + q * QS)] = v[i * R + r];
            }
            __syncthreads();
            StockhamFrom<L, E, Ns * R, INV>::run(v, lds, QS, NS, q, t, tw, NT);
        }
    }
};

template <int L, int E>
struct FirstStage {
    static constexpr int R = pick_radix(L, E);
};

// first-stage index of register slot k (= i R1 + r)
template <int L, int E>
__device__ __forceinline__ int in_index(int k, int t) {
    constexpr int R = FirstStage<L, E>::R;
    constexpr int P = L / E;
    return t + (k / R) * P + (k % R) * (L / R);
}

// last-stage index of register slot k
template <int L, int E, int Ns>
struct LastR {
    static constexpr int R0 = pick_radix(L / Ns, E);
    static constexpr int value = (Ns * R0 == L) ? R0 : LastR<L, E, (Ns * R0 == L ? L : Ns * R0)>::value;
};
template <int L, int E>
struct LastR<L, E, L> {
    static constexpr int value = 1;
};
template <int L, int E>
__device__ __forceinline__ int out_index(int k, int t) {
    constexpr int R = LastR<L, E, 1>::value;
    constexpr int P = L / E;
    return t + (k / R) * P + (k % R) * (L / R);
}

// ---------------------------------------------------------------------------
// pass R: real rows -> half-spectrum rows (one row per P threads)
// ---------------------------------------------------------------------------
// Element n of a row is the pair (2n, 2n+1).  With an extension mask the row
// is assembled on the fly (Sec. 3.5 step 6): cls2[n] holds the classes of the
// pair (bits 0-1 and 2-3: 0 FAR, 1 IN, 2 STRIP); IN values come from `in`,
// STRIP values from `strip` (same layout as `in`), FAR values are 0.
// Pair classes for the masked row pass are stored per row in thread order:
// byte t*E + k is the class of element in_index(k, t), so each thread reads its
// E class bytes with one vector load.  Bits 0-1 / 2-3: class of 2n / 2n+1.
template <int E>
struct ClassWord;
template <> struct ClassWord<2> { typedef uint16_t type; };
template <> struct ClassWord<4> { typedef uint32_t type; };
template <> struct ClassWord<8> { typedef uint64_t type; };
template <> struct ClassWord<16> { typedef uint4 type; };

template <int E>
__device__ __forceinline__ void load_classes(const uint8_t* p, uint8_t* out) {
    typedef typename ClassWord<E>::type W;
    W w = *(const W*)p;
    __builtin_memcpy(out, &w, E);
}

// Row block of this block for the transposed-spectrum row passes (nrb row
// blocks; gridDim.x = nrb rounded up to a multiple of 8): blocks are dealt
// round-robin to the 8 XCDs, so XCD x takes the contiguous range starting at
// x * ceil(nrb / 8); neighbouring row blocks share the 128-byte lines of each
// spectrum column and so share one L2.  -1 for a padding block.
__device__ __forceinline__ int xcd_row_block(int nrb) {
    const int per_xcd = (nrb + 7) / 8;
    const int rb = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
    return rb < nrb ? rb : -1;
}

// Position of bin k of row i of field f in a transposed half spectrum (ncol
// bins, nx rows, nx a multiple of 8), in complex elements: the rows are kept in
// groups of 8, ((f nx/8 + i/8) ncol + k) 8 + i % 8.  The 8 rows of a group fill
// one 128-byte line per bin and a group's bins follow each other, so the row
// passes stream a group as one contiguous range; a column is nx/8 whole lines.
__device__ __forceinline__ int64_t tpos(int f, int k, int i, int nx, int ncol) {
    return (((int64_t)f * (nx >> 3) + (i >> 3)) * ncol + k) * 8 + (i & 7);
}

__device__ const double2 g_zero_pair[1] = {{0.0, 0.0}};

// Streaming (non-temporal) 16-byte loads and stores: the passes touch every
// element once, so they bypass the cache's normal retention (measured on a
// 1 GiB device copy: 6.2 TB/s with non-temporal accesses, 4.3-5.7 TB/s without).
typedef double nt_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_nt(const double2* p) {
    const nt_d2 v = __builtin_nontemporal_load((const nt_d2*)p);
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void st_nt(double2* p, double2 x) {
    nt_d2 v;
    v.x = x.x;
    v.y = x.y;
    __builtin_nontemporal_store(v, (nt_d2*)p);
}

// One unconditional 16-byte load per pair from a selected source: both IN ->
// the field, both STRIP -> the strip values, anything else -> a cached zero
// pair (mixed pairs are fixed up afterwards).
__device__ __forceinline__ const double2* pair_source(const double* row, const double* srow, int c, int n) {
    return c == 5 ? (const double2*)row + n : (c == 10 ? (const double2*)srow + n : g_zero_pair);
}

__device__ __forceinline__ double2 mixed_pair(const double* row, const double* srow, int c, int n) {
    const int c0 = c & 3, c1 = (c >> 2) & 3;
    double2 z;
    z.x = c0 == 1 ? row[2 * n] : (c0 == 2 ? srow[2 * n] : 0.0);
    z.y = c1 == 1 ? row[2 * n + 1] : (c1 == 2 ? srow[2 * n + 1] : 0.0);
    return z;
}

// TRANS: the half spectrum is written transposed (tpos: rows in groups of 8,
// a bin's 8 rows of a group on one 128-byte line), the RPB rows of a block as
// RPB x 16 contiguous bytes per bin; the LDS rows are padded to L + 2 so the
// RPB rows of one bin sit in different banks.
template <int L, int E, int RPB, bool MASKED, bool TRANS>
__global__ __launch_bounds__(RPB * (L / E)) void k_rows_r2c(const double* __restrict__ in, double2* __restrict__ out,
                                                            int nx, const double2* __restrict__ tw,
                                                            const double* __restrict__ strip,
                                                            const uint8_t* __restrict__ cls2, int ld) {
    constexpr int P = L / E;
    constexpr int N = 2 * L;
    constexpr int QS = TRANS ? L + 2 : L;
    __shared__ double2 lds[RPB * QS];
    const int q = threadIdx.x / P;
    const int t = threadIdx.x % P;
    const int rblk = TRANS ? xcd_row_block((nx + RPB - 1) / RPB) : (int)blockIdx.x;
    if (rblk < 0) return;   // padding block (uniform)
    const int row = rblk * RPB + q;
    const int f = blockIdx.y;
    const bool live = row < nx;
    const int64_t roff = ((int64_t)f * nx + (live ? row : 0)) * N;
    const double* src = in + roff;
    const double* ssrc = MASKED ? strip + roff : nullptr;
    double2 v[E];
    if constexpr (MASKED) {
        uint8_t cb[E];
        load_classes<E>(cls2 + (int64_t)(live ? row : 0) * L + t * E, cb);
#pragma unroll
        for (int k = 0; k < E; ++k) v[k] = ld_nt(pair_source(src, ssrc, cb[k], in_index<L, E>(k, t)));
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const int c = cb[k];
            if (c != 0 && c != 5 && c != 10) v[k] = mixed_pair(src, ssrc, c, in_index<L, E>(k, t));
        }
    } else {
#pragma unroll
        for (int k = 0; k < E; ++k) v[k] = ld_nt((const double2*)src + in_index<L, E>(k, t));
    }
    StockhamFrom<L, E, 1, false>::run(v, lds, QS, 1, q, t, tw, N);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) lds[swz(q * QS + out_index<L, E>(k, t))] = v[k];
    __syncthreads();
    // split into the L + 1 bins of the real transform: thread (qq, k0) takes
    // row qq, bins k = k0 + m P, with W_N^k = W_N^k0 times powers of W_N^P
    // (row-major output: qq = q, k0 = t; transposed: the RPB rows of a bin
    // on consecutive lanes)
    const int qq = TRANS ? (int)(threadIdx.x % RPB) : q;
    const int k0 = TRANS ? (int)(threadIdx.x / RPB) : t;
    const int orow = rblk * RPB + qq;
    if (orow >= nx) return;
    const double2 wstep = unit_root(P, N);
    double2 wk = unit_root(k0, N);
    for (int k = k0; k <= L; k += P) {
        const double2 zk = lds[swz(qq * QS + (k == L ? 0 : k))];
        const double2 zc = cconj(lds[swz(qq * QS + (k == 0 ? 0 : L - k))]);
        const double2 Eh = make_double2(0.5 * (zk.x + zc.x), 0.5 * (zk.y + zc.y));
        const double2 D = make_double2(0.5 * (zk.x - zc.x), 0.5 * (zk.y - zc.y));
        const double2 O = make_double2(D.y, -D.x);   // D / i
        const double2 X = cadd(Eh, cmul(wk, O));
        if (TRANS) out[tpos(f, k, orow, nx, L + 1)] = X;
        else st_nt(out + ((int64_t)f * nx + orow) * ld + k, X);
        wk = cmul(wk, wstep);
    }
}

// pass R': half-spectrum rows -> real rows, scaled
// TRANS: the half spectrum is read transposed (tpos); the block first stages
// its RPB rows in LDS (RPB x 16 contiguous bytes per bin, the bins of a row
// group one line apart).
template <int L, int E, int RPB, bool TRANS>
__global__ __launch_bounds__(RPB * (L / E)) void k_rows_c2r(const double2* __restrict__ in, double* __restrict__ out,
                                                            int nx, const double2* __restrict__ tw, double scale,
                                                            int ld) {
    constexpr int P = L / E;
    constexpr int N = 2 * L;
    constexpr int QS = TRANS ? L + 2 : L;
    __shared__ double2 lds[RPB * QS];
    const int q = threadIdx.x / P;
    const int t = threadIdx.x % P;
    const int rblk = TRANS ? xcd_row_block((nx + RPB - 1) / RPB) : (int)blockIdx.x;
    if (rblk < 0) return;   // padding block (uniform)
    const int row = rblk * RPB + q;
    const int f = blockIdx.y;
    const bool live = row < nx;
    const double2* src = in + ((int64_t)f * nx + (live ? row : 0)) * ld;
    if constexpr (TRANS) {
        // bins 0..L of the block's rows: every load in flight before the first
        // LDS write (a loop that waits for each load in turn leaves the pass
        // latency-bound)
        constexpr int NIT = (RPB * (L + 1) + RPB * P - 1) / (RPB * P);
        double2 st[NIT];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int e = threadIdx.x + it * RPB * P;
            const int qq = e % RPB, n = e / RPB;
            const int r = rblk * RPB + qq;
            st[it] = (e < RPB * (L + 1) && r < nx) ? in[tpos(f, n, r, nx, L + 1)] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int e = threadIdx.x + it * RPB * P;
            if (e < RPB * (L + 1)) lds[(e % RPB) * QS + e / RPB] = st[it];
        }
        __syncthreads();
        src = lds + q * QS;
    }
    double2 v[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const int n = in_index<L, E>(k, t);
        const double2 xk = src[n];
        const double2 xc = cconj(src[L - n]);
        const double2 S = cadd(xk, xc);
        const double2 Dw = cmul(csub(xk, xc), cconj(tw[n]));   // exp(+2 pi i n / N)
        v[k] = make_double2(S.x - Dw.y, S.y + Dw.x);           // S + i Dw
    }
    StockhamFrom<L, E, 1, true>::run(v, lds, QS, 1, q, t, tw, N);
    if (!live) return;
    double2* dst = (double2*)(out + ((int64_t)f * nx + row) * N);
#pragma unroll
    for (int k = 0; k < E; ++k) st_nt(dst + out_index<L, E>(k, t), make_double2(v[k].x * scale, v[k].y * scale));
}

// ---------------------------------------------------------------------------
// pass C: complex transform along x of T adjacent columns, in place.
// Tiles are assigned so that consecutive tiles run on the same XCD (blocks
// are dispatched round-robin over the 8 XCDs), letting the two halves of a
// 128-byte line be served by one L2.
// ---------------------------------------------------------------------------
// Block -> (field, column tile).  Blocks are dealt round-robin to the 8 XCDs.
// by_field (field count a multiple of 8): XCD x takes whole fields x, x + 8, ...,
// so no cache line is fetched by two XCDs (the 16-byte shift of the half-spectrum
// rows puts the column-range boundaries inside lines); otherwise each XCD takes
// a contiguous range of tiles of every field (grid y = field).
__device__ __forceinline__ bool col_block(int ntiles, bool by_field, int* tile, int* field) {
    if (by_field) {
        const int local = blockIdx.x / 8;
        *tile = local % ntiles;
        *field = (local / ntiles) * 8 + (int)(blockIdx.x % 8);
        return true;
    }
    const int per_xcd = (ntiles + 7) / 8;
    *tile = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    *field = blockIdx.y;
    return *tile < ntiles;
}

// NT: rows of the half spectrum start on 128-byte lines and a tile row is a
// whole number of lines (T >= 8): loads and stores stream past the caches
// (with lines shared between tiles, non-temporal stores cost more than they save)
template <int L, int E, int T, bool INV, bool NT>
__global__ __launch_bounds__(T * (L / E)) void k_cols(double2* __restrict__ data, int ncol, int ld,
                                                      const double2* __restrict__ tw, int by_field) {
    constexpr int P = L / E;
    __shared__ double2 lds[L * T];
    const int q = threadIdx.x % T;
    const int t = threadIdx.x / T;
    const int ntiles = (ncol + T - 1) / T;
    int tile, field;
    if (!col_block(ntiles, by_field != 0, &tile, &field)) return;   // uniform per block
    const int col = tile * T + q;
    const bool live = col < ncol;
    double2* base = data + (int64_t)field * L * ld + (live ? col : 0);
    double2 v[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const double2* p = base + (int64_t)in_index<L, E>(k, t) * ld;
        v[k] = NT ? ld_nt(p) : *p;
    }
    StockhamFrom<L, E, 1, INV>::run(v, lds, 1, T, q, t, tw, L);
    if (!live) return;
#pragma unroll
    for (int k = 0; k < E; ++k) {
        double2* p = base + (int64_t)out_index<L, E>(k, t) * ld;
        if (NT) st_nt(p, v[k]);
        else *p = v[k];
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

// row-pass configurations: (L, E, rows per block); the transposed-spectrum
// forms take 4 rows per block (64 contiguous bytes per bin)
template <bool FWD, bool TRANS>
static void launch_rows(int L, int nx, int nf, const void* in, void* out, const double2* tw, double scale,
                        const double* strip, const uint8_t* cls2, hipStream_t s, int ld) {
#define FC2D_ROWS(LL, EE, RR0)                                                                             \
    case LL: {                                                                                             \
        constexpr int RR = TRANS ? 4 : RR0;                                                                \
        if constexpr (!TRANS || LL <= 2048) {                                                              \
            const int nrb = (nx + RR - 1) / RR;                                                            \
            dim3 g(TRANS ? (nrb + 7) / 8 * 8 : nrb, nf);                                                   \
            if (FWD && cls2)                                                                               \
                k_rows_r2c<LL, EE, RR, true, TRANS><<<g, RR * (LL / EE), 0, s>>>((const double*)in, (double2*)out, nx, tw, strip, cls2, ld); \
            else if (FWD)                                                                                  \
                k_rows_r2c<LL, EE, RR, false, TRANS><<<g, RR * (LL / EE), 0, s>>>((const double*)in, (double2*)out, nx, tw, nullptr, nullptr, ld); \
            else k_rows_c2r<LL, EE, RR, TRANS><<<g, RR * (LL / EE), 0, s>>>((const double2*)in, (double*)out, nx, tw, scale, ld); \
        }                                                                                                  \
        break;                                                                                             \
    }
    switch (L) {
        FC2D_ROWS(8, 2, 32)
        FC2D_ROWS(16, 2, 16)
        FC2D_ROWS(32, 2, 8)
        FC2D_ROWS(64, 2, 4)
        FC2D_ROWS(128, 2, 2)
        FC2D_ROWS(256, 4, 2)
        FC2D_ROWS(512, 8, 1)
        FC2D_ROWS(1024, 16, 1)
        FC2D_ROWS(2048, 16, 1)
        FC2D_ROWS(4096, 16, 1)
    }
#undef FC2D_ROWS
}

// Row-pass elements per thread for half length L (the configuration table of launch_rows).
int row_elems(int L) {
    switch (L) {
        case 8: case 16: case 32: case 64: case 128: return 2;
        case 256: return 4;
        case 512: return 8;
        case 1024: case 2048: case 4096: return 16;
    }
    return 0;
}

// Permute one row's pair classes into the masked row pass's thread order.
void row_class_layout(int L, const uint8_t* pairs, uint8_t* out) {
    const int E = row_elems(L);
    const int P = L / E;
    int R = 16;
    while (R > E || L % R != 0) R >>= 1;   // first-stage radix
    for (int t = 0; t < P; ++t)
        for (int k = 0; k < E; ++k) out[t * E + k] = pairs[t + (k / R) * P + (k % R) * (L / R)];
}

// Column-tile widths (columns per block, 16 B each) per log2(nx); the
// autotuner (fc2d_tune_set) may change them among the compiled choices.
// column-pass launch shape per length nx = 2^lg: elements per thread E and
// columns per block T (compiled pairs below; the autotuner may switch)
static int g_col_tile[14] = {0, 0, 0, 0, 16, 8, 8, 4, 4, 4, 4, 2, 1, 0};
static int g_col_elems[14] = {0, 0, 0, 0, 2, 2, 2, 2, 4, 8, 16, 16, 16, 0};

static bool col_cfg_ok(int nx, int E, int T) {
    switch (nx) {
        case 16: case 32: case 64: return E == 2 && (T == 4 || T == 8 || T == 16);
        case 128: return E == 2 && (T == 4 || T == 8);
        case 256: return E == 4 && (T == 4 || T == 8);
        case 512: return (E == 4 || E == 8) && (T == 4 || T == 8);
        case 1024: return (E == 8 || E == 16) && (T == 2 || T == 4 || T == 8);
        case 2048: return (E == 16 && (T == 1 || T == 2 || T == 4)) || (E == 8 && (T == 1 || T == 2));
        case 4096: return (E == 16 && (T == 1 || T == 2)) || (E == 8 && T == 1);
    }
    return false;
}

static int log2_len(int nx) {
    int lg = 0;
    while ((1 << lg) < nx) ++lg;
    return lg;
}

int col_tile_get(int nx) {
    const int lg = log2_len(nx);
    return (lg >= 4 && lg <= 12) ? g_col_tile[lg] : 0;
}

int col_elems_get(int nx) {
    const int lg = log2_len(nx);
    return (lg >= 4 && lg <= 12) ? g_col_elems[lg] : 0;
}

int col_cfg_set(int nx, int E, int T) {
    if (!col_cfg_ok(nx, E, T)) return FC2D_E_ARG;
    const int lg = log2_len(nx);
    g_col_elems[lg] = E;
    g_col_tile[lg] = T;
    return FC2D_OK;
}

int col_tile_set(int nx, int T) { return col_cfg_set(nx, col_elems_get(nx), T); }
int col_elems_set(int nx, int E) { return col_cfg_set(nx, E, col_tile_get(nx)); }

// Rows 128-byte aligned (ld a multiple of 8 complex): tiles of at least 8
// columns where compiled, so each tile row is whole cache lines, written
// with non-temporal stores.
template <bool INV>
static void launch_cols(int nx, int ncol, int nf, double2* data, const double2* tw, hipStream_t s, int ld) {
    int T = col_tile_get(nx);
    const int E = col_elems_get(nx);
    const bool aligned = ld % 8 == 0;
    if (aligned && T < 8 && col_cfg_ok(nx, E, 8)) T = 8;
    const bool nt = aligned && T >= 8;
#define FC2D_COLT(LL, EE, TT)                                                                             \
    if (nx == LL && E == EE && T == TT) {                                                                 \
        const int ntiles = (ncol + TT - 1) / TT;                                                          \
        const bool byf = nf % 8 == 0;                                                                     \
        const dim3 g = byf ? dim3((unsigned)(nf * ntiles)) : dim3(((ntiles + 7) / 8) * 8, nf);            \
        if constexpr (TT >= 8) {                                                                          \
            if (nt) {                                                                                     \
                k_cols<LL, EE, TT, INV, true><<<g, TT * (LL / EE), 0, s>>>(data, ncol, ld, tw, byf ? 1 : 0); \
                return;                                                                                   \
            }                                                                                             \
        }                                                                                                 \
        k_cols<LL, EE, TT, INV, false><<<g, TT * (LL / EE), 0, s>>>(data, ncol, ld, tw, byf ? 1 : 0);     \
        return;                                                                                           \
    }
    FC2D_COLT(16, 2, 4) FC2D_COLT(16, 2, 8) FC2D_COLT(16, 2, 16)
    FC2D_COLT(32, 2, 4) FC2D_COLT(32, 2, 8) FC2D_COLT(32, 2, 16)
    FC2D_COLT(64, 2, 4) FC2D_COLT(64, 2, 8) FC2D_COLT(64, 2, 16)
    FC2D_COLT(128, 2, 4) FC2D_COLT(128, 2, 8)
    FC2D_COLT(256, 4, 4) FC2D_COLT(256, 4, 8)
    FC2D_COLT(512, 4, 4) FC2D_COLT(512, 4, 8) FC2D_COLT(512, 8, 4) FC2D_COLT(512, 8, 8)
    FC2D_COLT(1024, 8, 2) FC2D_COLT(1024, 8, 4) FC2D_COLT(1024, 8, 8)
    FC2D_COLT(1024, 16, 2) FC2D_COLT(1024, 16, 4) FC2D_COLT(1024, 16, 8)
    FC2D_COLT(2048, 8, 1) FC2D_COLT(2048, 8, 2)
    FC2D_COLT(2048, 16, 1) FC2D_COLT(2048, 16, 2) FC2D_COLT(2048, 16, 4)
    FC2D_COLT(4096, 8, 1)
    FC2D_COLT(4096, 16, 1) FC2D_COLT(4096, 16, 2)
#undef FC2D_COLT
}

int fft_prepare(int nx, int ny) {
    return (twiddles(nx) && twiddles(ny)) ? FC2D_OK : FC2D_E_NOMEM;
}

bool fft_ready(int nx, int ny) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    std::lock_guard<std::mutex> lk(g_tw_mu);
    return g_tw.count({dev, nx}) > 0 && g_tw.count({dev, ny}) > 0;
}

int fft_rows_fwd(const fc2d_grid* g, const double* in, double* out, int nf, hipStream_t s, const double* strip,
                 const uint8_t* cls2, int ld) {
    const double2* twy = twiddles(g->ny);
    if (!twy) { set_error("twiddle table allocation failed"); return FC2D_E_NOMEM; }
    launch_rows<true, false>(g->ny / 2, g->nx, nf, in, out, twy, 1.0, strip, cls2, s, ld > 0 ? ld : g->ny / 2 + 1);
    return check(cls2 ? "k_rows_r2c_ext" : "k_rows_r2c", s);
}

int fft_rows_fwd_t(const fc2d_grid* g, const double* in, double* out, int nf, hipStream_t s, const double* strip,
                   const uint8_t* cls2) {
    if (g->ny > 4096 || g->nx % 8) {
        set_error("transposed spectra: rows of at most 4096 points, a multiple of 8 rows");
        return FC2D_E_ARG;
    }
    const double2* twy = twiddles(g->ny);
    if (!twy) { set_error("twiddle table allocation failed"); return FC2D_E_NOMEM; }
    launch_rows<true, true>(g->ny / 2, g->nx, nf, in, out, twy, 1.0, strip, cls2, s, g->ny / 2 + 1);
    return check(cls2 ? "k_rows_r2c_ext" : "k_rows_r2c", s);
}

int fft_cols(const fc2d_grid* g, double* data, int nf, bool inv, hipStream_t s, int ld) {
    const double2* twx = twiddles(g->nx);
    if (!twx) { set_error("twiddle table allocation failed"); return FC2D_E_NOMEM; }
    const int ncol = g->ny / 2 + 1;
    if (inv) launch_cols<true>(g->nx, ncol, nf, (double2*)data, twx, s, ld > 0 ? ld : ncol);
    else launch_cols<false>(g->nx, ncol, nf, (double2*)data, twx, s, ld > 0 ? ld : ncol);
    return check(inv ? "k_cols_inv" : "k_cols", s);
}

int fft_rows_inv(const fc2d_grid* g, const double* in, double* out, int nf, hipStream_t s, int ld) {
    const double2* twy = twiddles(g->ny);
    if (!twy) { set_error("twiddle table allocation failed"); return FC2D_E_NOMEM; }
    launch_rows<false, false>(g->ny / 2, g->nx, nf, in, out, twy, 1.0 / ((double)g->nx * (double)g->ny), nullptr,
                              nullptr, s, ld > 0 ? ld : g->ny / 2 + 1);
    return check("k_rows_c2r", s);
}

int fft_rows_inv_t(const fc2d_grid* g, const double* in, double* out, int nf, hipStream_t s) {
    if (g->ny > 4096 || g->nx % 8) {
        set_error("transposed spectra: rows of at most 4096 points, a multiple of 8 rows");
        return FC2D_E_ARG;
    }
    const double2* twy = twiddles(g->ny);
    if (!twy) { set_error("twiddle table allocation failed"); return FC2D_E_NOMEM; }
    launch_rows<false, true>(g->ny / 2, g->nx, nf, in, out, twy, 1.0 / ((double)g->nx * (double)g->ny), nullptr,
                             nullptr, s, g->ny / 2 + 1);
    return check("k_rows_c2r", s);
}

int fft2_r2c(const fc2d_grid* g, const double* in, double* out, int nf, hipStream_t s, const double* strip,
             const uint8_t* cls2, int ld) {
    int st = fft_rows_fwd(g, in, out, nf, s, strip, cls2, ld);
    if (st) return st;
    return fft_cols(g, out, nf, false, s, ld);
}

int fft2_c2r(const fc2d_grid* g, double* in, double* out, int nf, hipStream_t s, int ld) {
    int st = fft_cols(g, in, nf, true, s, ld);
    if (st) return st;
    return fft_rows_inv(g, in, out, nf, s, ld);
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

// Propagation of a mode by t (eq. wave_2d_ff): with w = 2 pi c |k| the
// spectra (f0, f1) = (u_hat, u_t_hat) map to
//     (cos(w t) f0 + sin(w t)/w f1,  -w sin(w t) f0 + cos(w t) f1),
// and to (f0 + t f1, f1) for the zero mode.  The factors depend only on
// (|l|, m) (row i and row nx - i share them): FFCoef holds them for one pair.
struct FFCoef {
    double cw, sinc, mw;
};

// factors of the modes with |row frequency| la and column frequency m
// (iLx = 1 / Lx, iLy = 1 / Ly)
__device__ __forceinline__ FFCoef ff_coef(int la, int m, double iLx, double iLy, double c, double t) {
    FFCoef k;
    if (la == 0 && m == 0) {
        k.cw = 1.0;
        k.sinc = t;
        k.mw = 0.0;
        return k;
    }
    const double a = (double)la * iLx, b = (double)m * iLy;
    const double wpi = 2.0 * c * sqrt(a * a + b * b);   // w / pi
    const double w = M_PI * wpi;
    // sin(w t), cos(w t) as sincospi(t w / pi): an exact argument reduction
    // without the large-argument path of sincos
    double sw, cw;
    sincospi(wpi * t, &sw, &cw);
    k.cw = cw;
    k.sinc = sw / w;
    k.mw = -w * sw;
    return k;
}

__device__ __forceinline__ void ff_apply(const FFCoef& k, double2 f0, double2 f1, double2* ra, double2* rt) {
    *ra = make_double2(k.cw * f0.x + k.sinc * f1.x, k.cw * f0.y + k.sinc * f1.y);
    *rt = make_double2(k.mw * f0.x + k.cw * f1.x, k.mw * f0.y + k.cw * f1.y);
}

// |row frequency| of row i of an nx-point transform
__device__ __forceinline__ int row_freq(int i, int nx) { return i <= nx / 2 ? i : nx - i; }

__global__ void k_ff(const double2* u0, const double2* u1, double2* uh, double2* uth, int64_t n, int nx, int ny,
                     double h, double c, double t) {
    const int ncol = ny / 2 + 1;
    const double iLx = 1.0 / (nx * h), iLy = 1.0 / (ny * h);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        int i, j;
        mode_of(e, nx, ncol, &i, &j);
        double2 ra, rt;
        ff_apply(ff_coef(row_freq(i, nx), j, iLx, iLy, c, t), u0[e], u1[e], &ra, &rt);
        uh[e] = ra;
        if (uth) uth[e] = rt;   // uth may be NULL when only the field is wanted
    }
}

// Inverse column pass of a propagated spectrum with the propagation fused into
// its loads: out (row-major half spectrum, columns transformed back along x)
// = the inverse column transform of cos(w t) u0_hat + sin(w t) / w u1_hat, the
// same sums as ff_apply followed by the inverse column pass of that length.
template <int L, int E, int T>
__global__ __launch_bounds__(T * (L / E)) void k_cols_prop(const double2* __restrict__ u0, const double2* __restrict__ u1,
                                                           double2* __restrict__ out, int ncol, double Lx, double Ly,
                                                           double c, double t, int by_field) {
    __shared__ double2 lds[L * T];
    const int q = threadIdx.x % T;
    const int tt = threadIdx.x / T;
    const int ntiles = (ncol + T - 1) / T;
    int tile, field;
    if (!col_block(ntiles, by_field != 0, &tile, &field)) return;   // uniform per block
    const int col = tile * T + q;
    const bool live = col < ncol;
    const int cl = live ? col : 0;
    const int64_t base = (int64_t)field * L * ncol + cl;
    const double iLx = 1.0 / Lx, iLy = 1.0 / Ly;
    double2 v[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const int r = in_index<L, E>(k, tt);
        double2 rt;
        ff_apply(ff_coef(row_freq(r, L), cl, iLx, iLy, c, t), u0[base + (int64_t)r * ncol],
                 u1[base + (int64_t)r * ncol], &v[k], &rt);
    }
    StockhamFrom<L, E, 1, true>::run(v, lds, 1, T, q, tt, nullptr, L);
    if (!live) return;
#pragma unroll
    for (int k = 0; k < E; ++k) out[base + (int64_t)out_index<L, E>(k, tt) * ncol] = v[k];
}

int prop_c2r(const fc2d_grid* g, double c, double t, const double* u0, const double* u1, double* spec, double* out,
             int nf, hipStream_t s) {
    const int ncol = g->ny / 2 + 1;
    const double Lx = g->nx * g->h, Ly = g->ny * g->h;
    const int E = col_elems_get(g->nx), T = col_tile_get(g->nx);
    bool done = false;
#define FC2D_COLPROP(LL, EE, TT)                                                                              \
    if (!done && g->nx == LL && E == EE && T == TT) {                                                        \
        const int ntiles = (ncol + TT - 1) / TT;                                                             \
        const bool byf = nf % 8 == 0;                                                                        \
        const dim3 grid = byf ? dim3((unsigned)(nf * ntiles)) : dim3(((ntiles + 7) / 8) * 8, nf);            \
        k_cols_prop<LL, EE, TT><<<grid, TT * (LL / EE), 0, s>>>((const double2*)u0, (const double2*)u1,      \
                                                               (double2*)spec, ncol, Lx, Ly, c, t,          \
                                                               byf ? 1 : 0);                                 \
        done = true;                                                                                         \
    }
    FC2D_COLPROP(256, 4, 4) FC2D_COLPROP(256, 4, 8) FC2D_COLPROP(512, 4, 4) FC2D_COLPROP(512, 4, 8)
    FC2D_COLPROP(512, 8, 4) FC2D_COLPROP(512, 8, 8) FC2D_COLPROP(1024, 8, 4) FC2D_COLPROP(1024, 16, 2)
    FC2D_COLPROP(1024, 16, 4) FC2D_COLPROP(2048, 16, 1) FC2D_COLPROP(2048, 16, 2)
#undef FC2D_COLPROP
    int st;
    if (done) {
        if ((st = check("k_cols_prop", s))) return st;
    } else {   // other lengths and launch shapes: propagation, then the inverse column pass
        if ((st = ff_apply(g, c, t, u0, u1, spec, nullptr, nf, s))) return st;
        if ((st = fft_cols(g, spec, nf, true, s))) return st;
    }
    return fft_rows_inv(g, spec, out, nf, s);
}

// Column pass fused with the propagation, for spectra whose rows are already
// transformed (the middle of a Fourier-Forwarding step): a block takes the
// same T/2 adjacent columns of u_hat and of u_t_hat of one field, transforms
// them along x, propagates every mode by t (the partner value comes through
// LDS), transforms back along x and writes both in place.  Replaces forward
// column pass + propagation + inverse column pass (three reads and writes of
// both spectra) by one.
// TRANS: spectra stored transposed (tpos: each column nx/8 whole 128-byte
// lines), as the transposed row passes write and read them.
template <int L, int E, int T, bool TRANS>
__global__ __launch_bounds__(T * (L / E), 4) void k_cols_ff(double2* __restrict__ su, double2* __restrict__ sut,
                                                         int ncol, int nx, double Lx, double Ly, double c, double t,
                                                         int by_field) {
    constexpr int H = T / 2;
    __shared__ double2 lds[L * T];
    const int q = threadIdx.x % T;
    const int tt = threadIdx.x / T;
    const int comp = q / H;            // 0: u_hat, 1: u_t_hat
    const int ntiles = (ncol + H - 1) / H;
    int tile, field;
    if (!col_block(ntiles, by_field != 0, &tile, &field)) return;   // uniform per block
    const int col = tile * H + q % H;
    const bool live = col < ncol;
    const int cl = live ? col : 0;
    double2* sp = comp ? sut : su;
    // element r of the block's column
    auto at = [&](int r) -> int64_t {
        return TRANS ? tpos(field, cl, r, L, ncol) : (int64_t)field * L * ncol + cl + (int64_t)r * ncol;
    };
    double2 v[E];
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = sp[at(in_index<L, E>(k, tt))];
    StockhamFrom<L, E, 1, false>::run(v, lds, 1, T, q, tt, nullptr, L);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) lds[swz(out_index<L, E>(k, tt) * T + q)] = v[k];
    __syncthreads();
    // propagate every (row i, column pair) in LDS; one |row frequency| at a
    // time (rows la and L - la share the factors) keeps the transcendental work
    // out of the unrolled register code and computes each factor once
    const int tile_col0 = tile * H;
    const double iLx = 1.0 / Lx, iLy = 1.0 / Ly;
#pragma unroll 1
    for (int e = threadIdx.x; e < (L / 2 + 1) * H; e += T * (L / E)) {
        const int la = e / H, cq = e % H;
        const FFCoef k = ff_coef(la, tile_col0 + cq, iLx, iLy, c, t);
        const int a = swz(la * T + cq), b = swz(la * T + cq + H);
        double2 ra, rt;
        ff_apply(k, lds[a], lds[b], &ra, &rt);
        lds[a] = ra;
        lds[b] = rt;
        if (la > 0 && la < L / 2) {
            const int a2 = swz((L - la) * T + cq), b2 = swz((L - la) * T + cq + H);
            ff_apply(k, lds[a2], lds[b2], &ra, &rt);
            lds[a2] = ra;
            lds[b2] = rt;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = lds[swz(in_index<L, E>(k, tt) * T + q)];
    __syncthreads();   // the inverse transform reuses lds
    StockhamFrom<L, E, 1, true>::run(v, lds, 1, T, q, tt, nullptr, L);
    if (!live) return;
#pragma unroll
    for (int k = 0; k < E; ++k) sp[at(out_index<L, E>(k, tt))] = v[k];
}

// The same fused step with one column of u_hat and the same column of u_t_hat
// per block, both transformed by the same threads with the same index
// pattern: after the forward transforms each thread holds both spectra at the
// same modes, so the propagation happens in registers (no partner exchange),
// and the two transforms take turns on one column of LDS (16 L bytes for L / E
// threads: at L = 2048 five blocks fit a CU where the two-spectra kernel fits
// two).
template <int L, int E, bool TRANS>
__global__ __launch_bounds__(L / E) void k_cols_ffp(double2* __restrict__ su, double2* __restrict__ sut, int ncol,
                                                   double Lx, double Ly, double c, double t, int by_field) {
    __shared__ double2 lds[L];
    const int tt = threadIdx.x;
    int col, field;
    if (!col_block(ncol, by_field != 0, &col, &field)) return;   // uniform per block
    // element r of the block's column
    auto at = [&](int r) -> int64_t {
        return TRANS ? tpos(field, col, r, L, ncol) : (int64_t)field * L * ncol + col + (int64_t)r * ncol;
    };
    double2 a[E], b[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
        a[k] = su[at(in_index<L, E>(k, tt))];
        b[k] = sut[at(in_index<L, E>(k, tt))];
    }
    StockhamFrom<L, E, 1, false>::run(a, lds, 1, 1, 0, tt, nullptr, L);
    __syncthreads();   // the last stage of a may still read lds
    StockhamFrom<L, E, 1, false>::run(b, lds, 1, 1, 0, tt, nullptr, L);
    // a[k], b[k]: row out_index(k, tt) of both spectra
    const double iLx = 1.0 / Lx, iLy = 1.0 / Ly;
#pragma unroll
    for (int k = 0; k < E; ++k)
        ff_apply(ff_coef(row_freq(out_index<L, E>(k, tt), L), col, iLx, iLy, c, t), a[k], b[k], &a[k], &b[k]);
    // inverse transforms in turn: to the input order through lds, transform, write
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) lds[swz(out_index<L, E>(k, tt))] = a[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) a[k] = lds[swz(in_index<L, E>(k, tt))];
    __syncthreads();
    StockhamFrom<L, E, 1, true>::run(a, lds, 1, 1, 0, tt, nullptr, L);
#pragma unroll
    for (int k = 0; k < E; ++k) su[at(out_index<L, E>(k, tt))] = a[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) lds[swz(out_index<L, E>(k, tt))] = b[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) b[k] = lds[swz(in_index<L, E>(k, tt))];
    __syncthreads();
    StockhamFrom<L, E, 1, true>::run(b, lds, 1, 1, 0, tt, nullptr, L);
#pragma unroll
    for (int k = 0; k < E; ++k) sut[at(out_index<L, E>(k, tt))] = b[k];
}

// shapes of the fused kernel per length 2^lg (elements per thread and columns
// per block of k_cols_ff, then the paired k_cols_ffp shapes): g_colff_var[lg]
// indexes the compiled list of that length
static int g_colff_var[14] = {0};

int colff_variants(int nx) {
    switch (nx) {
        case 256: case 512: return 3;
        case 1024: return 6;
        case 2048: return 6;
        case 4096: return 2;
        case 16: case 32: case 64: case 128: return 1;
    }
    return 0;
}
int colff_get(int nx) { int lg = 0; while ((1 << lg) < nx) ++lg; return lg <= 13 ? g_colff_var[lg] : 0; }
int colff_set(int nx, int v) {
    if (v < 0 || v >= colff_variants(nx)) return FC2D_E_ARG;
    int lg = 0;
    while ((1 << lg) < nx) ++lg;
    g_colff_var[lg] = v;
    return FC2D_OK;
}

int cols_ff(const fc2d_grid* g, double c, double t, double* su, double* sut, int nf, hipStream_t s, bool trans) {
    const int ncol = g->ny / 2 + 1;
    const double Lx = g->nx * g->h, Ly = g->ny * g->h;
    const int var = colff_get(g->nx);
#define FC2D_COLFF(LL, VV, EE, TT)                                                                            \
    if (g->nx == LL && var == VV) {                                                                          \
        const int ntiles = (ncol + TT / 2 - 1) / (TT / 2);                                                   \
        const bool byf = nf % 8 == 0;                                                                        \
        const dim3 grid = byf ? dim3((unsigned)(nf * ntiles)) : dim3(((ntiles + 7) / 8) * 8, nf);            \
        if (trans)                                                                                           \
            k_cols_ff<LL, EE, TT, true><<<grid, TT * (LL / EE), 0, s>>>((double2*)su, (double2*)sut, ncol,   \
                                                                       g->nx, Lx, Ly, c, t, byf ? 1 : 0);   \
        else                                                                                                 \
            k_cols_ff<LL, EE, TT, false><<<grid, TT * (LL / EE), 0, s>>>((double2*)su, (double2*)sut, ncol,  \
                                                                        g->nx, Lx, Ly, c, t, byf ? 1 : 0);  \
        return check("k_cols_ff", s);                                                                        \
    }
    FC2D_COLFF(16, 0, 2, 8) FC2D_COLFF(32, 0, 2, 8) FC2D_COLFF(64, 0, 2, 8) FC2D_COLFF(128, 0, 2, 8)
    FC2D_COLFF(256, 0, 4, 8) FC2D_COLFF(256, 1, 4, 4) FC2D_COLFF(256, 2, 2, 8)
    FC2D_COLFF(512, 0, 8, 8) FC2D_COLFF(512, 1, 8, 4) FC2D_COLFF(512, 2, 4, 8)
    FC2D_COLFF(1024, 0, 8, 4) FC2D_COLFF(1024, 1, 8, 8) FC2D_COLFF(1024, 2, 16, 4)
    FC2D_COLFF(1024, 4, 8, 2) FC2D_COLFF(1024, 5, 16, 2)
    FC2D_COLFF(2048, 0, 8, 2) FC2D_COLFF(2048, 1, 8, 4) FC2D_COLFF(2048, 2, 16, 2) FC2D_COLFF(2048, 3, 16, 4)
    FC2D_COLFF(4096, 0, 16, 2)
#undef FC2D_COLFF
#define FC2D_COLFFP(LL, VV, EE)                                                                               \
    if (g->nx == LL && var == VV) {                                                                          \
        const bool byf = nf % 8 == 0;                                                                        \
        const dim3 grid = byf ? dim3((unsigned)(nf * ncol)) : dim3(((ncol + 7) / 8) * 8, nf);                \
        if (trans)                                                                                           \
            k_cols_ffp<LL, EE, true><<<grid, LL / EE, 0, s>>>((double2*)su, (double2*)sut, ncol, Lx, Ly, c, t, \
                                                              byf ? 1 : 0);                                  \
        else                                                                                                 \
            k_cols_ffp<LL, EE, false><<<grid, LL / EE, 0, s>>>((double2*)su, (double2*)sut, ncol, Lx, Ly, c,  \
                                                               t, byf ? 1 : 0);                              \
        return check("k_cols_ff", s);                                                                        \
    }
    FC2D_COLFFP(1024, 3, 8) FC2D_COLFFP(2048, 4, 8) FC2D_COLFFP(2048, 5, 16) FC2D_COLFFP(4096, 1, 16)
#undef FC2D_COLFFP
    set_error("cols_ff: unsupported length");
    return FC2D_E_ARG;
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
