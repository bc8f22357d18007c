// Cartesian Evaluation kernels (Sec. 3.5 steps 5-6).
//
//  k_match   four lanes per (normal p, field): the red-star values along the
//            grid lines, the matching values along the normal (Sec. 3.2) and
//            c_p = Q^T f_{D_p}, each a compensated dot product with
//            double-double weights (rounded once); the stencil values are
//            gathered in address order and exchanged through LDS.
//  k_strip   one thread per two STRIP points (consecutive in foot-parameter
//            order, sharing most of their normals) looping over a chunk of
//            fields, the block's Gram records staged in LDS: interpolation onto
//            H n V+ (Sec. 3.4).  Because every normal carries the same level weights
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
#include <mutex>
#include <string>

#include "dd.h"
#include "internal.h"
#include "lagrange_dev.h"

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

// LDS slot of stencil value (star s, node k) in the block of group gi (M * M
// doubles per group): the node pairs (k even, k + 1) of a star are permuted by
// an XOR with bits of the star and the group, so the 16-byte reads of the 8
// lanes of two neighbouring groups (stars s = sq, sq + 4 at the same k) fall
// in different banks
template <int M>
__device__ __forceinline__ int xg_index(int s, int k, int gi) {
    if constexpr (M == 8) {
        const int sw = ((s & 3) >> 1) | ((gi & 1) << 1);
        return s * 8 + ((((k >> 1) ^ sw) << 1) | (k & 1));
    } else {
        return s * M + k;
    }
}

// Matching values and Gram coefficients of normal p for field f, computed by
// the 4 consecutive lanes sq = 0..3 of a group.
//  1. Gather: the normal's M*M stencil values (star s, node k) are listed in
//     order of their address (plan: mref, mlab); lane sq loads list entries
//     4u + sq, u = 0, 1, ..., so the four lanes of a load read neighbouring
//     addresses, and stores each value in the group's LDS block xg at s M + k.
//  2. Red stars (first interpolation, along the grid lines): lane sq forms
//     stars sq, sq + 4, ... from xg; the others travel by cross-lane shuffles.
//     With boundary data the M-th node along the normal is the point on Gamma
//     (the boundary sample; its stencil entries are padding), otherwise a star.
//  3. Matching values along the normal (second interpolation) q = sq, sq + 4, ...
//     (q < d - 1; q < d for a plan built from interior data only, io = 1,
//     where the value on Gamma is interpolated too instead of read from bv)
//  4. Gram coefficients c_j, j = sq, sq + 4, ...
// Every sum is a Dot2 over the stencil in node / star order, as in a one-lane
// evaluation.  DT > 0 fixes d = DT at compile time; DT = 0 takes d = Drt.
// `live` lanes store; the others only take part in the shuffles.  The caller
// is one 64-lane block (16 groups); the LDS exchange is fenced by barriers.
template <int M, int DT>
__device__ __forceinline__ void match_group(const int32_t* __restrict__ mref, const uint8_t* __restrict__ mlab,
                                            const double* __restrict__ mwv, const double* __restrict__ mwn,
                                            const double* __restrict__ Q, int Drt, int B, int io,
                                            const double* __restrict__ g, const double* __restrict__ bv, int p,
                                            int sq, bool live, double* __restrict__ co, double* __restrict__ fo,
                                            double* xg) {
    const int D = DT > 0 ? DT : Drt;
    constexpr int NU = (M * M + 15) / 16 * 4;   // list entries per lane (a multiple of 4)
    const int lane = threadIdx.x & 63;
    const int gbase = lane & ~3;
    const int gi = lane >> 2;
    // 1. gather in address order (entries and labels read as 16- and 4-byte words)
    {
        const int4* ref4 = (const int4*)(mref + ((int64_t)p * 4 + sq) * NU);
        const uint32_t* lab4 = (const uint32_t*)(mlab + ((int64_t)p * 4 + sq) * NU);
        int32_t rr[NU];
        int slot[NU];
#pragma unroll
        for (int u4 = 0; u4 < NU / 4; ++u4) {
            const int4 r = ref4[u4];
            const uint32_t l = lab4[u4];
            rr[4 * u4] = r.x; rr[4 * u4 + 1] = r.y; rr[4 * u4 + 2] = r.z; rr[4 * u4 + 3] = r.w;
#pragma unroll
            for (int b = 0; b < 4; ++b) slot[4 * u4 + b] = (l >> (8 * b)) & 255;
        }
        double val[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u)
            val[u] = slot[u] < M * M ? *(rr[u] >= 0 ? g + rr[u] : bv + B + (-rr[u] - 1)) : 0.0;
#pragma unroll
        for (int u = 0; u < NU; ++u)
            if (slot[u] < M * M) xg[xg_index<M>(slot[u] / M, slot[u] % M, gi)] = val[u];
    }
    __syncthreads();
    // 2. red-star values along the grid lines (Sec. 3.2, first interpolation): stars sq, sq + 4, ...
    constexpr int RS = (M + 3) / 4;   // stars per lane
    const double* wv = mwv + (int64_t)p * RS * M * 4 * 2;   // [r][k][sq] double-double
    dd mine[RS];
#pragma unroll
    for (int r = 0; r < RS; ++r) {
        const int s = sq + 4 * r;
        Acc2 a;
        if (s < M) {
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const int o = (r * M + k) * 4 + sq;
                a.add(dd{wv[2 * o], wv[2 * o + 1]}, xg[xg_index<M>(s, k, gi)]);
            }
        }
        mine[r] = a.result();
    }
    __syncthreads();   // xg may be overwritten by the caller's next item
    dd star[M];
#pragma unroll
    for (int s = 0; s < M; ++s) {
        const int src = gbase + (s & 3);
        const dd v = mine[s >> 2];
        star[s] = dd{__shfl(v.hi, src, 64), __shfl(v.lo, src, 64)};
    }
    // with boundary data the last node along the normal is the point on Gamma
    // (depth 0): its value is the boundary sample, not a red star
    const double fbs = io ? 0.0 : bv[p];   // boundary sample (not read from interior data only)
    if (!io) star[M - 1] = dd{fbs, 0.0};
    // 3. matching values along the normal (second interpolation)
    const int NQ = D - 1 + io;   // matching values interpolated along the normal
    const int RQ = (NQ + 3) / 4;
    const double* wn = mwn + (int64_t)p * RQ * M * 4 * 2;   // [r][s][sq] double-double
    dd fq[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const int q = sq + 4 * r;
        Acc2 a;
        if (q < NQ) {
#pragma unroll
            for (int s = 0; s < M; ++s) {
                const int o = (r * M + s) * 4 + sq;
                a.add(dd{wn[2 * o], wn[2 * o + 1]}, star[s]);
            }
        }
        fq[r] = q < NQ ? a.result() : dd{fbs, 0.0};
    }
    dd fD[12];
    double fbp = fbs;   // f_{D_p}[d-1]: the sample, or its interpolated value
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        if (q < D) {
            const int src = gbase + (q & 3);
            const dd v = (q < 4) ? fq[0] : ((q < 8) ? fq[1] : fq[2]);
            const dd x = dd{__shfl(v.hi, src, 64), __shfl(v.lo, src, 64)};
            fD[q] = q < NQ ? x : dd{fbs, 0.0};
            if (q == D - 1) fbp = fD[q].hi;
        }
    }
    // 4. c_p = Q^T f_{D_p}, stored with the boundary value appended: [c_0..c_{d-1}, f_{D_p}[d-1], 0 pad]
    const int DP = (D + 2) & ~1;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const int j = sq + 4 * r;
        if (j < D) {
            Acc2 a;
#pragma unroll
            for (int q = 0; q < 12; ++q)
                if (q < D) a.add(fD[q], Q[q * D + j]);
            if (live) co[j] = a.result().hi;
        }
    }
    if (live && sq == 0) {
        co[D] = fbp;
        if (DP > D + 1) co[D + 1] = 0.0;
    }
    if (live && fo) {
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const int q = sq + 4 * r;
            if (q < D) fo[q] = fq[r].hi;   // this lane's own value (the boundary value for q = d-1)
        }
    }
}

// Consecutive normals share grid lines: each XCD (blocks are dealt
// round-robin to the 8 XCDs) gets a contiguous range of normals so they share
// an L2.  Local work index l -> normal.
__device__ __forceinline__ int xcd_normal(int l, int B) {
    const int per_xcd = (B + 7) / 8;
    return (l % 8) * per_xcd + l / 8;
}

// A wave (one block) takes NPW consecutive normals and 16 / NPW fields, 4
// lanes per (normal, field) (as in match_group).  With NPW = 1 the normal's
// references and weights are shared by the wave; with NPW > 1 the lanes of one
// field gather from overlapping stencils, so fewer distinct lines.
template <int M, int DT, int NPW>
__global__ __launch_bounds__(64) void k_match(const int32_t* __restrict__ mref, const uint8_t* __restrict__ mlab,
                                              const double* __restrict__ mwv, const double* __restrict__ mwn,
                                              const double* __restrict__ Q, int D, int B, int io,
                                              const double* __restrict__ fg, int64_t npts,
                                              const double* __restrict__ fb, int64_t nbdry, int nf,
                                              double* __restrict__ c_out, double* __restrict__ fD_out) {
    __shared__ __attribute__((aligned(16))) double xg[16 * M * M];
    constexpr int FPW = 16 / NPW;
    const int nq = (B + NPW - 1) / NPW;
    const int qd = xcd_normal(blockIdx.x, nq);
    if (qd >= nq) return;   // uniform per block
    const int gi = threadIdx.x / 4;
    const int pn = qd * NPW + gi / FPW;
    const int fl = blockIdx.y * FPW + gi % FPW;
    const bool live = fl < nf && pn < B;
    const int f = fl < nf ? fl : 0;
    const int p = pn < B ? pn : B - 1;
    const int DP = (D + 2) & ~1;
    match_group<M, DT>(mref, mlab, mwv, mwn, Q, D, B, io, fg + (int64_t)f * npts, fb ? fb + (int64_t)f * nbdry : fb, p,
                       threadIdx.x & 3, live, c_out + ((int64_t)f * B + p) * DP,
                       fD_out ? fD_out + ((int64_t)f * B + p) * D : nullptr, xg + gi * M * M);
}

// Persistent form over several plans (a batch): work item w covers four
// consecutive normals x four fields of one plan (as k_match with NPW = 4);
// items of plan k start at a multiple of 8 so the XCD assignment is kept.
// Every block loops until the items run out.
template <int M, int DT>
__global__ __launch_bounds__(64) void k_match_multi(const PlanDev* __restrict__ pd, int np, int64_t total) {
    __shared__ __attribute__((aligned(16))) double xg[16 * M * M];
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        int k = 0;
        while (k + 1 < np && pd[k + 1].off_match <= w) ++k;
        const PlanDev& P = pd[k];
        const int64_t l = w - P.off_match;
        const int nq = (P.B + 3) / 4;
        const int padQ = (nq + 7) & ~7;
        const int qd = xcd_normal((int)(l % padQ), nq);
        if (qd >= nq) continue;   // uniform per block
        const int gi = threadIdx.x / 4;
        const int pn = qd * 4 + gi / 4;
        const int fl = (int)(l / padQ) * 4 + gi % 4;
        const bool live = fl < P.nf && pn < P.B;
        const int f = fl < P.nf ? fl : 0;
        const int p = pn < P.B ? pn : P.B - 1;
        const int DP = (P.D + 2) & ~1;
        match_group<M, DT>(P.mref, P.mlab, P.mwv, P.mwn, P.Q, P.D, P.B, P.io, P.u + (int64_t)f * P.npts,
                           P.fb + (int64_t)f * P.nbdry, p, threadIdx.x & 3, live, P.c + ((int64_t)f * P.B + p) * DP,
                           nullptr, xg + gi * M * M);
    }
}

// F[l, p] = (A_r c_p)_{l-1}, l >= 1; F[0, p] = f_{D_p}[d-1] (stored after c_p)
__global__ void k_blend(const double* __restrict__ c, const double* __restrict__ Ar, int D, int B, int Cr,
                        double* __restrict__ F) {
    const int64_t n = (int64_t)(Cr + 1) * B;
    const int f = blockIdx.y;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int l = (int)(k / B);
        const int p = (int)(k - (int64_t)l * B);
        const int DP = (D + 2) & ~1;
        double v;
        if (l == 0) {
            v = c[((int64_t)f * B + p) * DP + D];
        } else {
            v = 0.0;
            for (int j = 0; j < D; ++j) v += Ar[(l - 1) * D + j] * c[((int64_t)f * B + p) * DP + j];
        }
        F[(int64_t)f * n + k] = v;
    }
}

// Per-point part of the interpolation at STRIP point k: theta weights w over
// S_{theta^Q} (nodes p0 - kl .. p0 - kl + M - 1), the factored level vector u
// (u[j] = sum_l v_l A_r[l-1, j], u[d] = v_0 at level 0) and the grid index.
// DT > 0 fixes d = DT at compile time (straight-line code); DT = 0 takes d = Drt.
template <int M>
struct StripPt {
    double w[M];
    double u[13];   // d + 1 <= 13 entries
    int p0;
    int32_t idx;
};

// First normal index of the stencil window of foot parameter th (before the
// shift by kl): the interval [p0 k2, (p0 + 1) k2) for even M, the nearest node for odd M
template <int M>
__device__ __forceinline__ int strip_p0(double th, double k2) {
    return (M % 2 == 0) ? (int)floor(th / k2) : (int)rint(th / k2);
}

template <int M, int DT>
__device__ __forceinline__ void strip_setup(const int32_t* __restrict__ sidx, const double* __restrict__ sth,
                                            const double* __restrict__ seta, int64_t k, const double* sAr, int Drt,
                                            int Cr, double k2, double lev_scale, StripPt<M>& P) {
    const int D = DT > 0 ? DT : Drt;
    const double th = sth[k];
    const double eta = seta[k];
    P.idx = sidx[k];
    constexpr int kl = (M - 1) / 2;
    P.p0 = strip_p0<M>(th, k2);
    equi_weights<M>((th - (double)(P.p0 - kl) * k2) / k2, P.w);
    // level weights at s = eta n_r / k1 (nodes l0..l0+M-1) and u = A_r^T v (factored blend)
    const double s = eta * lev_scale;
    int l0 = (int)floor(s) - M / 2 + 1;
    l0 = l0 < 0 ? 0 : (l0 > Cr - M + 1 ? Cr - M + 1 : l0);
    double v[M];
    equi_weights<M>(s - (double)l0, v);
#pragma unroll
    for (int j = 0; j < 13; ++j) P.u[j] = 0.0;
#pragma unroll
    for (int l = 0; l < M; ++l) {
        const int lev = l0 + l;            // level 0 is the boundary value, not a row of A_r
        const double vl = lev >= 1 ? v[l] : 0.0;
        const double* row = sAr + (lev >= 1 ? lev - 1 : 0) * D;
#pragma unroll
        for (int j = 0; j < 12; ++j)
            if (j < D) P.u[j] += vl * row[j];
    }
    // slot D of each normal's record holds its boundary value: weight v_0 when l0 = 0
    P.u[D] = (l0 == 0) ? v[0] : 0.0;
}

// u . c_q for the Gram record of normal q (slots 0..d-1 = c, slot d = boundary value)
__device__ __forceinline__ double record_dot(const double* __restrict__ cf, int q, int DP, const double* u) {
    const double2* rec = (const double2*)(cf + (int64_t)q * DP);
    double g = 0.0;
#pragma unroll
    for (int j2 = 0; j2 < 7; ++j2) {   // DP <= 14
        if (2 * j2 < DP) {
            const double2 cc = rec[j2];
            g += u[2 * j2] * cc.x + u[2 * j2 + 1] * cc.y;
        }
    }
    return g;
}

__device__ __forceinline__ int wrap_index(int q, int B) {
    q %= B;
    return q < 0 ? q + B : q;
}

// Two STRIP points A, Bp (hasb = false: A only) for fields [f0, f1) (one
// thread).  The Gram record of normal q (unwrapped index) for field f is read
// at base + (f - f0) fstride + r DP, r = q - qoff when the records are staged
// (STAGED: a window of consecutive normals in LDS), else r = q mod B (the
// plan's record array).  The points are consecutive in foot-parameter order,
// so their stencils usually start at the same or the next normal: then the
// M + 1 records of the shared window are read once for both points.
template <int M, int DT, bool STAGED>
__device__ __forceinline__ void strip_pair_fields(const StripPt<M>& A, const StripPt<M>& Bp, bool hasb, int Drt,
                                                  int B, const double* base, int64_t fstride, int qoff,
                                                  double* __restrict__ out, int64_t npts, int f0, int f1) {
    const int D = DT > 0 ? DT : Drt;
    constexpr int kl = (M - 1) / 2;
    const int DP = (D + 2) & ~1;
    const int dlt = Bp.p0 - A.p0;
    auto rec_index = [&](int q) { return STAGED ? q - qoff : wrap_index(q, B); };
    if (hasb && (dlt == 0 || dlt == 1)) {
        double wa[M + 1], wb[M + 1];
        int pj[M + 1];
#pragma unroll
        for (int m = 0; m <= M; ++m) {
            wa[m] = m < M ? A.w[m] : 0.0;
            wb[m] = dlt == 0 ? (m < M ? Bp.w[m] : 0.0) : (m >= 1 ? Bp.w[m - 1] : 0.0);
            pj[m] = rec_index(A.p0 - kl + m) * DP;
        }
#pragma unroll 1
        for (int f = f0; f < f1; ++f) {
            const double* cf = base + (int64_t)(f - f0) * fstride;
            double ea = 0.0, eb = 0.0;
#pragma unroll
            for (int m = 0; m <= M; ++m) {
                const double2* rec = (const double2*)(cf + pj[m]);
                double ga = 0.0, gb = 0.0;
#pragma unroll
                for (int j2 = 0; j2 < 7; ++j2) {   // DP <= 14
                    if (2 * j2 < DP) {
                        const double2 cc = rec[j2];
                        ga += A.u[2 * j2] * cc.x + A.u[2 * j2 + 1] * cc.y;
                        gb += Bp.u[2 * j2] * cc.x + Bp.u[2 * j2 + 1] * cc.y;
                    }
                }
                ea += wa[m] * ga;
                eb += wb[m] * gb;
            }
            out[(int64_t)f * npts + A.idx] = ea;
            out[(int64_t)f * npts + Bp.idx] = eb;
        }
        return;
    }
    // stencils apart (or a single point): one window each
    int pa[M], pb[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        pa[m] = rec_index(A.p0 - kl + m);
        pb[m] = rec_index(Bp.p0 - kl + m);
    }
#pragma unroll 1
    for (int f = f0; f < f1; ++f) {
        const double* cf = base + (int64_t)(f - f0) * fstride;
        double ea = 0.0, eb = 0.0;
#pragma unroll
        for (int m = 0; m < M; ++m) ea += A.w[m] * record_dot(cf, pa[m], DP, A.u);
        out[(int64_t)f * npts + A.idx] = ea;
        if (hasb) {
#pragma unroll
            for (int m = 0; m < M; ++m) eb += Bp.w[m] * record_dot(cf, pb[m], DP, Bp.u);
            out[(int64_t)f * npts + Bp.idx] = eb;
        }
    }
}

// Gram records of the normals q0 .. q0 + L - 1 (wrapped mod B) for fields
// [f0, f0 + nfs) copied to LDS: record r of local field f at st + (f lcap + r) DP.
__device__ __forceinline__ void stage_records(const double* __restrict__ c, int B, int DP, int q0, int L, int lcap,
                                              int f0, int nfs, double* st) {
    const int per = L * DP / 2;   // 16-byte parts per field (DP is even)
    for (int e = threadIdx.x; e < nfs * per; e += blockDim.x) {
        const int f = e / per;
        const int h = 2 * (e - f * per);
        const int r = h / DP;
        const int j = h - r * DP;
        const double2 v = *(const double2*)(c + ((int64_t)(f0 + f) * B + wrap_index(q0 + r, B)) * DP + j);
        *(double2*)(st + ((int64_t)f * lcap + r) * DP + j) = v;
    }
}

// One block = 512 consecutive STRIP points (foot-parameter order, two per
// thread; block pb) x fields [f0, f1).  The block's stencils cover the normals
// p0(first) - kl .. p0(last) - kl + M (p0 is monotone in theta); when that
// window has at most lcap normals, its Gram records are staged in LDS (st),
// fstage fields at a time, and every thread reads its records from there;
// otherwise the threads read the plan's record array c ([nf][B][DP]) directly.
// Every thread of the block calls this with the same arguments.
template <int M, int DT>
__device__ __forceinline__ void strip_block(const int32_t* __restrict__ sidx, const double* __restrict__ sth,
                                            const double* __restrict__ seta, int64_t S, const double* sAr, int D,
                                            int Cr, int B, double k2, double lev_scale, const double* __restrict__ c,
                                            double* __restrict__ out, int64_t npts, int pb, int f0, int f1, int lcap,
                                            int fstage, double* st) {
    const int64_t kfirst = (int64_t)pb * 512;
    const int64_t klast = min(S - 1, kfirst + 511);
    const int64_t ka = kfirst + 2 * threadIdx.x;   // two consecutive points per thread
    const bool live = ka < S;
    const int Dd = DT > 0 ? DT : D;
    const int DP = (Dd + 2) & ~1;
    constexpr int kl = (M - 1) / 2;
    StripPt<M> A, Bp;
    const bool hasb = ka + 1 < S;
    if (live) {
        strip_setup<M, DT>(sidx, sth, seta, ka, sAr, D, Cr, k2, lev_scale, A);
        strip_setup<M, DT>(sidx, sth, seta, hasb ? ka + 1 : ka, sAr, D, Cr, k2, lev_scale, Bp);
    }
    const int pfirst = strip_p0<M>(sth[kfirst], k2);
    const int L = strip_p0<M>(sth[klast], k2) - pfirst + M + 1;   // uniform over the block
    if (L <= lcap) {
        for (int fs = f0; fs < f1; fs += fstage) {
            const int nfs = min(fstage, f1 - fs);
            __syncthreads();   // the stage's previous contents have been read
            stage_records(c, B, DP, pfirst - kl, L, lcap, fs, nfs, st);
            __syncthreads();
            if (live)
                strip_pair_fields<M, DT, true>(A, Bp, hasb, D, B, st, (int64_t)lcap * DP, pfirst - kl, out, npts, fs,
                                               fs + nfs);
        }
    } else if (live) {
        strip_pair_fields<M, DT, false>(A, Bp, hasb, D, B, c + (int64_t)f0 * B * DP, (int64_t)B * DP, 0, out, npts,
                                        f0, f1);
    }
}

// LDS of the strip kernels: the blend table A_r, then the record stage
__device__ __forceinline__ double* strip_stage(double* smem, int Cr, int D) { return smem + ((Cr * D + 1) & ~1); }

template <int M, int DT>
__global__ __launch_bounds__(256) void k_strip(const int32_t* __restrict__ sidx, const double* __restrict__ sth,
                                               const double* __restrict__ seta, int64_t S, const double* __restrict__ Ar,
                                               int D, int Cr, int B, double k2, double lev_scale,
                                               const double* __restrict__ c, double* __restrict__ out, int64_t npts,
                                               int nf, int fpt, int lcap, int fstage) {
    extern __shared__ double smem[];
    double* sAr = smem;
    for (int k = threadIdx.x; k < Cr * D; k += blockDim.x) sAr[k] = Ar[k];
    __syncthreads();
    // blocks are dealt round-robin to the 8 XCDs: when the field chunks divide
    // evenly, each XCD gets a contiguous range of them, so its L2 holds only
    // those fields' Gram records
    const int pblocks = (int)((S + 511) / 512);   // 256 threads x 2 points
    const int nchunks = (nf + fpt - 1) / fpt;
    int chunk, pb;
    if (nchunks % 8 == 0) {
        const int local = blockIdx.x / 8;
        chunk = (blockIdx.x % 8) * (nchunks / 8) + local / pblocks;
        pb = local % pblocks;
    } else {
        chunk = blockIdx.x / pblocks;
        pb = blockIdx.x % pblocks;
    }
    const int f0 = chunk * fpt;
    strip_block<M, DT>(sidx, sth, seta, S, sAr, D, Cr, B, k2, lev_scale, c, out, npts, pb, f0, min(nf, f0 + fpt), lcap,
                       fstage, strip_stage(smem, Cr, D));
}

// Persistent form over several plans: work item w = (plan, block of 512 STRIP
// points, chunk of fpt fields).  All plans of a batch share the FC-Gram tables.
template <int M, int DT>
__global__ __launch_bounds__(256) void k_strip_multi(const PlanDev* __restrict__ pd, int np, int64_t total, int fpt,
                                                     const double* __restrict__ Ar, int D, int Cr, int lcap,
                                                     int fstage) {
    extern __shared__ double smem[];
    double* sAr = smem;
    for (int k = threadIdx.x; k < Cr * D; k += blockDim.x) sAr[k] = Ar[k];
    __syncthreads();
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        int kk = 0;
        while (kk + 1 < np && pd[kk + 1].off_strip <= w) ++kk;
        const PlanDev& P = pd[kk];
        const int64_t l = w - P.off_strip;
        const int64_t pblocks = (P.S + 511) / 512;
        const int pb = (int)(l % pblocks);
        const int f0 = (int)(l / pblocks) * fpt;
        strip_block<M, DT>(P.sidx, P.sth, P.seta, P.S, sAr, D, Cr, P.B, P.k2, P.lev_scale, P.c, P.u, P.npts, pb, f0,
                           min(P.nf, f0 + fpt), lcap, fstage, strip_stage(smem, Cr, D));
    }
}

// Boundary values for the next Fourier-Forwarding step: bval_one (lagrange_dev.h)
// at each boundary point.
template <int M>
__global__ void k_bvals(const double* __restrict__ bxy, int64_t nb, const double* __restrict__ u, int nx, int ny,
                        double x0, double y0, double h, int nf, double* __restrict__ fb) {
    const int64_t total = nb * nf;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int f = (int)(e / nb);
        const int64_t k = e - (int64_t)f * nb;
        fb[e] = bval_one<M>(u + (int64_t)f * nx * ny, nx, ny, x0, y0, h, bxy[2 * k], bxy[2 * k + 1]);
    }
}

template <int M>
__global__ void k_bvals_multi(const PlanDev* __restrict__ pd, int np, int64_t total) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        int kk = 0;
        while (kk + 1 < np && pd[kk + 1].off_bv <= e) ++kk;
        const PlanDev& P = pd[kk];
        const int64_t l = e - P.off_bv;
        const int f = (int)(l / P.nbdry);
        const int64_t k = l - (int64_t)f * P.nbdry;
        if (f >= P.nf) continue;
        P.fb[(int64_t)f * P.nbdry + k] =
            bval_one<M>(P.u + (int64_t)f * P.npts, P.nx, P.ny, P.x0, P.y0, P.h, P.bxy[2 * k], P.bxy[2 * k + 1]);
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
// ---------------------------------------------------------------------------
// Fixed scratch for fc2d_extend_fft_noalloc (callers that cannot allocate:
// code under graph capture, serving loops, harnesses that forbid allocation).
// One copy per device, held until the process ends; every such call on a
// device shares it, so calls that overlap on one device race.  In host code
// the array's name is not a device address: its address on the current device
// comes from hipGetSymbolAddress, looked up once per device and kept.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

static std::mutex g_scratch_mu;
static constexpr int kMaxDevices = 64;
static double* g_scratch_ptr[kMaxDevices];

int static_scratch(double** p, size_t* bytes) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
        return FC2D_E_HIP;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("fixed scratch: device index out of range");
        return FC2D_E_ARG;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* a = nullptr;
        e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !a) {
            set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return FC2D_E_HIP;
        }
        g_scratch_ptr[dev] = (double*)a;
    }
    *p = g_scratch_ptr[dev];
    *bytes = kScratchBytes;
    return FC2D_OK;
}

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
    // four normals x four fields per wave when there are enough fields to share
    const int npw = nf >= 4 ? 4 : 1;
    const int nq = (pl->B + npw - 1) / npw;
    dim3 grid(((nq + 7) / 8) * 8, (nf + 16 / npw - 1) / (16 / npw));
    switch (pl->M) {
#define FC2D_MATCH(MM) \
        case MM: \
            if (pl->d == 5 && npw == 4) k_match<MM, 5, 4><<<grid, 64, 0, s>>>(pl->d_mref, pl->d_mlab, pl->d_mwv, pl->d_mwn, pl->d_Q, pl->d, pl->B, pl->interior_only ? 1 : 0, f_grid, npts, f_bdry, nbdry, nf, c_out, fD_out); \
            else if (pl->d == 5) k_match<MM, 5, 1><<<grid, 64, 0, s>>>(pl->d_mref, pl->d_mlab, pl->d_mwv, pl->d_mwn, pl->d_Q, pl->d, pl->B, pl->interior_only ? 1 : 0, f_grid, npts, f_bdry, nbdry, nf, c_out, fD_out); \
            else if (npw == 4) k_match<MM, 0, 4><<<grid, 64, 0, s>>>(pl->d_mref, pl->d_mlab, pl->d_mwv, pl->d_mwn, pl->d_Q, pl->d, pl->B, pl->interior_only ? 1 : 0, f_grid, npts, f_bdry, nbdry, nf, c_out, fD_out); \
            else k_match<MM, 0, 1><<<grid, 64, 0, s>>>(pl->d_mref, pl->d_mlab, pl->d_mwv, pl->d_mwn, pl->d_Q, pl->d, pl->B, pl->interior_only ? 1 : 0, f_grid, npts, f_bdry, nbdry, nf, c_out, fD_out); \
            break;
        FC2D_MATCH(4) FC2D_MATCH(5) FC2D_MATCH(6) FC2D_MATCH(7) FC2D_MATCH(8) FC2D_MATCH(13) FC2D_MATCH(15)
#undef FC2D_MATCH
        default: set_error("unsupported M"); return FC2D_E_ARG;
    }
    return launch_check("k_match", s);
}

int launch_blend(const fc2d_plan* pl, const double* c, double* F, int nf,
                 hipStream_t s) {
    const int64_t n = (int64_t)(pl->Cr + 1) * pl->B;
    dim3 grid((unsigned)std::min<int64_t>((n + 255) / 256, 4096), nf);
    k_blend<<<grid, 256, 0, s>>>(c, pl->d_Ar, pl->d, pl->B, pl->Cr, F);
    return launch_check("k_blend", s);
}

// LDS of the strip kernels: the blend table, then the staged Gram records (a
// block's window of at most lcap normals, at most 16 KB per field and 32 KB
// per stage of fstage fields)
static int g_strip_wcap = 0;   // cap on the staged window (normals), 0 = none; set through the tuning interface
int strip_wcap_get() { return g_strip_wcap; }
int strip_wcap_set(int v) {
    if (v < 0) return FC2D_E_ARG;
    g_strip_wcap = v;
    return FC2D_OK;
}

size_t strip_lds(int wmax, int d, int Cr, int fpt, int* lcap, int* fstage) {
    const size_t rec_bytes = (size_t)((d + 2) & ~1) * sizeof(double);
    if (g_strip_wcap > 0) wmax = std::min(wmax, g_strip_wcap);
    *lcap = (int)std::max<size_t>(1, std::min<size_t>((size_t)wmax, 16384 / rec_bytes));
    *fstage = (int)std::max<size_t>(1, std::min<size_t>((size_t)std::min(fpt, 8), 32768 / (*lcap * rec_bytes)));
    return (size_t)((Cr * d + 1) & ~1) * sizeof(double) + (size_t)*fstage * *lcap * rec_bytes;
}

int launch_strip(const fc2d_plan* pl, const double* c, const double* f_bdry, int64_t nbdry, double* out, int nf,
                 hipStream_t s) {
    const int64_t S = pl->n_strip;
    if (S == 0) return FC2D_OK;
    const int64_t npts = (int64_t)pl->grid.nx * pl->grid.ny;
    // fields per thread: at most 8, the chunks a multiple of 8 (an equal range
    // per XCD) when there are at least 8 fields; two points per thread
    const int64_t pblocks = (S + 511) / 512;
    int fpt = g_strip_fpt;
    if (fpt <= 0) fpt = nf >= 8 ? (nf + 8 * ((nf + 63) / 64) - 1) / (8 * ((nf + 63) / 64)) : 1;
    fpt = std::max(1, std::min(fpt, nf));
    const int64_t nchunks = (nf + fpt - 1) / fpt;
    const dim3 grid((unsigned)(nchunks * pblocks));
    int lcap, fstage;
    const size_t lds = strip_lds(pl->strip_wmax, pl->d, pl->Cr, fpt, &lcap, &fstage);
    const double lev_scale = pl->n_r / pl->k1;
    switch (pl->M) {
#define FC2D_STRIP(MM) \
        case MM: \
            if (pl->d == 5) k_strip<MM, 5><<<grid, 256, lds, s>>>(pl->d_sidx, pl->d_sth, pl->d_seta, S, pl->d_Ar, pl->d, pl->Cr, pl->B, pl->k2, lev_scale, c, out, npts, nf, fpt, lcap, fstage); \
            else k_strip<MM, 0><<<grid, 256, lds, s>>>(pl->d_sidx, pl->d_sth, pl->d_seta, S, pl->d_Ar, pl->d, pl->Cr, pl->B, pl->k2, lev_scale, c, out, npts, nf, fpt, lcap, fstage); \
            break;
        FC2D_STRIP(4) FC2D_STRIP(5) FC2D_STRIP(6) FC2D_STRIP(7) FC2D_STRIP(8) FC2D_STRIP(13) FC2D_STRIP(15)
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

namespace fc2d {

int launch_bvals(const fc2d_plan* pl, const double* u, double* fb, int nf, hipStream_t s) {
    const int64_t nb = pl->B + (int64_t)pl->squares.size() / 2;
    const int64_t total = nb * nf;
    const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 65535);
    const fc2d_grid& g = pl->grid;
    switch (pl->M) {
#define FC2D_BV(MM) \
        case MM: k_bvals<MM><<<blocks, 256, 0, s>>>(pl->d_bxy, nb, u, g.nx, g.ny, g.x0, g.y0, g.h, nf, fb); break;
        FC2D_BV(4) FC2D_BV(5) FC2D_BV(6) FC2D_BV(7) FC2D_BV(8) FC2D_BV(13) FC2D_BV(15)
#undef FC2D_BV
        default: set_error("unsupported M"); return FC2D_E_ARG;
    }
    return launch_check("k_bvals", s);
}

int launch_multi(int which, int M, const PlanDev* d_pd, int np, int64_t total, int fpt, const double* Ar, int D,
                 int Cr, int wmax, int grid_blocks, hipStream_t s) {
    // the matching kernel's blocks are single waves: twice the blocks fill the
    // 16 waves per CU its registers allow (the others have four waves per block)
    const int64_t cap = which == 0 ? 2 * (int64_t)grid_blocks : (int64_t)grid_blocks;
    const unsigned g = (unsigned)std::max<int64_t>(8, std::min<int64_t>(total, cap));
    int lcap = 1, fstage = 1;
    const size_t lds = which == 1 ? strip_lds(wmax, D, Cr, fpt, &lcap, &fstage) : 0;
    switch (M) {
#define FC2D_MULTI(MM)                                                                                 \
        case MM:                                                                                       \
            if (which == 0 && D == 5) k_match_multi<MM, 5><<<g, 64, 0, s>>>(d_pd, np, total);          \
            else if (which == 0) k_match_multi<MM, 0><<<g, 64, 0, s>>>(d_pd, np, total);               \
            else if (which == 1 && D == 5) k_strip_multi<MM, 5><<<g, 256, lds, s>>>(d_pd, np, total, fpt, Ar, D, Cr, lcap, fstage); \
            else if (which == 1) k_strip_multi<MM, 0><<<g, 256, lds, s>>>(d_pd, np, total, fpt, Ar, D, Cr, lcap, fstage); \
            else k_bvals_multi<MM><<<g, 256, 0, s>>>(d_pd, np, total);                                 \
            break;
        FC2D_MULTI(4) FC2D_MULTI(5) FC2D_MULTI(6) FC2D_MULTI(7) FC2D_MULTI(8) FC2D_MULTI(13) FC2D_MULTI(15)
#undef FC2D_MULTI
        default: set_error("unsupported M"); return FC2D_E_ARG;
    }
    return launch_check(which == 0 ? "k_match_multi" : (which == 1 ? "k_strip_multi" : "k_bvals_multi"), s);
}

}  // namespace fc2d
