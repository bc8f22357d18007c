// Learned seed for the foot-of-normal solve (FC2D_SEED_MLP): the network, its
// training (forward, backward, Adam) and its use in the classification.
//
// Network: 8 rotation-invariant inputs of a point near a polar curve (its
// radial offset and r, r', ..., r^(5) at its polar angle), three hidden layers
// of 64 tanh units, 2 linear outputs, FP32.  Weights are read by wave-uniform
// addresses, so they come through the scalar unit and are shared by the wave.
//
// Layout inside a workgroup: one wave (64 lanes), lane = sample.  Activations
// live in LDS as [feature][65] columns (a lane reading its own sample, or a
// lane reading one feature across samples, hits 64 different banks) and the
// back-propagated deltas as [sample][68] rows (read four at a time, the same
// address for every lane, when forming weight gradients).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"
#include "seed_dev.h"

namespace fc2d {
namespace {

constexpr int kNin = FC2D_MLP_NIN;
constexpr int kH = FC2D_MLP_HIDDEN;
constexpr int kOffW0 = 0;
constexpr int kOffB0 = kOffW0 + kNin * kH;
constexpr int kOffW1 = kOffB0 + kH;
constexpr int kOffB1 = kOffW1 + kH * kH;
constexpr int kOffW2 = kOffB1 + kH;
constexpr int kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH;
constexpr int kOffB3 = kOffW3 + kH * 2;
constexpr int kNW = kOffB3 + 2;
static_assert(kNW == FC2D_MLP_NW, "weight count");
constexpr int kNWP = kNW + 2;          // per-workgroup partial record: gradient, loss, pad (multiple of 4)
constexpr int kSP = 65;                // activation column stride
constexpr int kDR = 68;                // delta row stride (16-byte aligned rows)
constexpr double kTargetScale = 100.0;

// features of (X, Y) near the polar curve a (n modes) for strip width w; phi
// and the first-order estimates (delta / w, eta / w) are returned alongside
__device__ inline void mlp_features(const double* a, int n, double X, double Y, double w, float* f, double* phi,
                                    double* base0, double* base1) {
    const double ph = atan2(Y, X);
    const double rho = sqrt(X * X + Y * Y);
    double R[6];
    polar_derivs(a, n, ph, R);
    const double f0 = (rho - R[0]) / w;
    const double f2 = R[1] / R[0];
    const double f7 = f0 * f2 / (1.0 + f2 * f2);
    f[0] = (float)f0;
    f[1] = (float)(R[0] - 1.0);
    f[2] = (float)f2;
    f[3] = (float)(R[2] / (R[0] * 2.0));
    f[4] = (float)(R[3] / (R[0] * 10.0));
    f[5] = (float)(R[4] / (R[0] * 60.0));
    f[6] = (float)(R[5] / (R[0] * 400.0));
    f[7] = (float)f7;
    *phi = ph;
    *base0 = f7 / R[0];
    *base1 = f0 / sqrt(1.0 + f2 * f2);
}

// hidden layer on one lane's column col[i * stride] (in place): tanh(b + x W)
template <int FI, int STRIDE>
__device__ inline void hidden_layer(const float* __restrict__ W, const float* __restrict__ b, const float* in,
                                    float* out) {
    float z[kH];
#pragma unroll
    for (int o = 0; o < kH; ++o) z[o] = b[o];
#pragma unroll 2
    for (int i = 0; i < FI; ++i) {
        const float x = in[i * STRIDE];
#pragma unroll
        for (int o = 0; o < kH; ++o) z[o] = fmaf(x, W[i * kH + o], z[o]);
    }
#pragma unroll
    for (int o = 0; o < kH; ++o) out[o * STRIDE] = tanhf(z[o]);
}

template <int STRIDE>
__device__ inline void output_layer(const float* __restrict__ w, const float* in, float* out) {
    float o0 = w[kOffB3], o1 = w[kOffB3 + 1];
#pragma unroll 4
    for (int i = 0; i < kH; ++i) {
        const float x = in[i * STRIDE];
        o0 = fmaf(x, w[kOffW3 + 2 * i], o0);
        o1 = fmaf(x, w[kOffW3 + 2 * i + 1], o1);
    }
    out[0] = o0;
    out[1] = o1;
}

// ---- inference on the matrix cores: FP32 MFMA 32x32x2 -------------------
// One wave evaluates 64 points: each layer is [64 points x K] x [K x 64] as
// 2 x 2 output tiles of 32 x 32, K/2 MFMA steps each.  Operand lanes (checked
// on the device): A lane l holds row l % 32, k = l / 32; B lane l holds k =
// l / 32, column l % 32; D lane l, element r holds row 8 (r / 4) + 4 (l / 32)
// + r % 4, column l % 32.  Activations pass between layers through per-wave
// LDS rows of stride kHS (odd, so both access patterns are conflict-free).
typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int kHS = 65;

template <int K>
__device__ inline void mfma_layer(const float* __restrict__ W, const float* __restrict__ b, float* Hs, int lane) {
    const int r32 = lane & 31, hi = lane >> 5;
    float a[2][K / 2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int ks = 0; ks < K / 2; ++ks) a[mt][ks] = Hs[(r32 + 32 * mt) * kHS + 2 * ks + hi];
    f32x16 acc[2][2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[mt][nt][r] = 0.0f;
#pragma unroll
    for (int ks = 0; ks < K / 2; ++ks) {
        const float b0 = W[(2 * ks + hi) * kH + r32];
        const float b1 = W[(2 * ks + hi) * kH + 32 + r32];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            acc[mt][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[mt][ks], b0, acc[mt][0], 0, 0, 0);
            acc[mt][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[mt][ks], b1, acc[mt][1], 0, 0, 0);
        }
    }
    // every input of this wave has been read (above, into registers): overwrite in place
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        const float bias = b[r32 + 32 * nt];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                Hs[(8 * (r / 4) + 4 * hi + (r & 3) + 32 * mt) * kHS + r32 + 32 * nt] = tanhf(acc[mt][nt][r] + bias);
    }
}

// Network outputs for the wave's 64 points; row `lane` of Hs holds this lane's
// 8 inputs on entry (all 64 lanes take part).
__device__ inline void forward_wave(const float* __restrict__ w, float* Hs, int lane, float* out) {
    mfma_layer<kNin>(w + kOffW0, w + kOffB0, Hs, lane);
    mfma_layer<kH>(w + kOffW1, w + kOffB1, Hs, lane);
    mfma_layer<kH>(w + kOffW2, w + kOffB2, Hs, lane);
    output_layer<1>(w, Hs + lane * kHS, out);
}

// forward pass of one lane; x0 = its inputs (stride STRIDE), a1..a3 its
// activation columns (stride STRIDE, may alias each other for inference)
template <int STRIDE>
__device__ inline void forward_lane(const float* __restrict__ w, const float* x0, float* a1, float* a2, float* a3,
                                    float* out) {
    hidden_layer<kNin, STRIDE>(w + kOffW0, w + kOffB0, x0, a1);
    hidden_layer<kH, STRIDE>(w + kOffW1, w + kOffB1, a1, a2);
    hidden_layer<kH, STRIDE>(w + kOffW2, w + kOffB2, a2, a3);
    output_layer<STRIDE>(w, a3, out);
}

}  // namespace

// ---------------------------------------------------------------------------
// classification with the learned seed: one lane per candidate point
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_seed_mlp(SeedArgs a, const float* __restrict__ w,
                                                 const int32_t* __restrict__ cand, int64_t ncand, int8_t* cls,
                                                 StripRec* rec, int64_t cap, int* counters) {
    __shared__ float Hs[64 * kHS];   // the wave's activation rows
    const int lane = threadIdx.x;
    const int64_t k = (int64_t)blockIdx.x * 64 + lane;
    const bool live = k < ncand;     // every lane takes part in the matrix products
    const int64_t idx = cand[live ? k : ncand - 1];
    const int i = (int)(idx / a.ny);
    const int j = (int)(idx - (int64_t)i * a.ny);
    const double X = a.x0 + i * a.h;
    const double Y = a.y0 + j * a.h;
    float f[kNin];
    double phi, b0, b1;
    mlp_features(a.curve.a, a.curve.nmodes, X, Y, a.width, f, &phi, &b0, &b1);
#pragma unroll
    for (int q = 0; q < kNin; ++q) Hs[lane * kHS + q] = f[q];
    float out[2];
    forward_wave(w, Hs, lane, out);
    if (!live) return;
    double th = phi + a.width * (b0 + (double)out[0] / kTargetScale);
    // two plain Newton steps, then the residual |g / g'|
    double o[6], dx = 0.0, dy = 0.0, g = 0.0, gp = 0.0;
    for (int s = 0; s < 3; ++s) {
        curve_eval(a.curve, th, o);
        dx = o[0] - X;
        dy = o[1] - Y;
        g = dx * o[2] + dy * o[3];
        gp = o[2] * o[2] + o[3] * o[3] + dx * o[4] + dy * o[5];
        if (s < 2) th -= g / gp;
    }
    const double res = fabs(g / gp);
    double theta = 0.0, eta = 0.0;
    int st = FOOT_OK, it = 3;
    if (res <= a.mlp_tol && gp > 0.0 && dx * dx + dy * dy <= a.dist2_max) {
        foot_finish(a.curve, X, Y, th - g / gp, &theta, &eta);
    } else {   // NaN seeds land here too
        atomicAdd(&counters[4], 1);
        int it2 = 0;
        st = foot_from_seed(a.curve, X, Y, phi, 2.0 * a.k2, a.maxit, &theta, &eta, &it2);
        it += it2;
    }
    store_solved(idx, X, Y, st, theta, eta, it, nearest_sample(theta, a.k2, a.B), a.width, cls, rec, cap, counters);
}

int launch_seed_mlp(const SeedArgs& a, const float* d_w, const int32_t* d_cand, int64_t ncand, int8_t* d_cls,
                    StripRec* d_rec, int64_t cap, int* d_counters, hipStream_t s) {
    if (ncand <= 0) return FC2D_OK;
    k_seed_mlp<<<(unsigned)((ncand + 63) / 64), 64, 0, s>>>(a, d_w, d_cand, ncand, d_cls, d_rec, cap, d_counters);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("MLP seed launch: ") + hipGetErrorString(e));
        return FC2D_E_HIP;
    }
    trace_point("k_seed_mlp", s);
    return FC2D_OK;
}

// ---------------------------------------------------------------------------
// training data, inference, training
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_data(const double* __restrict__ curves, int ncurves, int ncoef,
                                                  int nmodes, const int32_t* __restrict__ cidx,
                                                  const double* __restrict__ ths, const double* __restrict__ etas,
                                                  int64_t n, double w, int maxit, float* X, float* Y, double* foot,
                                                  int32_t* iters) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int c = cidx[k];
    if (c < 0 || c >= ncurves) {   // not a curve of the set: flagged, outputs untouched
        if (iters) iters[k] = -1;
        return;
    }
    const PolarRef cv{curves + (int64_t)c * ncoef, nmodes};
    double o[6];
    curve_eval(cv, ths[k], o);
    const double sp = sqrt(o[2] * o[2] + o[3] * o[3]);
    const double e = etas[k];
    const double Qx = o[0] + e * (o[3] / sp);
    const double Qy = o[1] + e * (-o[2] / sp);
    float f[kNin];
    double phi, b0, b1;
    mlp_features(cv.a, nmodes, Qx, Qy, w, f, &phi, &b0, &b1);
    double th = 0.0, eta = 0.0;
    int it = 0;
    const int st = foot_from_seed(cv, Qx, Qy, phi, 0x1p-10, maxit, &th, &eta, &it);
    double d = th - phi;
    d -= kTwoPi * rint(d / kTwoPi);
#pragma unroll
    for (int q = 0; q < kNin; ++q) X[k * kNin + q] = f[q];
    Y[2 * k] = (float)(kTargetScale * (d / w - b0));
    Y[2 * k + 1] = (float)(kTargetScale * (eta / w - b1));
    if (foot) {
        foot[2 * k] = th;
        foot[2 * k + 1] = eta;
    }
    if (iters) iters[k] = st == FOOT_OK ? it : -1;
}

__global__ __launch_bounds__(64) void k_mlp_forward(const float* __restrict__ w, const float* __restrict__ X,
                                                    int64_t n, float* out) {
    __shared__ float Hs[64 * kHS];
    const int lane = threadIdx.x;
    const int64_t k = (int64_t)blockIdx.x * 64 + lane;
    const int64_t kk = k < n ? k : n - 1;   // every lane takes part in the matrix products
#pragma unroll
    for (int q = 0; q < kNin; ++q) Hs[lane * kHS + q] = X[kk * kNin + q];
    float r[2];
    forward_wave(w, Hs, lane, r);
    if (k >= n) return;
    out[2 * k] = r[0];
    out[2 * k + 1] = r[1];
}

// sample at position q of the training sequence: pass e = q / n visits sample
// (A (q mod n) + hash(e)) mod n, a permutation of 0..n-1 for A coprime to n
__device__ inline int64_t sample_at(int64_t q, int64_t n, int64_t A) {
    const int64_t e = q / n;
    const int64_t r = q - e * n;
    const int64_t off = (int64_t)(((uint64_t)e * 0x9E3779B97F4A7C15ull) % (uint64_t)n);
    return (A * r + off) % n;
}

// weight gradient of one layer: lanes < FI own input feature i; acc[o] =
// sum_s act[i][s] delta[s][o]; bias gradient: lane o sums delta[s][o]
template <int FI, int FO>
__device__ inline void layer_grads(const float* act, const float* D, float* part, int offW, int offB, int lane) {
    if (lane < FI) {
        float acc[FO];
#pragma unroll
        for (int o = 0; o < FO; ++o) acc[o] = 0.0f;
        for (int s = 0; s < 64; ++s) {
            const float x = act[lane * kSP + s];
            if constexpr (FO % 4 == 0) {
                const float4* dr = reinterpret_cast<const float4*>(D + s * kDR);
#pragma unroll
                for (int q = 0; q < FO / 4; ++q) {
                    const float4 d = dr[q];
                    acc[4 * q] = fmaf(x, d.x, acc[4 * q]);
                    acc[4 * q + 1] = fmaf(x, d.y, acc[4 * q + 1]);
                    acc[4 * q + 2] = fmaf(x, d.z, acc[4 * q + 2]);
                    acc[4 * q + 3] = fmaf(x, d.w, acc[4 * q + 3]);
                }
            } else {
#pragma unroll
                for (int o = 0; o < FO; ++o) acc[o] = fmaf(x, D[s * kDR + o], acc[o]);
            }
        }
#pragma unroll
        for (int o = 0; o < FO; ++o) part[offW + lane * FO + o] = acc[o];
    }
    if (lane < FO) {
        float sb = 0.0f;
        for (int s = 0; s < 64; ++s) sb += D[s * kDR + lane];
        part[offB + lane] = sb;
    }
}

// delta of the layer below (lane = sample): d_prev[i] = (sum_o d[o] W[i][o]) (1 - a_i^2),
// a = the tanh output feeding this layer; overwrites this lane's delta row
template <int FO>
__device__ inline void back_delta(const float* __restrict__ W, const float* act, float* D, int lane) {
    float d[FO];
#pragma unroll
    for (int o = 0; o < FO; ++o) d[o] = D[lane * kDR + o];
    __syncthreads();   // every lane has read the rows the weight gradients used
    for (int i = 0; i < kH; ++i) {
        float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
        for (int o = 0; o < FO; o += 2) {
            s0 = fmaf(d[o], W[i * FO + o], s0);
            if (o + 1 < FO) s1 = fmaf(d[o + 1], W[i * FO + o + 1], s1);
        }
        const float a = act[i * kSP + lane];
        D[lane * kDR + i] = (s0 + s1) * (1.0f - a * a);
    }
    __syncthreads();
}

// One workgroup = 64 consecutive positions pos0 + 64 g + lane of the sample
// sequence (only the first nb positions count).  Writes its partial gradient of
// the mean loss over nb samples and its partial sum of 0.5 |r|^2.
__global__ __launch_bounds__(64) void k_mlp_grad(const float* __restrict__ w, const float* __restrict__ X,
                                                 const float* __restrict__ Yt, int64_t n, int64_t nb, int64_t pos0,
                                                 int64_t A, float* __restrict__ part_all) {
    __shared__ float sX[kNin * kSP];
    __shared__ float sA1[kH * kSP];
    __shared__ float sA2[kH * kSP];
    __shared__ float sA3[kH * kSP];
    __shared__ __align__(16) float sD[64 * kDR];
    const int lane = threadIdx.x;
    const int64_t jpos = (int64_t)blockIdx.x * 64 + lane;
    const bool valid = jpos < nb;
    float x[kNin], y0 = 0.0f, y1 = 0.0f;
    if (valid) {
        const int64_t idx = sample_at(pos0 + jpos, n, A);
#pragma unroll
        for (int q = 0; q < kNin; ++q) x[q] = X[idx * kNin + q];
        y0 = Yt[2 * idx];
        y1 = Yt[2 * idx + 1];
    } else {
#pragma unroll
        for (int q = 0; q < kNin; ++q) x[q] = 0.0f;
    }
#pragma unroll
    for (int q = 0; q < kNin; ++q) sX[q * kSP + lane] = x[q];
    float out[2];
    forward_lane<kSP>(w, sX + lane, sA1 + lane, sA2 + lane, sA3 + lane, out);
    const float inv = 1.0f / (float)nb;
    const float r0 = valid ? out[0] - y0 : 0.0f;
    const float r1 = valid ? out[1] - y1 : 0.0f;
    float lp = 0.5f * (r0 * r0 + r1 * r1);
    sD[lane * kDR] = r0 * inv;
    sD[lane * kDR + 1] = r1 * inv;
    __syncthreads();
    float* part = part_all + (int64_t)blockIdx.x * kNWP;
    layer_grads<kH, 2>(sA3, sD, part, kOffW3, kOffB3, lane);
    back_delta<2>(w + kOffW3, sA3, sD, lane);
    layer_grads<kH, kH>(sA2, sD, part, kOffW2, kOffB2, lane);
    back_delta<kH>(w + kOffW2, sA2, sD, lane);
    layer_grads<kH, kH>(sA1, sD, part, kOffW1, kOffB1, lane);
    back_delta<kH>(w + kOffW1, sA1, sD, lane);
    layer_grads<kNin, kH>(sX, sD, part, kOffW0, kOffB0, lane);
    // loss partial: sum over the wave
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) lp += __shfl_xor(lp, m, 64);
    if (lane == 0) part[kNW] = lp;
}

struct AdamArgs {
    int apply;
    float lr, b1, b2, eps, c1, c2;   // c1 = 1 - b1^t, c2 = 1 - b2^t
};

// Sums the G partial records in order; writes the gradient and/or applies Adam;
// the thread past the last weight writes the mean loss over nb samples.
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ part, int G, int64_t nb,
                                                    float* grad, float* w, float* m, float* v, AdamArgs ad,
                                                    float* loss) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > kNW) return;
    float s = 0.0f;
    for (int q = 0; q < G; ++q) s += part[(int64_t)q * kNWP + k];
    if (k == kNW) {
        if (loss) *loss = s / (float)nb;
        return;
    }
    if (grad) grad[k] = s;
    if (ad.apply) {
        const float mk = ad.b1 * m[k] + (1.0f - ad.b1) * s;
        const float vk = ad.b2 * v[k] + (1.0f - ad.b2) * s * s;
        m[k] = mk;
        v[k] = vk;
        w[k] -= ad.lr * (mk / ad.c1) / (sqrtf(vk / ad.c2) + ad.eps);
    }
}

}  // namespace fc2d

using namespace fc2d;

namespace {

int kernel_status(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string(what) + ": " + hipGetErrorString(e));
        return FC2D_E_HIP;
    }
    return FC2D_OK;
}

// multiplier of the sample order: a prime coprime to n
int64_t order_multiplier(int64_t n) {
    const int64_t primes[] = {1000000007LL, 998244353LL, 1000000009LL, 754974721LL};
    for (int64_t p : primes)
        if (n % p != 0) return p % n == 0 ? 1 : p;
    return 1;
}

}  // namespace

extern "C" {

int fc2d_mlp_make_data(const double* curves, int ncurves, int nmodes, const int32_t* cidx, const double* theta,
                       const double* eta, int64_t n, double width, float* X, float* Y, double* foot,
                       int32_t* iters, hipStream_t stream) {
    if (n < 0 || ncurves <= 0 || nmodes < 0 || nmodes > kMaxModes || !(width > 0.0)) {
        set_error("fc2d_mlp_make_data: invalid sizes");
        return FC2D_E_ARG;
    }
    if (n == 0) return FC2D_OK;
    if (!curves || !cidx || !theta || !eta || !X || !Y) {
        set_error("fc2d_mlp_make_data: NULL argument");
        return FC2D_E_ARG;
    }
    k_mlp_data<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(curves, ncurves, 1 + 2 * nmodes, nmodes, cidx, theta, eta, n,
                                                                 width, 60, X, Y, foot, iters);
    return kernel_status("fc2d_mlp_make_data launch");
}

int fc2d_mlp_forward(const float* weights, const float* X, int64_t n, float* out, hipStream_t stream) {
    if (n < 0) { set_error("fc2d_mlp_forward: negative n"); return FC2D_E_ARG; }
    if (n == 0) return FC2D_OK;
    if (!weights || !X || !out) { set_error("fc2d_mlp_forward: NULL argument"); return FC2D_E_ARG; }
    k_mlp_forward<<<(unsigned)((n + 63) / 64), 64, 0, stream>>>(weights, X, n, out);
    return kernel_status("fc2d_mlp_forward launch");
}

static int grad_steps(const float* weights, float* m, float* v, const float* X, const float* Y, int64_t n,
                      int64_t batch, int steps, int64_t t0, float lr0, float lr_min, int64_t t_total, float* grad,
                      float* loss, hipStream_t stream) {
    const int G = (int)((batch + 63) / 64);
    float* part = nullptr;
    if (hipMalloc((void**)&part, (size_t)G * kNWP * sizeof(float)) != hipSuccess) {
        set_error("hipMalloc failed (MLP partial gradients)");
        return FC2D_E_NOMEM;
    }
    const int64_t A = grad ? 1 : order_multiplier(n);
    int st = FC2D_OK;
    for (int s = 0; s < steps && st == FC2D_OK; ++s) {
        const int64_t t = t0 + s + 1;
        k_mlp_grad<<<G, 64, 0, stream>>>(weights, X, Y, n, batch, (t - 1) * batch, A, part);
        if ((st = kernel_status("MLP gradient launch"))) break;
        AdamArgs ad{};
        if (m) {
            const double tc = (double)std::min<int64_t>(t, t_total > 0 ? t_total : t);
            const double frac = t_total > 0 ? tc / (double)t_total : 0.0;
            ad.apply = 1;
            ad.lr = (float)(lr_min + (lr0 - lr_min) * 0.5 * (1.0 + cos(M_PI * frac)));
            ad.b1 = 0.9f;
            ad.b2 = 0.999f;
            ad.eps = 1e-8f;
            ad.c1 = (float)(1.0 - pow(0.9, (double)t));
            ad.c2 = (float)(1.0 - pow(0.999, (double)t));
        }
        k_mlp_reduce<<<(kNW + 1 + 255) / 256, 256, 0, stream>>>(part, G, batch, grad, const_cast<float*>(weights), m,
                                                                v, ad, loss ? loss + (m ? s : 0) : nullptr);
        st = kernel_status("MLP reduce launch");
    }
    hipError_t e = hipStreamSynchronize(stream);
    (void)hipFree(part);
    if (st == FC2D_OK && e != hipSuccess) {
        set_error(std::string("MLP training: ") + hipGetErrorString(e));
        st = FC2D_E_HIP;
    }
    return st;
}

int fc2d_mlp_loss_grad(const float* weights, const float* X, const float* Y, int64_t n, float* grad, float* loss,
                       hipStream_t stream) {
    if (n <= 0 || n >= ((int64_t)1 << 31)) { set_error("fc2d_mlp_loss_grad: n out of range"); return FC2D_E_ARG; }
    if (!weights || !X || !Y) { set_error("fc2d_mlp_loss_grad: NULL argument"); return FC2D_E_ARG; }
    return grad_steps(weights, nullptr, nullptr, X, Y, n, n, 1, 0, 0.0f, 0.0f, 0, grad, loss, stream);
}

int fc2d_mlp_train(float* weights, float* adam_m, float* adam_v, const float* X, const float* Y, int64_t n, int batch,
                   int steps, int64_t t0, float lr0, float lr_min, int64_t t_total, float* loss_hist,
                   hipStream_t stream) {
    if (n <= 0 || n >= ((int64_t)1 << 31) || batch <= 0 || batch > (1 << 22) || steps < 0 || t0 < 0 ||
        !(lr0 >= 0.0f) || !(lr_min >= 0.0f)) {
        set_error("fc2d_mlp_train: invalid sizes");
        return FC2D_E_ARG;
    }
    if (!weights || !adam_m || !adam_v || !X || !Y) { set_error("fc2d_mlp_train: NULL argument"); return FC2D_E_ARG; }
    if (steps == 0) return FC2D_OK;
    return grad_steps(weights, adam_m, adam_v, X, Y, n, batch, steps, t0, lr0, lr_min, t_total, nullptr, loss_hist,
                      stream);
}

}  // extern "C"
