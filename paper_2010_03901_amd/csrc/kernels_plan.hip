// Device part of the Geometrical Setup (Sec. 3.5 steps 3-4): classification of
// the Cartesian grid H and the foot of the normal of every point near Gamma.
//
//  k_near_scatter: proximity of Sec. 3.3 reduced to its normal index -- every
//    boundary sample q_p scatters (distance^2, p) into the grid points within
//    r_out of it with a 64-bit atomicMin, so each point near Gamma learns its
//    nearest sample p (ties to the smaller p).
//  k_classify: one thread per grid point.  Parity of the crossings of its grid
//    column with the boundary polygon gives IN / FAR; points near Gamma (outside
//    within r_out, inside within r_in of their nearest sample) solve for the
//    foot (theta^Q, eta_Q) from the seed p and are reclassified by eta:
//    IN (eta <= 0), STRIP (0 < eta <= C k1), FAR.  STRIP points append a record.
//  k_radial_band / k_seed_polar (polar curves): rho - r(phi) decides IN / FAR
//    away from Gamma and selects the candidates near it, which are compacted
//    into a list and solved from the seed phi = atan2(y, x), one thread each.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "seed_dev.h"

namespace fc2d {

__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_near_scatter(ClassifyArgs a, uint64_t* near) {
    const int p = blockIdx.x;
    const double qx = a.bx[p], qy = a.by[p];
    const double r2 = a.r_out * a.r_out;
    int i0 = (int)floor((qx - a.r_out - a.x0) / a.h);
    int i1 = (int)ceil((qx + a.r_out - a.x0) / a.h);
    int j0 = (int)floor((qy - a.r_out - a.y0) / a.h);
    int j1 = (int)ceil((qy + a.r_out - a.y0) / a.h);
    i0 = max(i0, 0);
    j0 = max(j0, 0);
    i1 = min(i1, a.nx - 1);
    j1 = min(j1, a.ny - 1);
    if (i1 < i0 || j1 < j0) return;
    const int wj = j1 - j0 + 1;
    const int n = (i1 - i0 + 1) * wj;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const int i = i0 + k / wj;
        const int j = j0 + k % wj;
        const double dx = (a.x0 + i * a.h) - qx;
        const double dy = (a.y0 + j * a.h) - qy;
        const double d2 = dx * dx + dy * dy;
        if (d2 <= r2) {
            const uint64_t key = ((uint64_t)__float_as_uint((float)d2) << 32) | (uint32_t)p;
            atomicMin((unsigned long long*)&near[(int64_t)i * a.ny + j], (unsigned long long)key);
        }
    }
}

template <int M>
__global__ __launch_bounds__(256) void k_classify(ClassifyArgs a, const uint64_t* near, int8_t* cls,
                                                  StripRec* rec, int64_t cap, int* counters) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)a.nx * a.ny) return;
    const int i = (int)(idx / a.ny);
    const int j = (int)(idx - (int64_t)i * a.ny);
    const double X = a.x0 + i * a.h;
    const double Y = a.y0 + j * a.h;
    // crossing parity along the column x = x_i (crossings strictly below y_j)
    int below = 0;
    for (int k = a.col_ptr[i]; k < a.col_ptr[i + 1]; ++k) below += (a.col_y[k] < Y) ? 1 : 0;
    const bool inside = (below & 1) != 0;
    int8_t c = inside ? 1 : 0;
    const uint64_t key = near[idx];
    if (key != ~0ull) {
        const float d2 = __uint_as_float((uint32_t)(key >> 32));
        const int p = (int)(key & 0xffffffffu);
        const bool band = inside ? ((double)d2 <= a.r_in * a.r_in) : true;
        if (band) {
            BndView bd{a.bx, a.by, a.bnx, a.bny, a.B, a.k2};
            double th = 0.0, eta = 0.0;
            int it = 0;
            const int stt = foot_solve<M>(a.curve, bd, X, Y, p, a.maxit, &th, &eta, &it);
            atomicAdd(&counters[3], 1);
            store_solved(idx, X, Y, stt, th, eta, it, p, a.width, cls, rec, cap, counters);
            return;
        }
    }
    cls[idx] = c;
}

// r(phi) of a polar curve at the point (X, Y) = rho (cos phi, sin phi), with
// cos m phi, sin m phi by the angle-addition recurrence from X / rho, Y / rho
__device__ inline double polar_radius_at(const CurveC& cv, double X, double Y, double rho) {
    const double c1 = X / rho, s1 = Y / rho;
    double cm = 1.0, sm = 0.0, r = cv.a[0];
    for (int m = 1; m <= cv.nmodes; ++m) {
        const double cn = cm * c1 - sm * s1;
        sm = sm * c1 + cm * s1;
        cm = cn;
        r += cv.a[2 * m - 1] * cm + cv.a[2 * m] * sm;
    }
    return r;
}

__global__ __launch_bounds__(256) void k_radial_band(SeedArgs a, int8_t* cls, int32_t* cand, int64_t cap,
                                                     int* counters) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)a.nx * a.ny) return;
    const int i = (int)(idx / a.ny);
    const int j = (int)(idx - (int64_t)i * a.ny);
    const double X = a.x0 + i * a.h;
    const double Y = a.y0 + j * a.h;
    const double rho = sqrt(X * X + Y * Y);
    int8_t c;
    if (rho == 0.0) {
        c = 1;   // the origin is inside a polar domain
    } else {
        const double dr = rho - polar_radius_at(a.curve, X, Y, rho);
        if (dr >= a.band_lo && dr <= a.band_hi) {
            const int slot = atomicAdd(&counters[3], 1);
            if (slot < cap) cand[slot] = (int32_t)idx;
            c = 3;   // pending: written by the seed kernel
        } else {
            c = dr < 0 ? 1 : 0;
        }
    }
    cls[idx] = c;
}

__global__ __launch_bounds__(256) void k_seed_polar(SeedArgs a, const int32_t* __restrict__ cand, int64_t ncand,
                                                    int8_t* cls, StripRec* rec, int64_t cap, int* counters) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ncand) return;
    const int64_t idx = cand[k];
    const int i = (int)(idx / a.ny);
    const int j = (int)(idx - (int64_t)i * a.ny);
    const double X = a.x0 + i * a.h;
    const double Y = a.y0 + j * a.h;
    double th = 0.0, eta = 0.0;
    int it = 0;
    const int st = foot_from_seed(a.curve, X, Y, atan2(Y, X), 2.0 * a.k2, a.maxit, &th, &eta, &it);
    store_solved(idx, X, Y, st, th, eta, it, nearest_sample(th, a.k2, a.B), a.width, cls, rec, cap, counters);
}

__global__ void k_zero_int(int* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

int launch_classify(const ClassifyArgs& a, int8_t* d_cls, StripRec* d_rec, int64_t cap, uint64_t* d_near,
                    int* d_counters, hipStream_t s) {
    const int64_t npts = (int64_t)a.nx * a.ny;
    k_zero_int<<<1, 64, 0, s>>>(d_counters, 8);
    k_fill_u64<<<(unsigned)((npts + 255) / 256), 256, 0, s>>>(d_near, npts, ~0ull);
    k_near_scatter<<<a.B, 256, 0, s>>>(a, d_near);
    const unsigned nb = (unsigned)((npts + 255) / 256);
    switch (a.M) {
        case 4: k_classify<4><<<nb, 256, 0, s>>>(a, d_near, d_cls, d_rec, cap, d_counters); break;
        case 5: k_classify<5><<<nb, 256, 0, s>>>(a, d_near, d_cls, d_rec, cap, d_counters); break;
        case 6: k_classify<6><<<nb, 256, 0, s>>>(a, d_near, d_cls, d_rec, cap, d_counters); break;
        case 7: k_classify<7><<<nb, 256, 0, s>>>(a, d_near, d_cls, d_rec, cap, d_counters); break;
        case 8: k_classify<8><<<nb, 256, 0, s>>>(a, d_near, d_cls, d_rec, cap, d_counters); break;
        case 13: k_classify<13><<<nb, 256, 0, s>>>(a, d_near, d_cls, d_rec, cap, d_counters); break;
        case 15: k_classify<15><<<nb, 256, 0, s>>>(a, d_near, d_cls, d_rec, cap, d_counters); break;
        default: set_error("unsupported M"); return FC2D_E_ARG;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("classification launch: ") + hipGetErrorString(e));
        return FC2D_E_HIP;
    }
    trace_point("k_classify", s);
    return FC2D_OK;
}

static int launch_status(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string(what) + ": " + hipGetErrorString(e));
        return FC2D_E_HIP;
    }
    return FC2D_OK;
}

int launch_radial_band(const SeedArgs& a, int8_t* d_cls, int32_t* d_cand, int64_t cap, int* d_counters,
                       hipStream_t s) {
    const int64_t npts = (int64_t)a.nx * a.ny;
    k_zero_int<<<1, 64, 0, s>>>(d_counters, 8);
    k_radial_band<<<(unsigned)((npts + 255) / 256), 256, 0, s>>>(a, d_cls, d_cand, cap, d_counters);
    if (int st = launch_status("radial band launch")) return st;
    trace_point("k_radial_band", s);
    return FC2D_OK;
}

int launch_seed_polar(const SeedArgs& a, const int32_t* d_cand, int64_t ncand, int8_t* d_cls, StripRec* d_rec,
                      int64_t cap, int* d_counters, hipStream_t s) {
    if (ncand <= 0) return FC2D_OK;
    k_seed_polar<<<(unsigned)((ncand + 255) / 256), 256, 0, s>>>(a, d_cand, ncand, d_cls, d_rec, cap, d_counters);
    if (int st = launch_status("polar seed launch")) return st;
    trace_point("k_seed_polar", s);
    return FC2D_OK;
}

}  // namespace fc2d
