// Kernels of the Fourier Forwarding solver's near-boundary stepper (U_B,
// Sec. 4.2): the second-order Taylor position and velocity updates of the
// stepped points, the interpolation closure of the boundary points, the
// 1D-FC (or short-run Lagrange) second derivatives along grid-line segments,
// and the combination with U_FC (eq. ff_soln).  All work lists are built on
// the host at solver creation (ffsolve.cpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "ffsolve_int.h"
#include "internal.h"

namespace fc2d {

namespace {

int ffs_check(const char* what, hipStream_t s) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string(what) + ": " + hipGetErrorString(e));
        return FC2D_E_HIP;
    }
    trace_point(what, s);
    return FC2D_OK;
}

unsigned blocks_for(int64_t n, int per) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + per - 1) / per, 1 << 16)); }

}  // namespace

__global__ void k_ffs_position(const int32_t* __restrict__ sidx, int64_t ns, double* __restrict__ u,
                               const double* __restrict__ v, const double* __restrict__ acc, double dt) {
    const double hdt2 = 0.5 * dt * dt;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < ns; k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = sidx[k];
        u[i] = u[i] + dt * v[i] + hdt2 * acc[k];
    }
}

__global__ void k_ffs_boundary(const FfBnd* __restrict__ bnd, int64_t nb, double* __restrict__ f,
                               const double* __restrict__ data) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nb; k += (int64_t)gridDim.x * blockDim.x) {
        const FfBnd b = bnd[k];
        double s = 0.0;
        for (int q = 0; q < b.nref; ++q) {
            const int32_t r = b.ref[q];
            s += b.w[q] * (r >= 0 ? f[r] : data[-1 - r]);
        }
        f[b.target] = s;
    }
}

// one wave per segment: the segment's values (and crossing data) in LDS, one
// output row per lane
__global__ __launch_bounds__(64) void k_ffs_accel(const FfSeg* __restrict__ seg, const int8_t* __restrict__ region,
                                                  const int32_t* __restrict__ sgrid, const double* __restrict__ mats,
                                                  int64_t ns, const double* __restrict__ u,
                                                  const double* __restrict__ ufc, const double* __restrict__ data,
                                                  double* __restrict__ accd) {
    __shared__ double val[kFfMaxSeg + 2];
    const FfSeg sg = seg[blockIdx.x];
    const int ax = sg.stride == 1 ? 1 : 0;
    for (int q = threadIdx.x; q < sg.n; q += 64) {
        const int64_t fi = sg.base + (int64_t)(sg.lo + q) * sg.stride;
        const int8_t r = region[fi];
        val[q] = (r == FFR_STEP || r == FFR_BND) ? u[fi] : ufc[fi];
    }
    if (threadIdx.x == 0) {
        val[sg.n] = sg.ca >= 0 ? data[sg.ca] : 0.0;
        val[sg.n + 1] = sg.cb >= 0 ? data[sg.cb] : 0.0;
    }
    __syncthreads();
    for (int p = sg.r0 + (int)threadIdx.x; p <= sg.r1; p += 64) {
        const int32_t k = sgrid[sg.base + (int64_t)p * sg.stride];
        if (k < 0) continue;
        const double* row = mats + sg.mat + (int64_t)(p - sg.row0) * sg.ld;
        // four partial sums, so four rows' loads are in flight together
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int q = 0;
        for (; q + 4 <= sg.ld; q += 4) {
            a0 = fma(row[q], val[q], a0);
            a1 = fma(row[q + 1], val[q + 1], a1);
            a2 = fma(row[q + 2], val[q + 2], a2);
            a3 = fma(row[q + 3], val[q + 3], a3);
        }
        for (; q < sg.ld; ++q) a0 = fma(row[q], val[q], a0);
        accd[(int64_t)ax * ns + k] = (a0 + a1) + (a2 + a3);
    }
}

__global__ void k_ffs_sum(const double* __restrict__ accd, int64_t ns, double* __restrict__ acc) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < ns; k += (int64_t)gridDim.x * blockDim.x)
        acc[k] = accd[k] + accd[ns + k];
}

__global__ void k_ffs_velocity(const int32_t* __restrict__ sidx, int64_t ns, double* __restrict__ v,
                               double* __restrict__ acc, const double* __restrict__ accd, double dt) {
    const double hdt = 0.5 * dt;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < ns; k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = sidx[k];
        const double an = accd[k] + accd[ns + k];
        v[i] = v[i] + hdt * (acc[k] + an);
        acc[k] = an;
    }
}

__global__ void k_ffs_combine(const int8_t* __restrict__ region, int64_t npts, const double* __restrict__ ufc,
                              const double* __restrict__ utfc, double* __restrict__ u, double* __restrict__ ut) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < npts; k += (int64_t)gridDim.x * blockDim.x) {
        const int8_t r = region[k];
        if (r == FFR_INT) {
            u[k] = ufc[k];
            ut[k] = utfc[k];
        } else if (r == FFR_OUT) {
            u[k] = 0.0;
            ut[k] = 0.0;
        }
    }
}

int ffs_position(const FfDev& d, double* u, const double* v, const double* acc, double dt, hipStream_t s) {
    if (d.ns == 0) return FC2D_OK;
    k_ffs_position<<<blocks_for(d.ns, 256), 256, 0, s>>>(d.sidx, d.ns, u, v, acc, dt);
    return ffs_check("k_ffs_position", s);
}

int ffs_boundary(const FfDev& d, double* f, const double* data, hipStream_t s) {
    if (d.nb == 0) return FC2D_OK;
    k_ffs_boundary<<<blocks_for(d.nb, 256), 256, 0, s>>>(d.bnd, d.nb, f, data);
    return ffs_check("k_ffs_boundary", s);
}

int ffs_accel(const FfDev& d, const double* u, const double* ufc, const double* data, double* accd, hipStream_t s) {
    if (d.nseg == 0) return FC2D_OK;
    k_ffs_accel<<<d.nseg, 64, 0, s>>>(d.seg, d.region, d.sgrid, d.mats, d.ns, u, ufc, data, accd);
    return ffs_check("k_ffs_accel", s);
}

int ffs_sum_acc(const FfDev& d, const double* accd, double* acc, hipStream_t s) {
    if (d.ns == 0) return FC2D_OK;
    k_ffs_sum<<<blocks_for(d.ns, 256), 256, 0, s>>>(accd, d.ns, acc);
    return ffs_check("k_ffs_sum", s);
}

int ffs_velocity(const FfDev& d, double* v, double* acc, const double* accd, double dt, hipStream_t s) {
    if (d.ns == 0) return FC2D_OK;
    k_ffs_velocity<<<blocks_for(d.ns, 256), 256, 0, s>>>(d.sidx, d.ns, v, acc, accd, dt);
    return ffs_check("k_ffs_velocity", s);
}

int ffs_combine(const FfDev& d, const double* ufc, const double* utfc, double* u, double* ut, hipStream_t s) {
    k_ffs_combine<<<blocks_for(d.npts, 256), 256, 0, s>>>(d.region, d.npts, ufc, utfc, u, ut);
    return ffs_check("k_ffs_combine", s);
}

}  // namespace fc2d
