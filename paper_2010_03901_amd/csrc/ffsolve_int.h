// Internal declarations of the Fourier Forwarding solver (ffsolve.cpp host
// set-up, kernels_ffsolve.hip kernels).  Not part of the public ABI.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime_api.h>

namespace fc2d {

// grid-point regions of the solver
enum { FFR_OUT = 0, FFR_INT = 1, FFR_STEP = 2, FFR_BND = 3 };

constexpr int kFfMaxSeg = 2048;   // longest derivative segment (values held in LDS)

// a boundary point: its value = sum_q w[q] * (ref[q] >= 0 ? field[ref[q]] : data[-1 - ref[q]])
struct FfBnd {
    int32_t target;
    int32_t nref;
    int32_t ref[4];
    double w[4];
};

// a derivative segment along one grid line: values at positions lo .. lo + n - 1
// (flat index base + position * stride); output rows r0 .. r1 (written at
// stepped points only), row p of the matrix at mat + (p - row0) * ld; lag
// segments append the crossing values ca, cb (-1: column unused) as columns
// n and n + 1
struct FfSeg {
    int64_t mat;
    int32_t base, stride;
    int32_t lo, n, r0, r1;
    int32_t row0, ld;
    int32_t ca, cb;
};

struct FfDev {
    const int8_t* region;
    const int32_t* sidx;
    const int32_t* sgrid;
    const FfBnd* bnd;
    const FfSeg* seg;
    const double* mats;
    int64_t ns, nb;
    int nseg;
    int64_t npts;
};

// u[stepped] += dt v + dt^2 / 2 acc
int ffs_position(const FfDev& d, double* u, const double* v, const double* acc, double dt, hipStream_t s);
// boundary points of f from the stepped points and the crossing data
int ffs_boundary(const FfDev& d, double* f, const double* data, hipStream_t s);
// per-direction second derivatives (times c^2) at the stepped points: accd [2][ns];
// segment values from u on the boundary region and from ufc elsewhere
int ffs_accel(const FfDev& d, const double* u, const double* ufc, const double* data, double* accd, hipStream_t s);
// acc = accd[0] + accd[1]
int ffs_sum_acc(const FfDev& d, const double* accd, double* acc, hipStream_t s);
// v[stepped] += dt (acc + a_new) / 2, acc <- a_new = accd[0] + accd[1]
int ffs_velocity(const FfDev& d, double* v, double* acc, const double* accd, double dt, hipStream_t s);
// interior points take U_FC, points outside Omega 0
int ffs_combine(const FfDev& d, const double* ufc, const double* utfc, double* u, double* ut, hipStream_t s);

}  // namespace fc2d
