// Device helper shared by the classification kernels: class of a solved point
// from its signed distance (Sec. 3.5 step 4) and its STRIP record.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace fc2d {

// status st of the foot solve of grid point idx = (X, Y); theta, eta its foot,
// it its Newton steps.  Within rounding distance of Gamma counts as on Gamma: IN.
__device__ inline void store_solved(int64_t idx, double X, double Y, int st, double theta, double eta, int it,
                                    int32_t seed, double width, int8_t* cls, StripRec* rec, int64_t cap,
                                    int* counters) {
    int8_t c = 0;
    if (st != FOOT_OK) {
        atomicAdd(&counters[1], 1);
    } else {
        const double on_tol = 1e-13 * (1.0 + fabs(X) + fabs(Y));
        c = eta <= on_tol ? 1 : (eta <= width ? 2 : 0);
        if (c == 2) {
            const int slot = atomicAdd(&counters[0], 1);
            if (slot < cap) {
                StripRec r;
                r.idx = (int32_t)idx;
                r.seed = seed;
                r.iters = it;
                r.pad = 0;
                r.theta = theta;
                r.eta = eta;
                rec[slot] = r;
            }
            atomicMax(&counters[2], it);
        }
    }
    atomicAdd(&counters[5], it);
    cls[idx] = c;
}

// nearest boundary sample index to theta in [0, 2 pi)
__device__ inline int32_t nearest_sample(double theta, double k2, int B) {
    int p = (int)rint(theta / k2);
    return p >= B ? p - B : p;
}

}  // namespace fc2d
