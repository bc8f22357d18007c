// Double-double arithmetic (an unevaluated sum hi + lo of two doubles) for
// device code: error-free TwoSum and FMA-based TwoProduct.  Contraction of
// a * b + c into an FMA is switched off inside these functions: fusing the
// product of TwoProduct into the following sum would break the error-free
// transformations.  Used where the
// continuation's amplification (|A_r Q^T| ~ 1e4) would otherwise turn
// float64 rounding in the matching values into visible error.
#pragma once

#include <hip/hip_runtime.h>

namespace fc2d {

struct dd {
    double hi, lo;
};

__device__ __forceinline__ dd dd_two_sum(double a, double b) {
#pragma clang fp contract(off)
    const double s = a + b;
    const double bb = s - a;
    const double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}

__device__ __forceinline__ dd dd_quick(double a, double b) {
#pragma clang fp contract(off)
    const double s = a + b;
    const double e = b - (s - a);
    return {s, e};
}

__device__ __forceinline__ dd dd_add(dd x, dd y) {
#pragma clang fp contract(off)
    dd s = dd_two_sum(x.hi, y.hi);
    const dd t = dd_two_sum(x.lo, y.lo);
    s.lo += t.hi;
    s = dd_quick(s.hi, s.lo);
    s.lo += t.lo;
    return dd_quick(s.hi, s.lo);
}

__device__ __forceinline__ dd dd_mul_d(dd x, double y) {
#pragma clang fp contract(off)
    const double p = x.hi * y;
    double e = fma(x.hi, y, -p);
    e = fma(x.lo, y, e);
    return dd_quick(p, e);
}

__device__ __forceinline__ dd dd_mul(dd x, dd y) {
#pragma clang fp contract(off)
    const double p = x.hi * y.hi;
    double e = fma(x.hi, y.hi, -p);
    e = fma(x.hi, y.lo, e);
    e = fma(x.lo, y.hi, e);
    return dd_quick(p, e);
}

__device__ __forceinline__ dd dd_shfl_xor(dd x, int m) {
    return {__shfl_xor(x.hi, m, 64), __shfl_xor(x.lo, m, 64)};
}

__device__ __forceinline__ dd dd_shfl(dd x, int src) {
    return {__shfl(x.hi, src, 64), __shfl(x.lo, src, 64)};
}

}  // namespace fc2d
