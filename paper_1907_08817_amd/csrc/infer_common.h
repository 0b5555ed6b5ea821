// Per-key device helpers of the map step shared by both inference forms:
// translate (input phase) and slot rounding (sorting phase).
#pragma once
#include "nnsort_internal.h"

namespace nns {

__device__ __forceinline__ bool translate_key(uint64_t bits, bool is_f64, double lo, double inv,
                                              double* xhat) {
    double x;
    if (is_f64) {
        if ((bits & 0x7FF0000000000000ull) == 0x7FF0000000000000ull) return false;  // Inf/NaN
        x = __longlong_as_double((long long)bits);
    } else {
        x = __ull2double_rn(bits);
    }
    double t = (x - lo) * inv;
    if (t != t) return false;
    t = t < 0.0 ? 0.0 : t;
    t = t > 1.0 ? 1.0 : t;
    *xhat = t;
    return true;
}

__device__ __forceinline__ uint32_t slot_of(double F, double M) {
    if (F != F) return kUnmapped;
    double v = F * M;
    v = v < 0.0 ? 0.0 : v;
    v = v > M ? M : v;
    double t = trunc(v);
    if (v - t >= 0.5) t += 1.0;
    return (uint32_t)t;
}

__device__ __forceinline__ float two_sum(float a, float b, float& err) {
    float s = a + b;
    float bb = s - a;
    err = (a - (s - bb)) + (b - bb);
    return s;
}

}  // namespace nns
