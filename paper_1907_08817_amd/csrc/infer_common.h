// Per-key device helpers of the map step shared by both inference forms:
// translate (input phase), slot rounding, and the hand-off of a key to its
// bucket region or to the spill list (sorting phase).
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

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Wave-aggregated append of one entry per participating lane.
__device__ __forceinline__ void spill_append(bool want, SpillEntry e, SpillEntry* spill,
                                             unsigned long long* counter) {
    unsigned long long mask = __ballot(want);
    if (mask == 0) return;
    int leader = __ffsll((long long)mask) - 1;
    unsigned long long base = 0;
    if ((int)lane_id() == leader) base = atomicAdd(counter, (unsigned long long)__popcll(mask));
    base = __shfl(base, leader);
    if (want) {
        unsigned long long below = mask & ((1ull << lane_id()) - 1ull);
        spill[base + __popcll(below)] = e;
    }
}

__device__ __forceinline__ void count_aggregate(bool want, unsigned long long* counter) {
    unsigned long long mask = __ballot(want);
    if (mask && (int)lane_id() == __ffsll((long long)mask) - 1)
        atomicAdd(counter, (unsigned long long)__popcll(mask));
}

__device__ __forceinline__ void place_key(const InferArgs& a, int64_t i, bool active, uint64_t okey,
                                          uint32_t slot) {
    bool unm = active && slot == kUnmapped;
    if (a.scatter) {
        bool to_spill = unm;
        if (active && !unm) {
            uint32_t b = slot >> kLogBucketSlots;
            uint32_t pos = atomicAdd(&a.cnt[b], 1u);
            if (pos < kBucketCap) {
                size_t e = (size_t)b * kBucketCap + pos;
                a.region_key[e] = okey;
                a.region_meta[e] = ((uint64_t)(uint32_t)i << 32) | (slot & (kBucketSlots - 1));
            } else {
                to_spill = true;
            }
        }
        SpillEntry se{okey, (uint32_t)i, slot};
        spill_append(to_spill, se, a.spill, &a.counters[kCntSpill]);
        count_aggregate(unm, &a.counters[kCntUnmapped]);
    }
}

}  // namespace nns
