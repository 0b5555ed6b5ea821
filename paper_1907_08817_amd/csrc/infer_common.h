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

// Spilled keys are staged per wave in LDS and written out 256 at a time with
// one atomic on the spill counter, so sparse spills (a few per wave) do not
// serialise the grid on that counter.  count is wave-uniform.
constexpr int kSpillStage = 256;
struct WaveSpill {
    SpillEntry* buf;  // this wave's LDS staging area (kSpillStage entries)
    uint32_t count;
    uint32_t unmapped;
};

__device__ __forceinline__ void spill_flush(WaveSpill& w, SpillEntry* spill, unsigned long long* counter) {
    if (w.count == 0) return;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(counter, (unsigned long long)w.count);
    base = __shfl(base, 0);
    for (uint32_t e = lane_id(); e < w.count; e += 64) spill[base + e] = w.buf[e];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    w.count = 0;
}

__device__ __forceinline__ void spill_stage(bool want, const SpillEntry& e, WaveSpill& w, SpillEntry* spill,
                                            unsigned long long* counter) {
    unsigned long long mask = __ballot(want);
    if (mask == 0) return;
    uint32_t n = (uint32_t)__popcll(mask);
    if (w.count + n > (uint32_t)kSpillStage) spill_flush(w, spill, counter);
    if (want) w.buf[w.count + __popcll(mask & ((1ull << lane_id()) - 1ull))] = e;
    w.count += n;
}

// Write out what the wave still stages, and its count of keys without a slot.
__device__ __forceinline__ void spill_finish(WaveSpill& w, const InferArgs& a) {
    if (!a.scatter) return;
    spill_flush(w, a.spill, &a.counters[kCntSpill]);
    if (w.unmapped && lane_id() == 0) atomicAdd(&a.counters[kCntUnmapped], (unsigned long long)w.unmapped);
}

__device__ __forceinline__ void count_aggregate(bool want, unsigned long long* counter) {
    unsigned long long mask = __ballot(want);
    if (mask && (int)lane_id() == __ffsll((long long)mask) - 1)
        atomicAdd(counter, (unsigned long long)__popcll(mask));
}

// Hand a key to the region of its slot range, or to the spill list when the
// region is full (or the key has no slot).  Once a range's counter is past its
// capacity every further key of the range goes straight to the spill list, so
// a dense range does not serialise the grid on its counter.
__device__ __forceinline__ void place_key(const InferArgs& a, int64_t i, bool active, uint64_t okey,
                                          uint32_t slot, WaveSpill& w) {
    bool unm = active && slot == kUnmapped;
    if (a.scatter) {
        bool to_spill = unm;
        if (active && !unm) {
            uint32_t b = slot >> kLogBucketSlots;
            uint32_t seen = __builtin_nontemporal_load(&a.cnt[b]);
            if (seen > kBucketCap) {
                to_spill = true;
            } else {
                uint32_t pos = atomicAdd(&a.cnt[b], 1u);
                if (pos < kBucketCap) {
                    RegionEntry r{okey, ((uint64_t)(uint32_t)i << 32) | (slot & (kBucketSlots - 1))};
                    a.region[(size_t)b * kBucketCap + pos] = r;
                } else {
                    to_spill = true;
                }
            }
        }
        SpillEntry se{okey, (uint32_t)i, slot};
        spill_stage(to_spill, se, w, a.spill, &a.counters[kCntSpill]);
        w.unmapped += (uint32_t)__popcll(__ballot(unm));
    }
}

}  // namespace nns
