// One pass of an LSD (least significant digit first) radix scatter on 64-bit
// keys with 256 digits, shared by the partition of keys by slot range and by
// the conventional sort of the residue.
//
// A pass is reduce-then-scan over tiles of kLsdTile keys in input order:
//   1. k_lsd_upsweep: each tile's digit histogram, stored as hist[tile][digit]
//      (coalesced);
//   2. launch_lsd_scan: offsets = exclusive prefix over (digit, tile), in two
//      coalesced passes over chunks of kScanTiles tiles;
//   3. k_lsd_downsweep: each key's rank among its tile's keys of the same
//      digit, the tile reordered by digit in LDS, then written out in runs.
// Only passes after the first must be stable (for LSD, the order that a later
// pass must keep is the one earlier passes made); the first pass ranks with
// LDS atomics, the others match digits within a wave by ballots, bit by bit.
//
// Keys move as unsigned order keys; in_mode / out_mode convert from / to the
// caller's bit patterns on the first / last pass (0 order keys, 1 binary64
// bits, 2 uint64).  A 32-bit payload (the slot) can travel with each key.
#pragma once
#include "nnsort_internal.h"

namespace nns {

constexpr int kLsdThreads = 512;
constexpr int kLsdTile = kPartTile;                   // 2048 keys
constexpr int kLsdItems = kLsdTile / kLsdThreads;     // 4 per thread
constexpr int kLsdWaves = kLsdThreads / 64;           // 8
constexpr int kScanTiles = 128;                       // tiles per scan chunk

__device__ __forceinline__ uint64_t to_order_key(uint64_t v, int mode) {
    return mode == 1 ? order_key(v, true) : v;  // modes 0 (order key) and 2 (u64) are identities
}
__device__ __forceinline__ uint64_t from_order_key(uint64_t v, int mode) {
    return mode == 1 ? order_key_inverse(v, true) : v;
}

// Digit of a (key, slot) pair: the range id's digit (partition by slot
// range) or the key's byte (radix sort).
struct RangeDigit {
    uint32_t NB;
    int shift;
    uint32_t mask;
    __device__ __forceinline__ uint32_t operator()(uint64_t, uint32_t slot) const {
        return (range_of(slot, NB) >> shift) & mask;
    }
};
struct KeyDigit {
    int shift;
    __device__ __forceinline__ uint32_t operator()(uint64_t key, uint32_t) const {
        return (uint32_t)(key >> shift) & 255u;
    }
};

// Tile of virtual index v.  Workgroups are dealt to the 8 XCDs in turn
// (workgroup i on XCD i mod 8), so XCD x is given the x-th contiguous eighth
// of the tiles: the runs that consecutive tiles write for one digit are then
// adjacent in memory and meet in the same L2 before they are written back.
__device__ __forceinline__ int64_t xcd_tile(int64_t v, int64_t ntiles) {
    const int64_t q = ntiles >> 3, r = ntiles & 7;
    const int64_t x = v & 7, j = v >> 3;
    return x * q + (x < r ? x : r) + j;
}

__device__ __forceinline__ uint32_t lanes_below(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Digit histogram of one tile.  PAYLOAD: the digit comes from the slot, so
// only slots are read; otherwise from the key (converted by in_mode).
template <bool PAYLOAD, class D>
__global__ void __launch_bounds__(kLsdThreads) k_lsd_upsweep(const uint64_t* __restrict__ keys,
                                                             const uint32_t* __restrict__ slots, int64_t n,
                                                             int in_mode, D dig, uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[256];
    if (threadIdx.x < 256) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kLsdTile;
    // full tile of a 16-byte-aligned array (a tile is a multiple of 16 bytes
    // long): 16-byte loads; otherwise one element per load
    const uintptr_t base = PAYLOAD ? (uintptr_t)slots : (uintptr_t)keys;
    if (t0 + kLsdTile <= n && (base & 15) == 0) {
        if (PAYLOAD) {
            const uint4* v = (const uint4*)(slots + t0);
#pragma unroll
            for (int k = 0; k < kLsdTile / (4 * kLsdThreads); ++k) {
                const uint4 q = v[k * kLsdThreads + threadIdx.x];
                atomicAdd(&h[dig(0, q.x)], 1u);
                atomicAdd(&h[dig(0, q.y)], 1u);
                atomicAdd(&h[dig(0, q.z)], 1u);
                atomicAdd(&h[dig(0, q.w)], 1u);
            }
        } else {
            const ulonglong2* v = (const ulonglong2*)(keys + t0);
#pragma unroll
            for (int k = 0; k < kLsdTile / (2 * kLsdThreads); ++k) {
                const ulonglong2 q = v[k * kLsdThreads + threadIdx.x];
                atomicAdd(&h[dig(to_order_key(q.x, in_mode), 0)], 1u);
                atomicAdd(&h[dig(to_order_key(q.y, in_mode), 0)], 1u);
            }
        }
    } else {
        for (int64_t i = t0 + threadIdx.x; i < n; i += kLsdThreads) {
            const uint32_t d = PAYLOAD ? dig(0, slots[i]) : dig(to_order_key(keys[i], in_mode), 0);
            atomicAdd(&h[d], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < 256) hist[(int64_t)blockIdx.x * 256 + threadIdx.x] = h[threadIdx.x];
}

// Scatter of one pass.  hist / chunk: the scanned offsets (a tile's output
// offset for digit d is hist[t][d] + chunk[t / kScanTiles][d]).  Keys are
// converted by in_mode on load and by out_mode on store.
//
// BATCH: a thread's kLsdItems loads are all issued before the first is
// ranked, instead of each after the previous item's ranking.  Measured per
// pass: the stable passes of a three-pass partition (1e9 keys) run 0.6 ms
// faster each that way, while the two passes at 1e8 keys and the first pass
// at 1e9 run 4-5% slower, so the partition asks for it only there.
template <bool STABLE, bool PAYLOAD, class D, bool BATCH = false>
__global__ void __launch_bounds__(kLsdThreads) k_lsd_downsweep(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ sin, uint64_t* __restrict__ kout,
    uint32_t* __restrict__ sout, int64_t n, int in_mode, int out_mode, D dig, int nbits,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ chunk, int64_t ntiles) {
    // the rank counters are dead once every key knows its place in the tile,
    // so they share storage with the staged payloads
    __shared__ uint64_t s_key[kLsdTile];
    __shared__ union {
        uint32_t slot[kLsdTile];
        uint32_t cnt[kLsdWaves][256];
    } s_u;
    __shared__ uint32_t dstart[256];
    __shared__ uint32_t gofs[256];
    __shared__ uint32_t wtot[kLsdWaves];
    const int lane = __lane_id();
    const int w = threadIdx.x >> 6;
    const int64_t tile = xcd_tile(blockIdx.x, ntiles);
    const int64_t tile0 = tile * kLsdTile;
    const int lim = (int)(n - tile0 < kLsdTile ? n - tile0 : kLsdTile);
    for (int i = threadIdx.x; i < kLsdWaves * 256; i += kLsdThreads) (&s_u.cnt[0][0])[i] = 0;
    if (threadIdx.x < 256)
        gofs[threadIdx.x] = hist[tile * 256 + threadIdx.x] + chunk[(tile / kScanTiles) * 256 + threadIdx.x];
    __syncthreads();

    const uint64_t* __restrict__ kb = kin + tile0;
    const uint32_t* __restrict__ sb = PAYLOAD ? sin + tile0 : nullptr;
    uint64_t key[kLsdItems];
    uint32_t slot[kLsdItems];
    uint32_t rank[kLsdItems];
    if (BATCH) {  // no branch between the loads: items past the tile's end read its last key again
#pragma unroll
        for (int k = 0; k < kLsdItems; ++k) {
            const int idx = w * (kLsdItems * 64) + k * 64 + lane;
            const int ic = idx < lim ? idx : lim - 1;
            key[k] = kb[ic];
            slot[k] = PAYLOAD ? sb[ic] : 0;
        }
    }
#pragma unroll
    for (int k = 0; k < kLsdItems; ++k) {
        const int idx = w * (kLsdItems * 64) + k * 64 + lane;
        const bool valid = idx < lim;
        if (BATCH) {
            key[k] = to_order_key(valid ? key[k] : 0, in_mode);
            slot[k] = valid ? slot[k] : 0;
        } else {
            key[k] = to_order_key(valid ? kb[idx] : 0, in_mode);
            slot[k] = PAYLOAD && valid ? sb[idx] : 0;
        }
        const uint32_t d = dig(key[k], slot[k]);
        if (STABLE) {
            unsigned long long peers = __ballot(valid);
#pragma unroll
            for (int bit = 0; bit < 8; ++bit) {
                if (bit >= nbits) break;
                const bool on = (d >> bit) & 1u;
                const unsigned long long bb = __ballot(on);
                peers &= on ? bb : ~bb;
            }
            const uint32_t below = lanes_below(peers);
            const uint32_t base = valid ? s_u.cnt[w][d] : 0;
            rank[k] = base + below;
            if (valid && below == 0) s_u.cnt[w][d] = base + (uint32_t)__popcll(peers);
        } else {
            if (valid) rank[k] = atomicAdd(&s_u.cnt[0][d], 1u);
        }
    }
    __syncthreads();
    // digit d = threadIdx.x < 256 (waves 0..3): tile total, block-wide
    // exclusive scan over digits, then (STABLE) each wave's start inside the
    // digit's run
    {
        const uint32_t d = threadIdx.x;
        uint32_t tot = 0, inc = 0;
        if (d < 256) {
            if (STABLE) {
#pragma unroll
                for (int ww = 0; ww < kLsdWaves; ++ww) tot += s_u.cnt[ww][d];
            } else {
                tot = s_u.cnt[0][d];
            }
            inc = tot;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                uint32_t y = __shfl_up(inc, o);
                if (lane >= o) inc += y;
            }
            if (lane == 63) wtot[w] = inc;
        }
        __syncthreads();
        if (d < 256) {
            uint32_t run = inc - tot;
            for (int ww = 0; ww < w; ++ww) run += wtot[ww];
            dstart[d] = run;
            if (STABLE) {
#pragma unroll
                for (int ww = 0; ww < kLsdWaves; ++ww) {
                    uint32_t c = s_u.cnt[ww][d];
                    s_u.cnt[ww][d] = run;
                    run += c;
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kLsdItems; ++k) {
        const int idx = w * (kLsdItems * 64) + k * 64 + lane;
        if (idx < lim) {
            const uint32_t d = dig(key[k], slot[k]);
            rank[k] += STABLE ? s_u.cnt[w][d] : dstart[d];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kLsdItems; ++k) {
        const int idx = w * (kLsdItems * 64) + k * 64 + lane;
        if (idx < lim) {
            s_key[rank[k]] = key[k];
            if (PAYLOAD) s_u.slot[rank[k]] = slot[k];
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < lim; i += kLsdThreads) {
        const uint64_t k = s_key[i];
        const uint32_t sl = PAYLOAD ? s_u.slot[i] : 0;
        const uint32_t d = dig(k, sl);
        const uint32_t pos = gofs[d] + (uint32_t)i - dstart[d];
        kout[pos] = from_order_key(k, out_mode);
        if (PAYLOAD) sout[pos] = sl;
    }
}

// Host side (lsd.hip): the offsets scan of one pass, and the workspace words
// of the tile histograms plus chunk offsets for n keys.
hipError_t launch_lsd_scan(uint32_t* hist, int64_t ntiles, hipStream_t st);
size_t lsd_hist_words(int64_t n);

}  // namespace nns
