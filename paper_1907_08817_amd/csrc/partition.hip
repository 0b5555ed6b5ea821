// Hand-off of keys to slot ranges (Sec. 2, Sorting Phase: each key goes to the
// slot its predicted position names).  Keys are grouped by slot range with a
// stable LSD partition on the range id -- digit histograms per tile, one
// exclusive scan over (digit, tile), and a scatter that ranks keys inside a
// wave by ballot matching -- so within a range keys keep their input order:
// the first key of a slot in range order is the slot's first arrival.  No
// per-key atomics: MI355X's 8 XCDs keep separate L2s, and a device-wide
// counter per range would serialise the scatter.
#include "nnsort_internal.h"

namespace nns {

constexpr int kPartThreads = 256;
constexpr int kPartItems = 16;
constexpr int kPartTile = kPartThreads * kPartItems;  // 4096
constexpr int kPartWaves = kPartThreads / 64;

// Range id of a slot; keys without a slot sort after every range.
__device__ __forceinline__ uint32_t range_of(uint32_t slot, uint32_t NB) {
    return slot == kUnmapped ? NB : (slot >> kLogBucketSlots);
}

__global__ void __launch_bounds__(kPartThreads) k_part_upsweep(const uint32_t* __restrict__ slots, int64_t n,
                                                               uint32_t NB, int shift, uint32_t mask,
                                                               uint32_t* blockhist, int64_t nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kPartTile;
#pragma unroll 4
    for (int k = 0; k < kPartItems; ++k) {
        int64_t i = t0 + k * kPartThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(range_of(slots[i], NB) >> shift) & mask], 1u);
    }
    __syncthreads();
    blockhist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of (key, slot) pairs by one digit of the range id.  in_bits:
// keys arrive as caller bit patterns (first pass) and leave as order keys.
__global__ void __launch_bounds__(kPartThreads) k_part_downsweep(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ sin, uint64_t* __restrict__ kout,
    uint32_t* __restrict__ sout, int64_t n, uint32_t NB, int shift, uint32_t mask, int in_bits, int is_f64,
    const uint32_t* __restrict__ scanned, int64_t nblocks) {
    __shared__ uint32_t wcnt[kPartWaves][256];
    __shared__ uint32_t gofs[256];
    const int lane = __lane_id();
    const int w = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < kPartWaves * 256; i += kPartThreads) (&wcnt[0][0])[i] = 0;
    gofs[threadIdx.x] = scanned[(int64_t)threadIdx.x * nblocks + blockIdx.x];
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kPartTile + (int64_t)w * (kPartItems * 64);
    uint64_t key[kPartItems];
    uint32_t slot[kPartItems];
    uint32_t rank[kPartItems];
    const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int k = 0; k < kPartItems; ++k) {
        int64_t i = t0 + k * 64 + lane;
        bool valid = i < n;
        uint64_t v = valid ? kin[i] : 0;
        key[k] = in_bits ? order_key(v, is_f64) : v;
        slot[k] = valid ? sin[i] : 0;
        uint32_t d = (range_of(slot[k], NB) >> shift) & mask;
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            unsigned long long bb = __ballot(valid && ((d >> bit) & 1u));
            peers &= ((d >> bit) & 1u) ? bb : ~bb;
        }
        uint32_t base = valid ? wcnt[w][d] : 0;
        rank[k] = base + (uint32_t)__popcll(peers & lt);
        if (valid && (peers & lt) == 0) wcnt[w][d] = base + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    {
        uint32_t d = threadIdx.x;
        uint32_t run = gofs[d];
#pragma unroll
        for (int ww = 0; ww < kPartWaves; ++ww) {
            uint32_t c = wcnt[ww][d];
            wcnt[ww][d] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPartItems; ++k) {
        int64_t i = t0 + k * 64 + lane;
        if (i < n) {
            uint32_t d = (range_of(slot[k], NB) >> shift) & mask;
            uint32_t pos = wcnt[w][d] + rank[k];
            kout[pos] = key[k];
            sout[pos] = slot[k];
        }
    }
}

// start[r] = first position of range r in the range-sorted slots (r = 0..NB,
// range NB holding the keys without a slot), start[NB + 1] = n; cnt[r] for
// r < NB.
__global__ void __launch_bounds__(256) k_range_bounds(const uint32_t* __restrict__ s, int64_t n, uint32_t NB,
                                                      int64_t* start) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > (int64_t)NB + 1) return;
    int64_t lo = 0, hi = n;
    if (r == (int64_t)NB + 1) {
        lo = n;
    } else {
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (range_of(s[mid], NB) < (uint32_t)r) lo = mid + 1;
            else hi = mid;
        }
    }
    start[r] = lo;
}

__global__ void __launch_bounds__(256) k_range_counts(const int64_t* __restrict__ start, uint32_t NB, uint32_t* cnt) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < (int64_t)NB) cnt[r] = (uint32_t)(start[r + 1] - start[r]);
}

__global__ void __launch_bounds__(256) k_check_slots(const uint32_t* __restrict__ s, int64_t n, int64_t S,
                                                     unsigned long long* bad) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint32_t v = s[i];
        c += (v != kUnmapped && (int64_t)v >= S) ? 1 : 0;
    }
    if (c) atomicAdd(bad, c);
}

// ---- dense ranges (more keys than one LDS tile holds) and keys without a
// slot: copied to G; a dense range's slot multiplicities are counted in LDS
// per chunk and added to its histogram, for the round counts.
constexpr int kChunk = 4096;

// chunk_pref[i] = number of chunks of big ranges 0..i-1 (i = 0..big_count).
__global__ void k_big_chunks(const int32_t* __restrict__ bigbucket, int64_t big_count,
                             const int64_t* __restrict__ start, int64_t* chunk_pref, int64_t* gpref) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t c = 0, g = 0;
    for (int64_t i = 0; i < big_count; ++i) {
        chunk_pref[i] = c;
        gpref[i] = g;
        int32_t b = bigbucket[i];
        int64_t len = start[b + 1] - start[b];
        c += (len + kChunk - 1) / kChunk;
        g += len;
    }
    chunk_pref[big_count] = c;
    gpref[big_count] = g;
}

__global__ void __launch_bounds__(256) k_big_gather(const int32_t* __restrict__ bigbucket, int64_t big_count,
                                                    const int64_t* __restrict__ chunk_pref,
                                                    const int64_t* __restrict__ gpref,
                                                    const int64_t* __restrict__ start,
                                                    const uint64_t* __restrict__ K, const uint32_t* __restrict__ Sl,
                                                    uint32_t* hist, uint64_t* G) {
    __shared__ uint32_t h[kBucketSlots];
    const int64_t chunk = blockIdx.x;
    // big range of this chunk: last i with chunk_pref[i] <= chunk
    int64_t lo = 0, hi = big_count - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (chunk_pref[mid] <= chunk) lo = mid;
        else hi = mid - 1;
    }
    const int64_t id = lo;
    const int32_t b = bigbucket[id];
    const int64_t s0 = start[b], len = start[b + 1] - s0;
    const int64_t c0 = (chunk - chunk_pref[id]) * kChunk;
    const int64_t c1 = c0 + kChunk < len ? c0 + kChunk : len;
    for (int i = threadIdx.x; i < (int)kBucketSlots; i += blockDim.x) h[i] = 0;
    __syncthreads();
    for (int64_t e = c0 + threadIdx.x; e < c1; e += blockDim.x) {
        G[gpref[id] + e] = K[s0 + e];
        atomicAdd(&h[Sl[s0 + e] & (kBucketSlots - 1)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < (int)kBucketSlots; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[id * kBucketSlots + i], h[i]);
}

__global__ void __launch_bounds__(256) k_copy_u64(const uint64_t* __restrict__ in, uint64_t* out, int64_t n) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = in[i];
}

// ---- host-side launch sequence ----
hipError_t exclusive_scan_u32(uint32_t* data, int64_t len, uint32_t* sums, hipStream_t st);

int range_passes(uint32_t NB, int* shifts, uint32_t* masks) {
    int bits = 1;
    while (bits < 32 && ((uint64_t)NB >> bits) != 0) ++bits;  // range ids 0..NB
    int passes = (bits + 7) / 8;
    int per = (bits + passes - 1) / passes;
    for (int p = 0; p < passes; ++p) {
        shifts[p] = p * per;
        int w = bits - p * per < per ? bits - p * per : per;
        masks[p] = (1u << w) - 1u;
    }
    return passes;
}

size_t partition_hist_words(int64_t n) {
    int64_t nblocks = (n + kPartTile - 1) / kPartTile;
    return (size_t)256 * (nblocks > 0 ? nblocks : 1);
}

// Partition (keys, slots) by range id.  in_keys are caller bit patterns;
// result in (K[res], S[res]) as order keys; returns res via *which.
hipError_t partition_by_range(const uint64_t* in_keys, const uint32_t* in_slots, int64_t n, uint32_t NB, bool is_f64,
                              uint64_t* K0, uint32_t* S0, uint64_t* K1, uint32_t* S1, uint32_t* blockhist,
                              uint32_t* sums, int* which, hipStream_t st) {
    int shifts[4];
    uint32_t masks[4];
    int passes = range_passes(NB, shifts, masks);
    const int64_t nblocks = (n + kPartTile - 1) / kPartTile;
    uint64_t* Kb[2] = {K0, K1};
    uint32_t* Sb[2] = {S0, S1};
    const uint64_t* kin = in_keys;
    const uint32_t* sin = in_slots;
    hipError_t e;
    for (int p = 0; p < passes; ++p) {
        uint64_t* ko = Kb[p & 1];
        uint32_t* so = Sb[p & 1];
        hipLaunchKernelGGL(k_part_upsweep, dim3((unsigned)nblocks), dim3(kPartThreads), 0, st, sin, n, NB, shifts[p],
                           masks[p], blockhist, nblocks);
        if ((e = exclusive_scan_u32(blockhist, 256 * nblocks, sums, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_part_downsweep, dim3((unsigned)nblocks), dim3(kPartThreads), 0, st, kin, sin, ko, so, n,
                           NB, shifts[p], masks[p], p == 0 ? 1 : 0, is_f64 ? 1 : 0, blockhist, nblocks);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        kin = ko;
        sin = so;
    }
    *which = (passes - 1) & 1;
    return hipSuccess;
}

hipError_t launch_range_bounds(const uint32_t* d_sorted_slots, int64_t n, uint32_t NB, int64_t* d_start,
                               uint32_t* d_cnt, hipStream_t st) {
    int64_t m = (int64_t)NB + 2;
    hipLaunchKernelGGL(k_range_bounds, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, d_sorted_slots, n, NB,
                       d_start);
    hipLaunchKernelGGL(k_range_counts, dim3((unsigned)((NB + 255) / 256 + 1)), dim3(256), 0, st, d_start, NB, d_cnt);
    return hipGetLastError();
}

hipError_t launch_check_slots(const uint32_t* d_slots, int64_t n, int64_t S, uint64_t* d_bad, hipStream_t st) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_check_slots, dim3((unsigned)blocks), dim3(256), 0, st, d_slots, n, S,
                       (unsigned long long*)d_bad);
    return hipGetLastError();
}

hipError_t launch_big_chunks(const int32_t* d_bigbucket, int64_t big_count, const int64_t* d_start,
                             int64_t* d_chunk_pref, int64_t* d_gpref, hipStream_t st) {
    hipLaunchKernelGGL(k_big_chunks, dim3(1), dim3(64), 0, st, d_bigbucket, big_count, d_start, d_chunk_pref, d_gpref);
    return hipGetLastError();
}

hipError_t launch_big_gather(const int32_t* d_bigbucket, int64_t big_count, int64_t nchunks,
                             const int64_t* d_chunk_pref, const int64_t* d_gpref, const int64_t* d_start,
                             const uint64_t* d_K, const uint32_t* d_S, uint32_t* d_hist, uint64_t* d_G,
                             hipStream_t st) {
    if (nchunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_big_gather, dim3((unsigned)nchunks), dim3(256), 0, st, d_bigbucket, big_count, d_chunk_pref,
                       d_gpref, d_start, d_K, d_S, d_hist, d_G);
    return hipGetLastError();
}

hipError_t launch_copy_u64(const uint64_t* d_in, uint64_t* d_out, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_copy_u64, dim3((unsigned)blocks), dim3(256), 0, st, d_in, d_out, n);
    return hipGetLastError();
}

}  // namespace nns
