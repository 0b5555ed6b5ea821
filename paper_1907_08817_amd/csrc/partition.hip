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

constexpr int kPartThreads = 512;
constexpr int kPartItems = kPartTile / kPartThreads;  // 16
constexpr int kPartWaves = kPartThreads / 64;

// Digit histogram of one kPartTile-key tile, stored as hist[tile * 256 + digit].
__global__ void __launch_bounds__(kPartThreads) k_part_upsweep(const uint32_t* __restrict__ slots, int64_t n,
                                                               uint32_t NB, int shift, uint32_t mask,
                                                               uint32_t* blockhist) {
    __shared__ uint32_t h[256];
    if (threadIdx.x < 256) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kPartTile;
    if (t0 + kPartTile <= n) {
        // full tile: 16-byte loads (the tile starts on a 16-byte boundary)
        const uint4* v = (const uint4*)(slots + t0);
#pragma unroll
        for (int k = 0; k < kPartTile / (4 * kPartThreads); ++k) {
            const uint4 q = v[k * kPartThreads + threadIdx.x];
            atomicAdd(&h[(range_of(q.x, NB) >> shift) & mask], 1u);
            atomicAdd(&h[(range_of(q.y, NB) >> shift) & mask], 1u);
            atomicAdd(&h[(range_of(q.z, NB) >> shift) & mask], 1u);
            atomicAdd(&h[(range_of(q.w, NB) >> shift) & mask], 1u);
        }
    } else {
        for (int64_t i = t0 + threadIdx.x; i < n; i += kPartThreads)
            atomicAdd(&h[(range_of(slots[i], NB) >> shift) & mask], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 256) blockhist[(int64_t)blockIdx.x * 256 + threadIdx.x] = h[threadIdx.x];
}

// Offsets from the tile histograms, in two coalesced passes.  Tiles are taken
// in chunks of kScanTiles: (1) per chunk and digit, the exclusive prefix over
// the chunk's tiles in place, and the chunk total; (2) per digit, the
// exclusive prefix over chunks plus the digit's start (all digits below it).
// A tile's output offset for digit d is then hist[t][d] + chunk[t / kScanTiles][d].
constexpr int kScanTiles = 128;

__global__ void __launch_bounds__(256) k_part_scan_chunks(uint32_t* hist, int64_t ntiles, uint32_t* chunk) {
    const int d = threadIdx.x;
    const int64_t t0 = (int64_t)blockIdx.x * kScanTiles;
    const int64_t t1 = t0 + kScanTiles < ntiles ? t0 + kScanTiles : ntiles;
    uint32_t run = 0;
    int64_t t = t0;
    for (; t + 8 <= t1; t += 8) {
        uint32_t v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = hist[(t + q) * 256 + d];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            hist[(t + q) * 256 + d] = run;
            run += v[q];
        }
    }
    for (; t < t1; ++t) {
        uint32_t v = hist[t * 256 + d];
        hist[t * 256 + d] = run;
        run += v;
    }
    chunk[(int64_t)blockIdx.x * 256 + d] = run;
}

// Per digit, the exclusive prefix over chunks plus the digit's start.  Four
// threads per digit, each over a quarter of the chunks, so that many loads
// are in flight.
__global__ void __launch_bounds__(1024) k_part_scan_top(uint32_t* chunk, int64_t nchunks) {
    __shared__ uint32_t s_q[4][256];
    __shared__ uint32_t s_base[256];
    __shared__ uint32_t wtot[4];
    const int t = threadIdx.x;
    const int d = t & 255, q = t >> 8;
    const int64_t per = (nchunks + 3) / 4;
    const int64_t c0 = q * per, c1 = c0 + per < nchunks ? c0 + per : nchunks;
    uint32_t tot = 0;
#pragma unroll 16
    for (int64_t c = c0; c < c1; ++c) tot += chunk[c * 256 + d];
    s_q[q][d] = tot;
    __syncthreads();
    uint32_t pre = 0, all = 0;
    for (int qq = 0; qq < 4; ++qq) {
        const uint32_t v = s_q[qq][d];
        pre += qq < q ? v : 0;
        all += v;
    }
    if (q == 0) {
        // start of digit d = sum of the totals of digits below it
        const int lane = d & 63, w = d >> 6;
        uint32_t inc = all;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t y = __shfl_up(inc, o);
            if (lane >= o) inc += y;
        }
        if (lane == 63) wtot[w] = inc;
        s_base[d] = inc - all;
    }
    __syncthreads();
    uint32_t run = s_base[d] + pre;
    for (int ww = 0; ww < (d >> 6); ++ww) run += wtot[ww];
    int64_t c = c0;
    for (; c + 8 <= c1; c += 8) {
        uint32_t v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = chunk[(c + k) * 256 + d];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            chunk[(c + k) * 256 + d] = run;
            run += v[k];
        }
    }
    for (; c < c1; ++c) {
        uint32_t v = chunk[c * 256 + d];
        chunk[c * 256 + d] = run;
        run += v;
    }
}

// Tile handled by workgroup `bid`.  Workgroups are dealt to the 8 XCDs in turn
// (workgroup i on XCD i mod 8), so XCD x is given the x-th contiguous eighth
// of the tiles: the runs that consecutive tiles write for one digit are then
// adjacent in memory and meet in the same L2 before they are written back.
__device__ __forceinline__ int64_t xcd_tile(int64_t bid, int64_t ntiles) {
    const int64_t q = ntiles >> 3, r = ntiles & 7;
    const int64_t x = bid & 7, j = bid >> 3;
    return x * q + (x < r ? x : r) + j;
}

__device__ __forceinline__ uint32_t lanes_below(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Scatter of (key, slot) pairs by one digit of the range id.  in_bits: keys
// arrive as caller bit patterns (first pass) and leave as order keys.
//
// STABLE (every pass after the first, as LSD grouping needs): a key's rank
// among the tile's keys of its digit follows input order -- within a wave by
// matching digits bit by bit with ballots, across waves by per-wave counters.
// The first pass need not be stable (only the last pass's order within a
// digit matters for grouping by range), so there one LDS atomic per key
// gives its rank.
//
// The tile is first reordered by digit in LDS, then written out by
// consecutive threads, so each digit's run of the tile (8 keys on average)
// leaves as a few full cache lines instead of 16 scattered 8-byte writes.
template <bool STABLE>
__global__ void __launch_bounds__(kPartThreads) k_part_downsweep(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ sin, uint64_t* __restrict__ kout,
    uint32_t* __restrict__ sout, int64_t n, uint32_t NB, int shift, uint32_t mask, int nbits, int in_bits,
    int is_f64, const uint32_t* __restrict__ hist, const uint32_t* __restrict__ chunk, int64_t nblocks) {
    // the rank counters are dead once every key knows its place in the tile,
    // so they share storage with the staged slots
    __shared__ uint64_t s_key[kPartTile];
    __shared__ union {
        uint32_t slot[kPartTile];
        uint32_t cnt[kPartWaves][256];
    } s_u;
    __shared__ uint32_t dstart[256];
    __shared__ uint32_t gofs[256];
    __shared__ uint32_t wtot[kPartWaves];
    const int lane = __lane_id();
    const int w = threadIdx.x >> 6;
    const int64_t tile = xcd_tile(blockIdx.x, nblocks);
    const int64_t tile0 = tile * kPartTile;
    const int lim = (int)(n - tile0 < kPartTile ? n - tile0 : kPartTile);
    for (int i = threadIdx.x; i < kPartWaves * 256; i += kPartThreads) (&s_u.cnt[0][0])[i] = 0;
    if (threadIdx.x < 256)
        gofs[threadIdx.x] = hist[tile * 256 + threadIdx.x] + chunk[(tile / kScanTiles) * 256 + threadIdx.x];
    __syncthreads();

    const uint64_t* __restrict__ kb = kin + tile0;
    const uint32_t* __restrict__ sb = sin + tile0;
    uint64_t key[kPartItems];
    uint32_t slot[kPartItems];
    uint32_t rank[kPartItems];
#pragma unroll
    for (int k = 0; k < kPartItems; ++k) {
        const int idx = w * (kPartItems * 64) + k * 64 + lane;
        const bool valid = idx < lim;
        const uint64_t v = valid ? kb[idx] : 0;
        key[k] = in_bits ? order_key(v, is_f64) : v;
        slot[k] = valid ? sb[idx] : 0;
        const uint32_t d = (range_of(slot[k], NB) >> shift) & mask;
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
                for (int ww = 0; ww < kPartWaves; ++ww) tot += s_u.cnt[ww][d];
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
                for (int ww = 0; ww < kPartWaves; ++ww) {
                    uint32_t c = s_u.cnt[ww][d];
                    s_u.cnt[ww][d] = run;
                    run += c;
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPartItems; ++k) {
        const int idx = w * (kPartItems * 64) + k * 64 + lane;
        if (idx < lim) {
            const uint32_t d = (range_of(slot[k], NB) >> shift) & mask;
            rank[k] += STABLE ? s_u.cnt[w][d] : dstart[d];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPartItems; ++k) {
        const int idx = w * (kPartItems * 64) + k * 64 + lane;
        if (idx < lim) {
            s_key[rank[k]] = key[k];
            s_u.slot[rank[k]] = slot[k];
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < lim; i += kPartThreads) {
        const uint32_t sl = s_u.slot[i];
        const uint32_t d = (range_of(sl, NB) >> shift) & mask;
        const uint32_t pos = gofs[d] + (uint32_t)i - dstart[d];
        kout[pos] = s_key[i];
        sout[pos] = sl;
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
    if (chunk >= chunk_pref[big_count]) return;  // the grid is an upper bound
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

// After the residue sort, G in order is: keys without a slot whose order key
// has the top bit clear (negative NaN, -inf), then the dense ranges' keys,
// then the other keys without a slot.  Where f is monotone across ranges the
// middle part is the dense ranges one after another, so range id's slice
// G[u_neg + gpref[id] ...] goes to its place out[u_neg + start[b] ...]; the
// boundary check that follows catches any overlap.
__global__ void __launch_bounds__(256) k_big_place(const int32_t* __restrict__ bigbucket, int64_t big_count,
                                                   const int64_t* __restrict__ chunk_pref,
                                                   const int64_t* __restrict__ gpref,
                                                   const int64_t* __restrict__ start, const uint64_t* __restrict__ Gs,
                                                   int64_t u_neg, uint64_t* __restrict__ out, int is_f64) {
    const int64_t chunk = blockIdx.x;
    if (chunk >= chunk_pref[big_count]) return;  // the grid is an upper bound
    int64_t lo = 0, hi = big_count - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (chunk_pref[mid] <= chunk) lo = mid;
        else hi = mid - 1;
    }
    const int64_t id = lo;
    const int32_t b = bigbucket[id];
    const int64_t len = start[b + 1] - start[b];
    const int64_t c0 = (chunk - chunk_pref[id]) * kChunk;
    const int64_t c1 = c0 + kChunk < len ? c0 + kChunk : len;
    const uint64_t* src = Gs + u_neg + gpref[id];
    uint64_t* dst = out + u_neg + start[b];
    for (int64_t e = c0 + threadIdx.x; e < c1; e += blockDim.x) dst[e] = order_key_inverse(src[e], is_f64);
}

// Keys without a slot whose order key has the top bit clear.
__global__ void __launch_bounds__(256) k_count_neg(const uint64_t* __restrict__ K, const int64_t* __restrict__ start,
                                                   uint32_t NB, int64_t n, unsigned long long* count) {
    const int64_t s0 = start[NB];
    unsigned long long c = 0;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = s0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        c += (K[i] >> 63) ? 0 : 1;
    if (c) atomicAdd(count, c);
}

__global__ void __launch_bounds__(256) k_copy_u64(const uint64_t* __restrict__ in, uint64_t* out, int64_t n) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = in[i];
}

// ---- host-side launch sequence ----

int range_passes(uint32_t NB, int* shifts, uint32_t* masks, int* widths) {
    int bits = 1;
    while (bits < 32 && ((uint64_t)NB >> bits) != 0) ++bits;  // range ids 0..NB
    int passes = (bits + 7) / 8;
    int per = (bits + passes - 1) / passes;
    for (int p = 0; p < passes; ++p) {
        shifts[p] = p * per;
        int w = bits - p * per < per ? bits - p * per : per;
        masks[p] = (1u << w) - 1u;
        widths[p] = w;
    }
    return passes;
}

// Tile histograms followed by the chunk offsets.
size_t partition_hist_words(int64_t n) {
    int64_t nblocks = (n + kPartTile - 1) / kPartTile;
    if (nblocks < 1) nblocks = 1;
    int64_t nchunks = (nblocks + kScanTiles - 1) / kScanTiles;
    return (size_t)256 * (nblocks + nchunks);
}

// Partition (keys, slots) by range id.  in_keys are caller bit patterns;
// result in (K[res], S[res]) as order keys; returns res via *which.
hipError_t partition_by_range(const uint64_t* in_keys, const uint32_t* in_slots, int64_t n, uint32_t NB, bool is_f64,
                              uint64_t* K0, uint32_t* S0, uint64_t* K1, uint32_t* S1, uint32_t* blockhist,
                              int* which, hipStream_t st) {
    int shifts[4], widths[4];
    uint32_t masks[4];
    int passes = range_passes(NB, shifts, masks, widths);
    const int64_t nblocks = (n + kPartTile - 1) / kPartTile;
    const int64_t nchunks = (nblocks + kScanTiles - 1) / kScanTiles;
    uint32_t* chunk = blockhist + 256 * nblocks;
    uint64_t* Kb[2] = {K0, K1};
    uint32_t* Sb[2] = {S0, S1};
    const uint64_t* kin = in_keys;
    const uint32_t* sin = in_slots;
    hipError_t e;
    for (int p = 0; p < passes; ++p) {
        uint64_t* ko = Kb[p & 1];
        uint32_t* so = Sb[p & 1];
        hipLaunchKernelGGL(k_part_upsweep, dim3((unsigned)nblocks), dim3(kPartThreads), 0, st, sin, n, NB, shifts[p],
                           masks[p], blockhist);
        hipLaunchKernelGGL(k_part_scan_chunks, dim3((unsigned)nchunks), dim3(256), 0, st, blockhist, nblocks, chunk);
        hipLaunchKernelGGL(k_part_scan_top, dim3(1), dim3(1024), 0, st, chunk, nchunks);
        if (p == 0)
            hipLaunchKernelGGL(k_part_downsweep<false>, dim3((unsigned)nblocks), dim3(kPartThreads), 0, st, kin, sin,
                               ko, so, n, NB, shifts[p], masks[p], widths[p], 1, is_f64 ? 1 : 0, blockhist, chunk,
                               nblocks);
        else
            hipLaunchKernelGGL(k_part_downsweep<true>, dim3((unsigned)nblocks), dim3(kPartThreads), 0, st, kin, sin,
                               ko, so, n, NB, shifts[p], masks[p], widths[p], 0, is_f64 ? 1 : 0, blockhist, chunk,
                               nblocks);
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

hipError_t launch_big_place(const int32_t* d_bigbucket, int64_t big_count, int64_t nchunks,
                            const int64_t* d_chunk_pref, const int64_t* d_gpref, const int64_t* d_start,
                            const uint64_t* d_Gs, int64_t u_neg, uint64_t* d_out, bool is_f64, hipStream_t st) {
    if (nchunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_big_place, dim3((unsigned)nchunks), dim3(256), 0, st, d_bigbucket, big_count, d_chunk_pref,
                       d_gpref, d_start, d_Gs, u_neg, d_out, is_f64 ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_count_neg(const uint64_t* d_K, const int64_t* d_start, uint32_t NB, int64_t n, uint64_t* d_count,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_count_neg, dim3(64), dim3(256), 0, st, d_K, d_start, NB, n, (unsigned long long*)d_count);
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
