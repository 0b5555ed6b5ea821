// Sorting and polish phases on slot-range buckets (Sec. 2, Procedure NN-sort
// and polish).
//
// Every round of the sorting phase stores, for each slot, the first key (in
// processing order) that maps to it; the rest go to the conflict array and are
// mapped again.  Since f is fixed, a key keeps its slot in every round, so a
// slot's keys never interact with another slot's: the rounds of the keys of
// one slot range can run on their own.  k_bucket_polish runs all rounds of one
// range in LDS (first arrival = smallest input index, decided with LDS
// atomic-min), lays the arrays o_r out slot by slot (o_1, o_2, ... then the
// range's part of the last conflict array), and polishes that nearly sorted
// sequence in LDS: sorting networks on 8-key tiles, then merges of
// neighbouring tiles only while a tile boundary is out of order.
// Adjacent ranges can overlap in key order where f is not monotone or jitters;
// k_boundary_* repairs each such overlap with an in-place merge, and reports a
// fallback when the overlap is not confined to neighbours.
#include "nnsort_internal.h"

namespace nns {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}
__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

static int blocks_for(int64_t n, int threads, int cap) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

hipError_t fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n, 256, 8192)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}
hipError_t fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(n, 256, 8192)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

__device__ __forceinline__ uint64_t load_key(const void* M, bool M_is_bits, bool is_f64, int64_t i) {
    uint64_t v = ((const uint64_t*)M)[i];
    return M_is_bits ? order_key(v, is_f64) : v;
}
__device__ __forceinline__ void store_key(void* M, bool M_is_bits, bool is_f64, int64_t i, uint64_t k) {
    ((uint64_t*)M)[i] = M_is_bits ? order_key_inverse(k, is_f64) : k;
}

// ---------------------------------------------------------------------------
// classify: small / big buckets, offsets of small segments, segment list
// ---------------------------------------------------------------------------
// Single workgroup; each thread owns a contiguous chunk of buckets.
// bucket_info layout (int64 each): bigmap[NB] (id of big bucket or -1),
// moff[NB] (offset of the segment in M), seglist[NB] (non-empty small buckets
// in order), bigbucket[big_max] (bucket of big id).
__global__ void __launch_bounds__(1024) k_classify(const uint32_t* __restrict__ cnt, int64_t NB,
                                                   int64_t big_max, int32_t* bigmap, uint64_t* moff,
                                                   int32_t* seglist, int32_t* bigbucket,
                                                   unsigned long long* counters) {
    __shared__ unsigned long long s_small[1024], s_big[1024], s_seg[1024], s_bigkeys[1024];
    int t = threadIdx.x;
    int64_t chunk = (NB + 1023) / 1024;
    int64_t b0 = t * chunk, b1 = b0 + chunk < NB ? b0 + chunk : NB;
    unsigned long long small = 0, big = 0, seg = 0, bigkeys = 0;
    for (int64_t b = b0; b < b1; ++b) {
        uint32_t c = cnt[b];
        if (c > kBucketCap) {
            ++big;
            bigkeys += c;
        } else {
            small += c;
            seg += c ? 1 : 0;
        }
    }
    s_small[t] = small;
    s_big[t] = big;
    s_seg[t] = seg;
    s_bigkeys[t] = bigkeys;
    __syncthreads();
    // inclusive Hillis-Steele scans over 1024 entries
    for (int off = 1; off < 1024; off <<= 1) {
        unsigned long long a = t >= off ? s_small[t - off] : 0;
        unsigned long long c = t >= off ? s_big[t - off] : 0;
        unsigned long long d = t >= off ? s_seg[t - off] : 0;
        unsigned long long e = t >= off ? s_bigkeys[t - off] : 0;
        __syncthreads();
        s_small[t] += a;
        s_big[t] += c;
        s_seg[t] += d;
        s_bigkeys[t] += e;
        __syncthreads();
    }
    unsigned long long po = s_small[t] - small, pb = s_big[t] - big, ps = s_seg[t] - seg;
    for (int64_t b = b0; b < b1; ++b) {
        uint32_t c = cnt[b];
        if (c > kBucketCap) {
            bigmap[b] = (int32_t)pb;
            if ((int64_t)pb < big_max) bigbucket[pb] = (int32_t)b;
            ++pb;
            moff[b] = po;
        } else {
            bigmap[b] = -1;
            moff[b] = po;
            po += c;
            if (c) seglist[ps++] = (int32_t)b;
        }
    }
    if (t == 1023) {
        counters[kCntBigBuckets] = s_big[1023];
        counters[kCntBigKeys] = s_bigkeys[1023];
        counters[kCntSmallBuckets] = s_seg[1023];
    }
}

hipError_t launch_classify(const uint32_t* d_cnt, int64_t NB, int64_t big_max, int32_t* d_bigmap,
                           uint64_t* d_moff, int32_t* d_seglist, int32_t* d_bigbucket,
                           uint64_t* d_counters, hipStream_t st) {
    hipLaunchKernelGGL(k_classify, dim3(1), dim3(1024), 0, st, d_cnt, NB, big_max, d_bigmap, d_moff,
                       d_seglist, d_bigbucket, (unsigned long long*)d_counters);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// big buckets: round counts from the slot multiplicities
// ---------------------------------------------------------------------------
// Round counts of big buckets from slot multiplicities k_s: round r stores
// min(k_s, r) - min(k_s, r - 1) keys of slot s and leaves max(0, k_s - r).
__global__ void __launch_bounds__(256) k_big_counts(const uint32_t* __restrict__ hist, int64_t total, int eps,
                                                    unsigned long long* counters) {
    __shared__ unsigned long long s_col[NNSORT_MAX_EPS], s_pl[NNSORT_MAX_EPS];
    if (threadIdx.x < NNSORT_MAX_EPS) {
        s_col[threadIdx.x] = 0;
        s_pl[threadIdx.x] = 0;
    }
    __syncthreads();
    unsigned long long col[NNSORT_MAX_EPS] = {0}, pl[NNSORT_MAX_EPS] = {0};
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        uint32_t k = hist[i];
        for (int r = 1; r <= eps; ++r) {
            col[r - 1] += k > (uint32_t)r ? k - r : 0;
            pl[r - 1] += k >= (uint32_t)r ? 1 : 0;
        }
    }
    for (int r = 0; r < eps; ++r) {
        atomicAdd(&s_col[r], col[r]);
        atomicAdd(&s_pl[r], pl[r]);
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)eps) {
        atomicAdd(&counters[kCntCollided + threadIdx.x], s_col[threadIdx.x]);
        atomicAdd(&counters[kCntPlaced + threadIdx.x], s_pl[threadIdx.x]);
    }
}

hipError_t launch_big_counts(const uint32_t* d_hist, int64_t big_count, int eps, uint64_t* d_counters,
                             hipStream_t st) {
    if (big_count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_big_counts, dim3(blocks_for(big_count * kBucketSlots, 256, 2048)), dim3(256), 0, st,
                       d_hist, big_count * (int64_t)kBucketSlots, eps, (unsigned long long*)d_counters);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-bucket rounds + polish in LDS
// ---------------------------------------------------------------------------
constexpr int kItems = kItemsPerThread;  // region entries per thread (16)
constexpr int kTile = 8;                 // keys per polish tile
constexpr int kMaxTileRounds = 8;        // odd-even tile rounds before the bitonic fallback

__device__ __forceinline__ void cswap(uint64_t& a, uint64_t& b) {
    uint64_t lo = a < b ? a : b;
    uint64_t hi = a < b ? b : a;
    a = lo;
    b = hi;
}

// Batcher's odd-even merge sort network for 8 keys (19 comparators).
__device__ __forceinline__ void sort8(uint64_t (&v)[8]) {
    cswap(v[0], v[1]); cswap(v[2], v[3]); cswap(v[4], v[5]); cswap(v[6], v[7]);
    cswap(v[0], v[2]); cswap(v[1], v[3]); cswap(v[4], v[6]); cswap(v[5], v[7]);
    cswap(v[1], v[2]); cswap(v[5], v[6]);
    cswap(v[0], v[4]); cswap(v[1], v[5]); cswap(v[2], v[6]); cswap(v[3], v[7]);
    cswap(v[2], v[4]); cswap(v[3], v[5]);
    cswap(v[1], v[2]); cswap(v[3], v[4]); cswap(v[5], v[6]);
}

// Merge two ascending 8-key runs: reverse the second (a bitonic sequence of
// 16) and apply the half-cleaners at distances 8, 4, 2, 1.
__device__ __forceinline__ void merge16(uint64_t (&v)[16]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        uint64_t t = v[8 + i];
        v[8 + i] = v[15 - i];
        v[15 - i] = t;
    }
#pragma unroll
    for (int d = 8; d > 0; d >>= 1)
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if ((i & d) == 0) cswap(v[i], v[i | d]);
}

// Merge-path split: number of elements taken from a (length na) among the
// first `diag` outputs of merge(a, b); ties go to a first (stable).
__device__ __forceinline__ int merge_split(const uint64_t* a, int na, const uint64_t* b, int nb, int diag) {
    int lo = diag > nb ? diag - nb : 0;
    int hi = diag < na ? diag : na;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] <= b[diag - 1 - mid]) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

struct BucketSmem {
    uint64_t keys[kBucketCap];
    uint32_t owner[kBucketSlots];  // rounds: first arrival per slot; then residue cursors
    uint32_t off[kBucketSlots];    // keys per slot, then their exclusive prefix
    uint32_t wsum[kBucketThreads];
    unsigned long long red[2 * NNSORT_MAX_EPS];
    int flag;
};

// One workgroup per slot range.  Steps, all in LDS:
//  1. slot multiplicities k_s and the rounds: in round r each slot keeps the
//     unplaced key with the smallest input index (its r-th arrival);
//  2. round counts from k_s: round r stores #{s : k_s >= r} keys and leaves
//     sum_s max(0, k_s - r) in the conflict array;
//  3. compaction, slot-major: slot s's keys at offset(s), ordered o_1, o_2, ...,
//     o_eps, then the slot's share of the last conflict array -- the arrays
//     o_r interleaved slot by slot, which a near-monotone f leaves nearly
//     sorted;
//  4. polish: 8-key tiles sorted by a network, then odd-even merges of
//     neighbouring tiles while any tile boundary is out of order (keys only
//     move as far as f misplaced them); a bitonic sort if that does not settle.
__global__ void __launch_bounds__(kBucketThreads) k_bucket_polish(
    const uint32_t* __restrict__ cnt_arr, const int64_t* __restrict__ start, const uint64_t* __restrict__ moff,
    const uint64_t* __restrict__ K, const uint32_t* __restrict__ Sl, int eps, void* M, int M_is_bits, int is_f64,
    uint64_t* segmin, uint64_t* segmax, unsigned long long* counters) {
    __shared__ BucketSmem sm;
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x;
    const uint32_t cnt = cnt_arr[b];
    if (cnt == 0 || cnt > kBucketCap) return;  // empty, or handled by the dense-range path
    // the range's keys, in input order (the partition is stable): position e
    // in the range is the processing order used for first arrival
    const uint64_t* rk = K + start[b];
    const uint32_t* rs = Sl + start[b];

    uint64_t key[kItems];
    uint32_t idx[kItems];
    uint32_t lsl[kItems];
    uint8_t rnd[kItems];  // round that stored the key (0 = still in conflict array)
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        uint32_t e = tid + k * kBucketThreads;
        rnd[k] = 0;
        key[k] = 0;
        idx[k] = 0;
        lsl[k] = 0;
        if (e < cnt) {
            key[k] = rk[e];
            idx[k] = e;
            lsl[k] = rs[e] & (kBucketSlots - 1);
        }
    }
    for (int i = tid; i < (int)kBucketSlots; i += kBucketThreads) sm.off[i] = 0;
    if (tid < 2 * NNSORT_MAX_EPS) sm.red[tid] = 0;
    if (tid == 0) sm.flag = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kItems; ++k)
        if (tid + k * kBucketThreads < cnt) atomicAdd(&sm.off[lsl[k]], 1u);

    // ---- 1. rounds ----
    for (int r = 1; r <= eps; ++r) {
        for (int i = tid; i < (int)kBucketSlots; i += kBucketThreads) sm.owner[i] = kUnmapped;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kItems; ++k)
            if (tid + k * kBucketThreads < cnt && rnd[k] == 0) atomicMin(&sm.owner[lsl[k]], idx[k]);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kItems; ++k)
            if (tid + k * kBucketThreads < cnt && rnd[k] == 0 && sm.owner[lsl[k]] == idx[k]) rnd[k] = (uint8_t)r;
        __syncthreads();
    }

    // ---- 2. round counts from slot multiplicities; 3a. slot offsets ----
    constexpr int kSlotsPer = kBucketSlots / kBucketThreads;  // 8
    uint32_t ks[kSlotsPer], run = 0;
    {
        unsigned long long pl[NNSORT_MAX_EPS] = {0}, co[NNSORT_MAX_EPS] = {0};
#pragma unroll
        for (int q = 0; q < kSlotsPer; ++q) {
            ks[q] = sm.off[tid * kSlotsPer + q];
            run += ks[q];
            for (int r = 1; r <= eps; ++r) {
                pl[r - 1] += ks[q] >= (uint32_t)r ? 1u : 0u;
                co[r - 1] += ks[q] > (uint32_t)r ? ks[q] - r : 0u;
            }
        }
        for (int r = 0; r < eps; ++r) {
            if (pl[r]) atomicAdd(&sm.red[r], pl[r]);
            if (co[r]) atomicAdd(&sm.red[NNSORT_MAX_EPS + r], co[r]);
        }
        sm.wsum[tid] = run;
    }
    for (int i = tid; i < (int)kBucketSlots; i += kBucketThreads) sm.owner[i] = 0;  // residue cursors
    __syncthreads();
    if (tid < eps) {
        atomicAdd(&counters[kCntPlaced + tid], sm.red[tid]);
        atomicAdd(&counters[kCntCollided + tid], sm.red[NNSORT_MAX_EPS + tid]);
    }
    // exclusive scan of the 256 per-thread slot totals (Hillis-Steele in place)
    for (int o = 1; o < kBucketThreads; o <<= 1) {
        uint32_t y = tid >= o ? sm.wsum[tid - o] : 0;
        __syncthreads();
        sm.wsum[tid] += y;
        __syncthreads();
    }
    {
        uint32_t base = sm.wsum[tid] - run;
#pragma unroll
        for (int q = 0; q < kSlotsPer; ++q) {
            sm.off[tid * kSlotsPer + q] = base;
            base += ks[q];
        }
    }
    __syncthreads();

    // ---- 3b. slot-major compaction ----
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (tid + k * kBucketThreads >= cnt) continue;
        uint32_t pos = sm.off[lsl[k]];
        pos += rnd[k] ? (uint32_t)(rnd[k] - 1) : (uint32_t)eps + atomicAdd(&sm.owner[lsl[k]], 1u);
        sm.keys[pos] = key[k];
    }
    const int ntiles = (int)((cnt + kTile - 1) / kTile);
    for (int i = (int)cnt + tid; i < ntiles * kTile; i += kBucketThreads) sm.keys[i] = ~0ull;
    __syncthreads();

    // ---- 4. polish ----
    for (int t = tid; t < ntiles; t += kBucketThreads) {
        uint64_t v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = sm.keys[t * 8 + q];
        sort8(v);
#pragma unroll
        for (int q = 0; q < 8; ++q) sm.keys[t * 8 + q] = v[q];
    }
    __syncthreads();
    bool settled = false;
    for (int round = 0; round <= kMaxTileRounds; ++round) {
        int bad = 0;
        for (int t = tid; t + 1 < ntiles; t += kBucketThreads)
            bad |= sm.keys[t * 8 + 7] > sm.keys[t * 8 + 8] ? 1 : 0;
        if (bad) sm.flag = round + 1;
        __syncthreads();
        int f = sm.flag;
        __syncthreads();
        if (f != round + 1) {
            settled = true;
            break;
        }
        if (round == kMaxTileRounds) break;
        const int parity = round & 1;
        for (int p = tid; 2 * p + parity + 1 < ntiles; p += kBucketThreads) {
            const int t0 = 2 * p + parity;
            uint64_t v[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = sm.keys[t0 * 8 + q];
            merge16(v);
#pragma unroll
            for (int q = 0; q < 16; ++q) sm.keys[t0 * 8 + q] = v[q];
        }
        __syncthreads();
    }
    if (!settled) {
        // f is far from monotone inside this range: bitonic sort of the range
        int npad = 8;
        while (npad < ntiles * 8) npad <<= 1;
        for (int i = ntiles * 8 + tid; i < npad; i += kBucketThreads) sm.keys[i] = ~0ull;
        __syncthreads();
        for (int kk = 2; kk <= npad; kk <<= 1) {
            for (int j = kk >> 1; j > 0; j >>= 1) {
                for (int i = tid; i < npad; i += kBucketThreads) {
                    int l = i ^ j;
                    if (l > i) {
                        uint64_t a = sm.keys[i], c = sm.keys[l];
                        bool up = (i & kk) == 0;
                        if ((a > c) == up) {
                            sm.keys[i] = c;
                            sm.keys[l] = a;
                        }
                    }
                }
                __syncthreads();
            }
        }
    }

    // ---- write the range's sorted keys to its segment of M ----
    const uint64_t off = moff[b];
    for (uint32_t i = tid; i < cnt; i += kBucketThreads) store_key(M, M_is_bits, is_f64, off + i, sm.keys[i]);
    if (tid == 0) {
        segmin[b] = sm.keys[0];
        segmax[b] = sm.keys[cnt - 1];
    }
}

hipError_t launch_bucket_polish(const uint32_t* d_cnt, const int64_t* d_start, const uint64_t* d_moff, int64_t NB,
                                const uint64_t* d_K, const uint32_t* d_S, int eps, void* d_M, bool M_is_bits,
                                bool is_f64, uint64_t* d_segmin, uint64_t* d_segmax, uint64_t* d_counters,
                                hipStream_t st) {
    if (NB <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bucket_polish, dim3((unsigned)NB), dim3(kBucketThreads), 0, st, d_cnt, d_start, d_moff, d_K,
                       d_S, eps, d_M, M_is_bits ? 1 : 0, is_f64 ? 1 : 0, d_segmin, d_segmax,
                       (unsigned long long*)d_counters);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// boundary fix-up between consecutive segments of M
// ---------------------------------------------------------------------------
constexpr int kZoneMax = 4096;  // keys a single boundary repair may hold in LDS

// zone[k] for the boundary between segment k and k+1: {start, tail, head}.
struct Zone {
    uint64_t start;
    uint32_t tail;
    uint32_t head;
};

// One thread per segment k: checks that overlaps involve neighbours only
// (max of segment k-1 <= min of segment k+1) and sizes the zone between k and
// k+1 by binary search in both sorted segments.
__global__ void __launch_bounds__(256) k_boundary_plan(const void* M, int M_is_bits, int is_f64,
                                                       const uint64_t* __restrict__ moff,
                                                       const uint32_t* __restrict__ cnt,
                                                       const int32_t* __restrict__ seglist, int64_t K,
                                                       const uint64_t* __restrict__ segmin,
                                                       const uint64_t* __restrict__ segmax, Zone* zones,
                                                       unsigned long long* counters) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    int32_t b = seglist[k];
    if (k > 0 && k + 1 < K) {
        if (segmax[seglist[k - 1]] > segmin[seglist[k + 1]]) atomicAdd(&counters[kCntFallback], 1ull);
    }
    Zone z{0, 0, 0};
    if (k + 1 < K) {
        int32_t b2 = seglist[k + 1];
        uint64_t mx = segmax[b], mn = segmin[b2];
        if (mx > mn) {
            // tail: keys of segment k greater than min of k+1
            int64_t s0 = moff[b], n0 = cnt[b];
            int64_t lo = 0, hi = n0;
            while (lo < hi) {
                int64_t mid = (lo + hi) >> 1;
                if (load_key(M, M_is_bits, is_f64, s0 + mid) > mn) hi = mid;
                else lo = mid + 1;
            }
            uint32_t tail = (uint32_t)(n0 - lo);
            // head: keys of segment k+1 less than max of k
            int64_t s1 = moff[b2], n1 = cnt[b2];
            lo = 0;
            hi = n1;
            while (lo < hi) {
                int64_t mid = (lo + hi) >> 1;
                if (load_key(M, M_is_bits, is_f64, s1 + mid) < mx) lo = mid + 1;
                else hi = mid;
            }
            uint32_t head = (uint32_t)lo;
            z.start = (uint64_t)(s0 + n0 - tail);
            z.tail = tail;
            z.head = head;
            atomicAdd(&counters[kCntBoundary], (unsigned long long)(tail + head));
            if (tail + head > (uint32_t)kZoneMax) atomicAdd(&counters[kCntFallback], 1ull);
        }
    }
    zones[k] = z;
}

// One workgroup per boundary: merge tail and head (adjacent in M) in place.
__global__ void __launch_bounds__(256) k_boundary_merge(void* M, int M_is_bits, int is_f64,
                                                        const Zone* __restrict__ zones, int64_t K) {
    __shared__ uint64_t buf[kZoneMax];
    int64_t k = blockIdx.x;
    if (k >= K) return;
    Zone z = zones[k];
    int total = (int)(z.tail + z.head);
    if (z.tail == 0 || z.head == 0 || total > kZoneMax) return;
    for (int i = threadIdx.x; i < total; i += blockDim.x) buf[i] = load_key(M, M_is_bits, is_f64, z.start + i);
    __syncthreads();
    const uint64_t* a = buf;
    const uint64_t* b = buf + z.tail;
    int na = z.tail, nb = z.head;
    int per = (total + blockDim.x - 1) / blockDim.x;
    int d0 = threadIdx.x * per;
    if (d0 < total) {
        int ia = merge_split(a, na, b, nb, d0);
        int ib = d0 - ia;
        int d1 = d0 + per < total ? d0 + per : total;
        for (int d = d0; d < d1; ++d) {
            bool takeA = ib >= nb || (ia < na && a[ia] <= b[ib]);
            uint64_t v = takeA ? a[ia] : b[ib];
            ia += takeA ? 1 : 0;
            ib += takeA ? 0 : 1;
            store_key(M, M_is_bits, is_f64, z.start + d, v);
        }
    }
}

hipError_t launch_boundary_plan(const void* d_M, bool M_is_bits, bool is_f64, const uint64_t* d_moff,
                                const uint32_t* d_cnt, const int32_t* d_seglist, int64_t K,
                                const uint64_t* d_segmin, const uint64_t* d_segmax, void* d_zones,
                                uint64_t* d_counters, hipStream_t st) {
    if (K <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_boundary_plan, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, st, d_M,
                       M_is_bits ? 1 : 0, is_f64 ? 1 : 0, d_moff, d_cnt, d_seglist, K, d_segmin,
                       d_segmax, (Zone*)d_zones, (unsigned long long*)d_counters);
    return hipGetLastError();
}

hipError_t launch_boundary_merge(void* d_M, bool M_is_bits, bool is_f64, const void* d_zones, int64_t K,
                                 hipStream_t st) {
    if (K <= 1) return hipSuccess;
    hipLaunchKernelGGL(k_boundary_merge, dim3((unsigned)(K - 1)), dim3(256), 0, st, d_M, M_is_bits ? 1 : 0,
                       is_f64 ? 1 : 0, (const Zone*)d_zones, K - 1);
    return hipGetLastError();
}

size_t zone_bytes() { return sizeof(Zone); }

}  // namespace nns
