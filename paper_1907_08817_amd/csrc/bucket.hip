// Sorting and polish phases on slot ranges (Sec. 2, Procedure NN-sort and
// polish).
//
// Every round of the sorting phase stores, for each slot, the first key to
// arrive there; the rest go to the conflict array and are mapped again.  f is
// fixed, so a key keeps its slot in every round: the keys of one slot never
// interact with another slot's, and the rounds of one slot range can run on
// their own.  k_bucket_polish takes one range (at most kBucketCap keys) into
// LDS and:
//  - counts the keys of each slot with LDS atomics; the value an atomic
//    returns is the key's arrival rank in its slot, so rank r - 1 < eps is
//    the key stored by round r (o_r), and ranks >= eps form the slot's share
//    of the last conflict array.  Round counts follow from the multiplicities
//    k_s: round r stores #{s : k_s >= r} keys and leaves sum_s max(0, k_s - r);
//  - lays the range out slot by slot (o_1 .. o_eps entries, then the residue
//    of each slot) and orders each slot's few keys: this merges the arrays o_r
//    and the residue slot by slot, and is the final order wherever f is
//    monotone;
//  - checks for descents, which appear only where f's rounding jitters
//    between neighbouring slots; such a range is repaired by merges of
//    neighbouring 8-key tiles, or re-sorted whole.
// The output position of every range is known from the partition, so each
// range writes its keys straight to their final place.  Ranges too dense for
// LDS and keys with no slot go to a conventional sort (the residue path:
// segsort.hip range by range, radix.hip for keys with no slot).
// k_boundary_* then checks every pair of neighbouring ranges and
// repairs overlaps (where f is not monotone across a range boundary) with an
// in-place merge, or reports a fallback to a full sort.
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

// ---------------------------------------------------------------------------
// classify: non-empty ranges in order, and the ranges too dense for LDS
// ---------------------------------------------------------------------------
// Three passes over blocks of 256 ranges: per-block counts, an exclusive scan
// of those counts, and the ordered write of both lists.
__device__ __forceinline__ uint32_t below_in_wave(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Ranges of more than kHalfCap keys (and at most kBucketCap) are polished by
// the larger-LDS variant, from a list.
constexpr uint32_t kHalfCap = kBucketCap / 2;
constexpr int kClsQ = 4;  // per block: non-empty, dense, dense keys, half-full

// Also stores each range's key count, cnt[b] = start[b + 1] - start[b].
__global__ void __launch_bounds__(256) k_cls_count(const int64_t* __restrict__ start, int64_t NB, uint32_t* cnt,
                                                   unsigned long long* bsum, unsigned long long* counters) {
    __shared__ unsigned long long s[kClsQ][4];
    __shared__ uint32_t s_max[4];
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const uint32_t c = b < NB ? (uint32_t)(start[b + 1] - start[b]) : 0;
    if (b < NB) cnt[b] = c;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    unsigned long long ne = __popcll(__ballot(c != 0));
    unsigned long long bg = __popcll(__ballot(c > kBucketCap));
    unsigned long long md = __popcll(__ballot(c > kHalfCap && c <= kBucketCap));
    unsigned long long bk = c > kBucketCap ? c : 0;
    uint32_t mx = c > kBucketCap ? c : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        bk += __shfl_xor(bk, o);
        const uint32_t y = __shfl_xor(mx, o);
        mx = y > mx ? y : mx;
    }
    if (lane == 0) {
        s[0][w] = ne;
        s[1][w] = bg;
        s[2][w] = bk;
        s[3][w] = md;
        s_max[w] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t m01 = s_max[0] > s_max[1] ? s_max[0] : s_max[1];
        const uint32_t m23 = s_max[2] > s_max[3] ? s_max[2] : s_max[3];
        const uint32_t m = m01 > m23 ? m01 : m23;
        if (m) atomicMax(&counters[kCntBigMax], (unsigned long long)m);
    }
    if (threadIdx.x < kClsQ)
        bsum[blockIdx.x * kClsQ + threadIdx.x] =
            s[threadIdx.x][0] + s[threadIdx.x][1] + s[threadIdx.x][2] + s[threadIdx.x][3];
}

// Exclusive scan of the per-block counts (in place); totals to the counters,
// with the first position of the keys without a slot (start[NB]), so that one
// copy brings everything the host needs.
__global__ void __launch_bounds__(256) k_cls_scan(unsigned long long* bsum, int64_t nblk,
                                                  const int64_t* __restrict__ start, int64_t NB,
                                                  unsigned long long* counters) {
    __shared__ unsigned long long s[kClsQ][256];
    const int t = threadIdx.x;
    const int64_t per = (nblk + 255) / 256;
    const int64_t b0 = t * per, b1 = b0 + per < nblk ? b0 + per : nblk;
    unsigned long long tot[kClsQ] = {0, 0, 0, 0};
    for (int64_t i = b0; i < b1; ++i)
        for (int q = 0; q < kClsQ; ++q) tot[q] += bsum[i * kClsQ + q];
    for (int q = 0; q < kClsQ; ++q) s[q][t] = tot[q];
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        unsigned long long y[kClsQ];
        for (int q = 0; q < kClsQ; ++q) y[q] = t >= off ? s[q][t - off] : 0;
        __syncthreads();
        for (int q = 0; q < kClsQ; ++q) s[q][t] += y[q];
        __syncthreads();
    }
    unsigned long long run[kClsQ];
    for (int q = 0; q < kClsQ; ++q) run[q] = s[q][t] - tot[q];
    for (int64_t i = b0; i < b1; ++i)
        for (int q = 0; q < kClsQ; ++q) {
            unsigned long long v = bsum[i * kClsQ + q];
            bsum[i * kClsQ + q] = run[q];
            run[q] += v;
        }
    if (t == 0) counters[kCntFirstUnmapped] = (unsigned long long)start[NB];
    if (t == 255) {
        counters[kCntSegments] = s[0][255];
        counters[kCntBigBuckets] = s[1][255];
        counters[kCntBigKeys] = s[2][255];
        counters[kCntHalfFull] = s[3][255];
    }
}

__global__ void __launch_bounds__(256) k_cls_write(const uint32_t* __restrict__ cnt, int64_t NB, int64_t big_max,
                                                   const unsigned long long* __restrict__ bsum, int32_t* seglist,
                                                   int32_t* bigbucket, int32_t* halflist) {
    __shared__ uint32_t s[3][4];
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const uint32_t c = b < NB ? cnt[b] : 0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const bool half = c > kHalfCap && c <= kBucketCap;
    const unsigned long long mne = __ballot(c != 0), mbg = __ballot(c > kBucketCap), mhf = __ballot(half);
    if (lane == 0) {
        s[0][w] = (uint32_t)__popcll(mne);
        s[1][w] = (uint32_t)__popcll(mbg);
        s[2][w] = (uint32_t)__popcll(mhf);
    }
    __syncthreads();
    unsigned long long pne = bsum[blockIdx.x * kClsQ + 0] + below_in_wave(mne);
    unsigned long long pbg = bsum[blockIdx.x * kClsQ + 1] + below_in_wave(mbg);
    unsigned long long phf = bsum[blockIdx.x * kClsQ + 3] + below_in_wave(mhf);
    for (int ww = 0; ww < w; ++ww) {
        pne += s[0][ww];
        pbg += s[1][ww];
        phf += s[2][ww];
    }
    if (c != 0) seglist[pne] = (int32_t)b;
    if (c > kBucketCap && (int64_t)pbg < big_max) bigbucket[pbg] = (int32_t)b;
    if (half) halflist[phf] = (int32_t)b;
}

size_t classify_ws_words(int64_t NB) { return (size_t)((NB + 255) / 256) * kClsQ; }

hipError_t launch_classify(const int64_t* d_start, uint32_t* d_cnt, int64_t NB, int64_t big_max, int32_t* d_seglist,
                           int32_t* d_bigbucket, int32_t* d_halflist, uint64_t* d_bsum, uint64_t* d_counters,
                           hipStream_t st) {
    const int64_t nblk = (NB + 255) / 256;
    unsigned long long* bs = (unsigned long long*)d_bsum;
    hipLaunchKernelGGL(k_cls_count, dim3((unsigned)nblk), dim3(256), 0, st, d_start, NB, d_cnt, bs,
                       (unsigned long long*)d_counters);
    hipLaunchKernelGGL(k_cls_scan, dim3(1), dim3(256), 0, st, bs, nblk, d_start, NB, (unsigned long long*)d_counters);
    hipLaunchKernelGGL(k_cls_write, dim3((unsigned)nblk), dim3(256), 0, st, d_cnt, NB, big_max, bs, d_seglist,
                       d_bigbucket, d_halflist);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// round counts from slot multiplicities
// ---------------------------------------------------------------------------
// Dense ranges: k_s from their slot histograms.  Round r stores
// min(k_s, r) - min(k_s, r - 1) keys of slot s and leaves max(0, k_s - r).
// Sum of v over the workgroup's threads, one value per wave combined in LDS.
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__global__ void __launch_bounds__(256) k_big_counts(const uint32_t* __restrict__ hist, int64_t total, int eps,
                                                    unsigned long long* counters) {
    __shared__ unsigned long long s_w[4][2 * NNSORT_MAX_EPS];
    unsigned long long col[NNSORT_MAX_EPS] = {0}, pl[NNSORT_MAX_EPS] = {0};
    auto add = [&](uint32_t k) {
#pragma unroll
        for (int r = 1; r <= NNSORT_MAX_EPS; ++r) {
            if (r > eps) break;
            col[r - 1] += k > (uint32_t)r ? k - r : 0;
            pl[r - 1] += k >= (uint32_t)r ? 1 : 0;
        }
    };
    // eight independent loads in flight per thread: few workgroups, so few
    // atomics on the 2 eps shared counters at the end
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 7 * stride < total; i += 8 * stride) {
        uint32_t k[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) k[q] = hist[i + q * stride];
#pragma unroll
        for (int q = 0; q < 8; ++q) add(k[q]);
    }
    for (; i < total; i += stride) add(hist[i]);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < NNSORT_MAX_EPS; ++r) {
        if (r >= eps) break;
        const unsigned long long a = wave_sum(col[r]), b = wave_sum(pl[r]);
        if (lane == 0) {
            s_w[w][r] = a;
            s_w[w][NNSORT_MAX_EPS + r] = b;
        }
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)eps) {
        const int r = threadIdx.x;
        const unsigned long long a = s_w[0][r] + s_w[1][r] + s_w[2][r] + s_w[3][r];
        const int q = NNSORT_MAX_EPS + r;
        const unsigned long long b = s_w[0][q] + s_w[1][q] + s_w[2][q] + s_w[3][q];
        if (a) atomicAdd(&counters[kCntCollided + r], a);
        if (b) atomicAdd(&counters[kCntPlaced + r], b);
    }
}

hipError_t launch_big_counts(const uint32_t* d_hist, int64_t big_count, int eps, uint64_t* d_counters,
                             hipStream_t st) {
    if (big_count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_big_counts, dim3(blocks_for(big_count * kBucketSlots, 256 * 8, 2048)), dim3(256), 0, st,
                       d_hist, big_count * (int64_t)kBucketSlots, eps, (unsigned long long*)d_counters);
    return hipGetLastError();
}

// Small ranges: each polish workgroup leaves its per-round counts in
// part[b * kPartStride + r] (stored) and [.. + NNSORT_MAX_EPS + r]
// (conflict); summed here instead of with contended global atomics.
constexpr int kPartStride = 2 * NNSORT_MAX_EPS;

__global__ void __launch_bounds__(256) k_sum_parts(const uint32_t* __restrict__ part, const uint32_t* __restrict__ cnt,
                                                   int64_t NB, int eps, unsigned long long* counters) {
    __shared__ unsigned long long s_w[4][kPartStride];
    unsigned long long acc[kPartStride] = {0};
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < NB; b += stride) {
        uint32_t c = cnt[b];
        if (c == 0 || c > kBucketCap) continue;
        for (int r = 0; r < eps; ++r) {
            acc[r] += part[b * kPartStride + r];
            acc[NNSORT_MAX_EPS + r] += part[b * kPartStride + NNSORT_MAX_EPS + r];
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < NNSORT_MAX_EPS; ++r) {
        if (r >= eps) break;
        const unsigned long long a = wave_sum(acc[r]), b = wave_sum(acc[NNSORT_MAX_EPS + r]);
        if (lane == 0) {
            s_w[w][r] = a;
            s_w[w][NNSORT_MAX_EPS + r] = b;
        }
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)eps) {
        const int r = threadIdx.x;
        const unsigned long long a = s_w[0][r] + s_w[1][r] + s_w[2][r] + s_w[3][r];
        const int q = NNSORT_MAX_EPS + r;
        const unsigned long long b = s_w[0][q] + s_w[1][q] + s_w[2][q] + s_w[3][q];
        if (a) atomicAdd(&counters[kCntPlaced + r], a);
        if (b) atomicAdd(&counters[kCntCollided + r], b);
    }
}

size_t polish_part_words(int64_t NB) { return (size_t)NB * kPartStride; }

// ---------------------------------------------------------------------------
// per-range rounds + polish in LDS
// ---------------------------------------------------------------------------
constexpr int kTile = 8;                 // keys per repair tile
constexpr int kMaxTileRounds = 8;        // odd-even tile rounds before the whole-range re-sort
constexpr uint32_t kGroupMax = 32;       // larger slot groups are ordered by the whole-range re-sort
// keys of a slot group compared per step: with about 0.8 keys per slot, 99%
// of keys are in groups of at most 4
constexpr int kGroupStep = 4;

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

template <int CAP, int NT>
struct BucketSmem {
    uint64_t keys[CAP];
    // per slot, 16 bits: its key count, then its first position; slot 2w in
    // the low half of word w, slot 2w + 1 in the high half
    uint32_t off[kBucketSlots / 2];
    uint32_t wsum[NT / 64];
    uint32_t red[(NT / 64) * NNSORT_MAX_EPS];  // per-wave stored counts per round
    int flag;
};

__device__ __forceinline__ uint32_t half_of(uint32_t word, uint32_t s) { return (word >> ((s & 1u) * 16u)) & 0xFFFFu; }

// Sort of a whole range in LDS, in place: the CAP = 8 NT keys (the range
// padded with the largest key) are sorted 8 per thread by the network above,
// then merged in rounds of doubling run length.  In a round each thread finds
// by merge path where its 8 outputs begin in the two runs it merges, merges
// them into registers, and writes them back after a barrier: 9 rounds for
// 4096 keys, against 78 barrier-separated stages of a bitonic sort.
//
// Between the first and the last write the keys sit in a swizzled layout
// (key i at swz(i)), so that threads reading or writing 8 consecutive keys
// start in different LDS banks; the range leaves in the plain layout.
__device__ __forceinline__ int swz(int i) { return i ^ ((i >> 4) & 15); }

__device__ __forceinline__ int merge_split_swz(const uint64_t* s, int pa, int na, int pb, int nb, int diag) {
    int lo = diag > nb ? diag - nb : 0;
    int hi = diag < na ? diag : na;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (s[swz(pa + mid)] <= s[swz(pb + diag - 1 - mid)]) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <int CAP, int NT>
__device__ void sort_range(BucketSmem<CAP, NT>& sm, uint32_t cnt, int tid) {
    static_assert(CAP == 8 * NT && CAP > 8 && CAP % 16 == 0, "8 keys per thread, at least one merge round");
    for (int i = (int)cnt + tid; i < CAP; i += NT) sm.keys[i] = ~0ull;
    __syncthreads();
    const int pos = 8 * tid;
    uint64_t v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = sm.keys[pos + q];
    sort8(v);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) sm.keys[swz(pos + q)] = v[q];
    __syncthreads();
    for (int w = 8; w < CAP; w <<= 1) {
        const int base = pos & ~(2 * w - 1);  // the pair of runs [base, base + w), [base + w, base + 2w)
        const int pb = base + w;
        const int d = pos - base;
        int i = merge_split_swz(sm.keys, base, w, pb, w, d);
        int j = d - i;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            // ties to A, as merge_split counts them; an exhausted run is not read
            const bool take_a = j >= w || (i < w && sm.keys[swz(base + i)] <= sm.keys[swz(pb + j)]);
            v[q] = take_a ? sm.keys[swz(base + i)] : sm.keys[swz(pb + j)];
            i += take_a ? 1 : 0;
            j += take_a ? 0 : 1;
        }
        __syncthreads();
        const bool last = 2 * w >= CAP;
#pragma unroll
        for (int q = 0; q < 8; ++q) sm.keys[last ? pos + q : swz(pos + q)] = v[q];
        __syncthreads();
    }
}

// Repair of a range whose slot-ordered layout has descents: sorting networks
// on 8-key tiles, odd-even merges of neighbouring tiles while any tile
// boundary is out of order (keys only move as far as f misplaced them), and a
// sort of the whole range if that does not settle.  Returns true if the
// whole-range sort ran.
template <int CAP, int NT>
__device__ bool repair_range(BucketSmem<CAP, NT>& sm, uint32_t cnt, int tid) {
    const int ntiles = (int)((cnt + kTile - 1) / kTile);
    for (int i = (int)cnt + tid; i < ntiles * kTile; i += NT) sm.keys[i] = ~0ull;
    __syncthreads();
    for (int t = tid; t < ntiles; t += NT) {
        uint64_t v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = sm.keys[t * 8 + q];
        sort8(v);
#pragma unroll
        for (int q = 0; q < 8; ++q) sm.keys[t * 8 + q] = v[q];
    }
    __syncthreads();
    for (int round = 0; round <= kMaxTileRounds; ++round) {
        int bad = 0;
        for (int t = tid; t + 1 < ntiles; t += NT)
            bad |= sm.keys[t * 8 + 7] > sm.keys[t * 8 + 8] ? 1 : 0;
        if (bad) sm.flag = round + 2;
        __syncthreads();
        int f = sm.flag;
        __syncthreads();
        if (f != round + 2) return false;
        if (round == kMaxTileRounds) break;
        const int parity = round & 1;
        for (int p = tid; 2 * p + parity + 1 < ntiles; p += NT) {
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
    // f is far from monotone inside this range: sort the whole range
    sort_range(sm, cnt, tid);
    return true;
}

// One workgroup per slot range with LO < count <= CAP keys (CAP a power of
// two; the LDS a workgroup needs grows with CAP, so ranges of up to half the
// capacity run in a variant with twice as many workgroups per CU).  K / Sl: the
// range-partitioned order keys and slots (range b at [start[b], start[b+1]));
// the range's keys are written as bit patterns to out[base + start[b] ...],
// where base, the number of keys without a slot that sort before every mapped
// key, is read from the counters (so the launch needs no value the host has
// not yet read back).
template <int CAP, int LO, int NT>
__global__ void __launch_bounds__(NT, CAP <= 2048 ? 7 : 4) k_bucket_polish(
    const int64_t* __restrict__ start, const int32_t* __restrict__ list, const uint64_t* __restrict__ K,
    const uint32_t* __restrict__ Sl, int eps, uint64_t* __restrict__ out, int is_f64, uint32_t* __restrict__ part,
    unsigned long long* counters) {
    constexpr int kItems = CAP / NT;
    constexpr int kSlotsPer = kBucketSlots / NT;  // slots owned per thread
    __shared__ BucketSmem<CAP, NT> sm;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int64_t b = list ? list[blockIdx.x] : blockIdx.x;
    const int64_t s0 = start[b];
    const uint32_t cnt = (uint32_t)(start[b + 1] - s0);
    if (cnt <= (uint32_t)LO || cnt > (uint32_t)CAP) return;  // another variant's, or the dense-range path's
    const uint64_t* rk = K + s0;
    const uint32_t* rs = Sl + s0;
    const int64_t base = (int64_t)counters[kCntUnmappedNeg];

    uint64_t key[kItems];
    uint32_t sl[kItems];
    uint32_t rank[kItems];
    // every load issued before any is used: no branches between them (items
    // past cnt read the range's last key again and are never used)
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const uint32_t e = tid + k * NT;
        const uint32_t ec = e < cnt ? e : cnt - 1;
        key[k] = rk[ec];
        sl[k] = rs[ec];
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) sl[k] &= kBucketSlots - 1;
    for (int i = tid; i < (int)kBucketSlots / 2; i += NT) sm.off[i] = 0;
    if (tid == 0) sm.flag = 0;
    __syncthreads();
    // arrival rank of each key in its slot
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (k * NT >= (int)cnt) break;
        if (tid + k * NT < cnt) {
            const uint32_t old = atomicAdd(&sm.off[sl[k] >> 1], 1u << ((sl[k] & 1u) * 16u));
            rank[k] = half_of(old, sl[k]);
        }
    }
    __syncthreads();

    // round counts from the multiplicities: round r stores #{s : k_s >= r}
    // keys (wave totals by ballot); the conflict array after round r holds
    // cnt - sum_{j <= r} stored_j.  Slot offsets by an exclusive scan.
    uint32_t ks[kSlotsPer], run = 0;
    {
        bool big_group = false;
#pragma unroll
        for (int q = 0; q < kSlotsPer / 2; ++q) {
            const uint32_t w = sm.off[tid * (kSlotsPer / 2) + q];
            ks[2 * q] = w & 0xFFFFu;
            ks[2 * q + 1] = w >> 16;
        }
        uint32_t wpl[NNSORT_MAX_EPS] = {0};
#pragma unroll
        for (int q = 0; q < kSlotsPer; ++q) {
            run += ks[q];
            big_group |= ks[q] > kGroupMax;
#pragma unroll
            for (int r = 1; r <= NNSORT_MAX_EPS; ++r) {
                if (r > eps) break;
                wpl[r - 1] += (uint32_t)__popcll(__ballot(ks[q] >= (uint32_t)r));
            }
        }
        if (lane == 0) {
            for (int r = 0; r < eps; ++r) sm.red[wv * NNSORT_MAX_EPS + r] = wpl[r];
        }
        if (__ballot(big_group) && lane == 0) sm.flag = 1;
    }
    uint32_t inc = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == 63) sm.wsum[wv] = inc;
    __syncthreads();
    {
        uint32_t pos = inc - run;
        for (int w = 0; w < wv; ++w) pos += sm.wsum[w];
#pragma unroll
        for (int q = 0; q < kSlotsPer / 2; ++q) {
            const uint32_t lo = pos;
            const uint32_t hi = pos + ks[2 * q];
            pos = hi + ks[2 * q + 1];
            sm.off[tid * (kSlotsPer / 2) + q] = lo | (hi << 16);
        }
    }
    if (tid < eps) {
        uint32_t stored = 0, cum = 0;
        for (int r = 0; r <= tid; ++r) {
            uint32_t p = 0;
            for (int w = 0; w < NT / 64; ++w) p += sm.red[w * NNSORT_MAX_EPS + r];
            cum += p;
            stored = p;
        }
        part[b * kPartStride + tid] = stored;
        part[b * kPartStride + NNSORT_MAX_EPS + tid] = cnt - cum;
    }
    __syncthreads();

    // slot-major layout: a slot's keys at its offset, in arrival order
    uint32_t g0[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (k * NT >= (int)cnt) break;
        if (tid + k * NT < cnt) {
            g0[k] = half_of(sm.off[sl[k] >> 1], sl[k]);
            sm.keys[g0[k] + rank[k]] = key[k];
        }
    }
    __syncthreads();

    // a slot group of more than kGroupMax keys: the slot-major layout is
    // sorted whole at once (tile merges would take many rounds to settle it)
    const bool big_group = sm.flag != 0;
    bool need_repair = big_group;
    if (!need_repair) {
        // a key's place inside its slot: its rank among the slot's keys by
        // (key, arrival); groups hold about one key on average
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            if (k * NT >= (int)cnt) break;
            if (tid + k * NT < cnt) {
                const uint32_t s = sl[k];
                const uint32_t g1 = s + 1 < kBucketSlots ? half_of(sm.off[(s + 1) >> 1], s + 1) : cnt;
                const uint64_t me = key[k];
                const uint32_t mine = g0[k] + rank[k];
                uint32_t pos = g0[k];
                for (uint32_t j0 = g0[k]; j0 < g1; j0 += kGroupStep) {
                    uint64_t y[kGroupStep];
#pragma unroll
                    for (int q = 0; q < kGroupStep; ++q) y[q] = j0 + q < g1 ? sm.keys[j0 + q] : ~0ull;
#pragma unroll
                    for (int q = 0; q < kGroupStep; ++q)
                        pos += (y[q] < me || (y[q] == me && j0 + q < mine)) ? 1u : 0u;
                }
                rank[k] = pos;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            if (k * NT >= (int)cnt) break;
            if (tid + k * NT < cnt) sm.keys[rank[k]] = key[k];
        }
        __syncthreads();
        // written out while checked for descents, which remain only where
        // f's slots jitter between neighbours (such a range is repaired and
        // written again below)
        int bad = 0;
        uint64_t* o = out + base + s0;
        for (uint32_t i = tid; i < cnt; i += NT) {
            const uint64_t v = sm.keys[i];
            if (i + 1 < cnt) bad |= v > sm.keys[i + 1] ? 1 : 0;
            o[i] = order_key_inverse(v, is_f64);
        }
        if (bad) sm.flag = 1;
        __syncthreads();
        need_repair = sm.flag != 0;
    }
    if (need_repair) {
        bool whole = true;
        if (big_group)
            sort_range(sm, cnt, tid);
        else
            whole = repair_range(sm, cnt, tid);
        if (whole && tid == 0) atomicAdd(&counters[kCntResorted], 1ull);
        // write the range's sorted keys to their final place
        uint64_t* o = out + base + s0;
        for (uint32_t i = tid; i < cnt; i += NT) o[i] = order_key_inverse(sm.keys[i], is_f64);
    }
}

// Ranges of at most kHalfCap keys: one workgroup per range id (others exit
// at once).
hipError_t launch_polish_small(const int64_t* d_start, int64_t NB, const uint64_t* d_K, const uint32_t* d_S, int eps,
                               uint64_t* d_out, bool is_f64, uint32_t* d_part, uint64_t* d_counters, hipStream_t st) {
    if (NB <= 0) return hipSuccess;
    static_assert(kBucketCap == 2 * kHalfCap && kHalfCap == 2048, "polish variants");
    hipLaunchKernelGGL((k_bucket_polish<2048, 0, kBucketThreads>), dim3((unsigned)NB), dim3(kBucketThreads), 0, st, d_start,
                       nullptr, d_K, d_S, eps, d_out, is_f64 ? 1 : 0, d_part, (unsigned long long*)d_counters);
    return hipGetLastError();
}

// The n_half ranges listed in d_halflist: the full-capacity variant, with
// twice the threads (its workgroups are few, so each one's latency counts).
constexpr int kHalfThreads = 512;
hipError_t launch_polish_half(const int64_t* d_start, const int32_t* d_halflist, int64_t n_half, const uint64_t* d_K,
                              const uint32_t* d_S, int eps, uint64_t* d_out, bool is_f64, uint32_t* d_part,
                              uint64_t* d_counters, hipStream_t st) {
    if (n_half <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_bucket_polish<4096, 2048, kHalfThreads>), dim3((unsigned)n_half), dim3(kHalfThreads), 0, st, d_start,
                       d_halflist, d_K, d_S, eps, d_out, is_f64 ? 1 : 0, d_part, (unsigned long long*)d_counters);
    return hipGetLastError();
}

// The ranges' round counts into the counters (after both variants).
hipError_t launch_sum_parts(const uint32_t* d_part, const uint32_t* d_cnt, int64_t NB, int eps, uint64_t* d_counters,
                            hipStream_t st) {
    if (NB <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sum_parts, dim3(blocks_for(NB, 256, 256)), dim3(256), 0, st, d_part, d_cnt, NB, eps,
                       (unsigned long long*)d_counters);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// boundaries between neighbouring ranges, in the output
// ---------------------------------------------------------------------------
constexpr int kZoneMax = 4096;

struct Zone {
    uint64_t start;
    uint32_t tail;
    uint32_t head;
};

__device__ __forceinline__ uint64_t out_key(const uint64_t* out, bool is_f64, int64_t i) {
    return order_key(out[i], is_f64);
}

// One thread per non-empty range k (in range order; every range is sorted in
// place at out[base + start[b]]): checks that overlaps involve neighbours
// only (max of range k-1 <= min of range k+1) and sizes the zone between k
// and k+1 by binary search in both.
__global__ void __launch_bounds__(256) k_boundary_plan(const uint64_t* __restrict__ out, int is_f64, int64_t base,
                                                       const int64_t* __restrict__ start,
                                                       const int32_t* __restrict__ seglist, int64_t K, Zone* zones,
                                                       unsigned long long* counters) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const int32_t b = seglist[k];
    const int64_t s0 = base + start[b], n0 = start[b + 1] - start[b];
    if (k > 0 && k + 1 < K) {
        const int32_t bp = seglist[k - 1], bn = seglist[k + 1];
        if (out_key(out, is_f64, base + start[bp + 1] - 1) > out_key(out, is_f64, base + start[bn]))
            atomicAdd(&counters[kCntFallback], 1ull);
    }
    Zone z{0, 0, 0};
    if (k + 1 < K) {
        const int32_t b2 = seglist[k + 1];
        const int64_t s1 = base + start[b2], n1 = start[b2 + 1] - start[b2];
        const uint64_t mx = out_key(out, is_f64, s0 + n0 - 1), mn = out_key(out, is_f64, s1);
        if (mx > mn) {
            // tail: keys of range k greater than the min of k+1
            int64_t lo = 0, hi = n0;
            while (lo < hi) {
                int64_t mid = (lo + hi) >> 1;
                if (out_key(out, is_f64, s0 + mid) > mn) hi = mid;
                else lo = mid + 1;
            }
            const uint32_t tail = (uint32_t)(n0 - lo);
            // head: keys of range k+1 less than the max of k
            lo = 0;
            hi = n1;
            while (lo < hi) {
                int64_t mid = (lo + hi) >> 1;
                if (out_key(out, is_f64, s1 + mid) < mx) lo = mid + 1;
                else hi = mid;
            }
            const uint32_t head = (uint32_t)lo;
            z.start = (uint64_t)(s0 + n0 - tail);
            z.tail = tail;
            z.head = head;
            atomicAdd(&counters[kCntBoundary], (unsigned long long)(tail + head));
            if (tail + head > (uint32_t)kZoneMax) atomicAdd(&counters[kCntFallback], 1ull);
        }
    }
    zones[k] = z;
}

// Boundaries kMergeSpan at a time per workgroup: its threads look at one
// zone each, the non-empty zones (usually none) are listed in LDS, and the
// workgroup merges each one's tail and head (adjacent in out) in place.
// Skipped whole when the plan reported a fallback (zones may then overlap);
// the host sorts the whole output instead.
constexpr int kMergeSpan = 256;

__global__ void __launch_bounds__(kMergeSpan) k_boundary_merge(uint64_t* out, int is_f64,
                                                               const Zone* __restrict__ zones, int64_t K,
                                                               const unsigned long long* __restrict__ counters) {
    __shared__ uint64_t buf[kZoneMax];
    __shared__ int s_list[kMergeSpan];
    __shared__ int s_n;
    if (counters[kCntFallback] != 0) return;
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    {
        const int64_t k = (int64_t)blockIdx.x * kMergeSpan + threadIdx.x;
        if (k < K) {
            const Zone z = zones[k];
            if (z.tail != 0 && z.head != 0 && z.tail + z.head <= (uint32_t)kZoneMax)
                s_list[atomicAdd(&s_n, 1)] = (int)threadIdx.x;
        }
    }
    __syncthreads();
    const int nz = s_n;
    for (int e = 0; e < nz; ++e) {
        const Zone z = zones[(int64_t)blockIdx.x * kMergeSpan + s_list[e]];
        const int total = (int)(z.tail + z.head);
        for (int i = threadIdx.x; i < total; i += kMergeSpan) buf[i] = out_key(out, is_f64, z.start + i);
        __syncthreads();
        const uint64_t* a = buf;
        const uint64_t* b = buf + z.tail;
        const int na = z.tail, nb = z.head;
        const int per = (total + kMergeSpan - 1) / kMergeSpan;
        const int d0 = threadIdx.x * per;
        if (d0 < total) {
            int ia = merge_split(a, na, b, nb, d0);
            int ib = d0 - ia;
            const int d1 = d0 + per < total ? d0 + per : total;
            for (int d = d0; d < d1; ++d) {
                const bool takeA = ib >= nb || (ia < na && a[ia] <= b[ib]);
                const uint64_t v = takeA ? a[ia] : b[ib];
                ia += takeA ? 1 : 0;
                ib += takeA ? 0 : 1;
                out[z.start + d] = order_key_inverse(v, is_f64);
            }
        }
        __syncthreads();  // buf is refilled for the next zone
    }
}

// After the fix-up the output is a sequence of sorted blocks: the keys
// without a slot below the mapped ones, each range's keys outside any zone,
// each merged zone, the keys without a slot above the mapped ones.  It is
// sorted iff every junction between adjacent blocks is.  The plan's test
// (max of range k-1 <= min of range k+1) keeps zones from overlapping but does
// not cover zones that end up side by side, or keys without a slot that are
// not the extremes, so the junctions are checked here: one thread per range
// (its first key, and both ends of the zone after it), one more for the start
// of the keys without a slot above the mapped ones (at index back).  Nothing
// to check after a fallback (the whole output gets sorted), or when there
// was no zone and every key has a slot (the plan saw every pair of
// neighbouring ranges in order).
__global__ void __launch_bounds__(256) k_junction_check(const uint64_t* __restrict__ out, int is_f64, int64_t base,
                                                        const int64_t* __restrict__ start,
                                                        const int32_t* __restrict__ seglist, int64_t K,
                                                        const Zone* __restrict__ zones, int64_t n, int64_t back,
                                                        int unmapped, unsigned long long* counters) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k > K || counters[kCntFallback] != 0 || (counters[kCntBoundary] == 0 && !unmapped)) return;
    bool bad = false;
    if (k == K) {
        if (back > 0 && back < n) bad = out_key(out, is_f64, back - 1) > out_key(out, is_f64, back);
    } else {
        const int64_t p = base + start[seglist[k]];
        if (p > 0) bad = out_key(out, is_f64, p - 1) > out_key(out, is_f64, p);
        const Zone z = zones[k];
        if (z.tail != 0 && z.head != 0) {
            const int64_t zs = (int64_t)z.start, ze = zs + z.tail + z.head;
            if (zs > 0) bad |= out_key(out, is_f64, zs - 1) > out_key(out, is_f64, zs);
            if (ze < n) bad |= out_key(out, is_f64, ze - 1) > out_key(out, is_f64, ze);
        }
    }
    if (bad) atomicAdd(&counters[kCntJunction], 1ull);
}

hipError_t launch_junction_check(const uint64_t* d_out, bool is_f64, int64_t base, const int64_t* d_start,
                                 const int32_t* d_seglist, int64_t K, const void* d_zones, int64_t n, int64_t back,
                                 bool unmapped, uint64_t* d_counters, hipStream_t st) {
    hipLaunchKernelGGL(k_junction_check, dim3((unsigned)((K + 1 + 255) / 256)), dim3(256), 0, st, d_out,
                       is_f64 ? 1 : 0, base, d_start, d_seglist, K, (const Zone*)d_zones, n, back, unmapped ? 1 : 0,
                       (unsigned long long*)d_counters);
    return hipGetLastError();
}

hipError_t launch_boundary_plan(const uint64_t* d_out, bool is_f64, int64_t base, const int64_t* d_start,
                                const int32_t* d_seglist, int64_t K, void* d_zones, uint64_t* d_counters,
                                hipStream_t st) {
    if (K <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_boundary_plan, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, st, d_out,
                       is_f64 ? 1 : 0, base, d_start, d_seglist, K, (Zone*)d_zones, (unsigned long long*)d_counters);
    return hipGetLastError();
}

hipError_t launch_boundary_merge(uint64_t* d_out, bool is_f64, const void* d_zones, int64_t K,
                                const uint64_t* d_counters, hipStream_t st) {
    if (K <= 1) return hipSuccess;
    hipLaunchKernelGGL(k_boundary_merge, dim3((unsigned)((K - 1 + kMergeSpan - 1) / kMergeSpan)), dim3(kMergeSpan),
                       0, st, d_out, is_f64 ? 1 : 0, (const Zone*)d_zones, K - 1, (const unsigned long long*)d_counters);
    return hipGetLastError();
}

size_t zone_bytes() { return sizeof(Zone); }

}  // namespace nns
