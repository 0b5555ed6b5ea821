// Hand-off of keys to slot ranges (Sec. 2, Sorting Phase: each key goes to the
// slot its predicted position names).  Keys and their slots are grouped by
// slot range with LSD passes on the range id (lsd.h): digit histograms per
// tile, one exclusive scan over (digit, tile), and a scatter staged in LDS.
// No per-key device atomics: MI355X's 8 XCDs keep separate L2s, and a
// device-wide counter per range would serialise the scatter.  Then the range
// bounds, and the gather of ranges too dense for one workgroup's LDS.
#include "lsd.h"

namespace nns {

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
// slot: a dense range's slot multiplicities are counted in LDS per chunk and
// added to its histogram, for the round counts; its keys are copied to G when
// the whole residue is radix-sorted there (ranges sorted one by one stay in
// the partition output).

// chunk_pref[i] = number of chunks of big ranges 0..i-1, gpref[i] = keys of
// big ranges 0..i-1 (i = 0..big_count): one workgroup of NT threads, each
// summing PER consecutive ranges, then a scan of the threads' totals by wave
// shuffles (one barrier per NT * PER ranges).  One range per thread of 256
// while that covers them all, eight per thread of 1024 beyond.
template <int NT, int PER>
__global__ void __launch_bounds__(NT) k_big_chunks(const int32_t* __restrict__ bigbucket, int64_t big_count,
                                                   const int64_t* __restrict__ start, int64_t* chunk_pref,
                                                   int64_t* gpref) {
    constexpr int kWaves = NT / 64;
    __shared__ int64_t s_c[kWaves], s_g[kWaves];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t cbase = 0, gbase = 0;
    for (int64_t i0 = 0; i0 < big_count; i0 += (int64_t)NT * PER) {
        const int64_t first = i0 + (int64_t)threadIdx.x * PER;
        int64_t len[PER];
        int64_t tc = 0, tg = 0;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            len[q] = 0;
            if (first + q < big_count) {
                const int32_t b = bigbucket[first + q];
                len[q] = start[b + 1] - start[b];
            }
            tc += (len[q] + kBigChunk - 1) / kBigChunk;
            tg += len[q];
        }
        int64_t ic = tc, ig = tg;  // inclusive scan over the wave
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t yc = __shfl_up(ic, o), yg = __shfl_up(ig, o);
            if (lane >= o) {
                ic += yc;
                ig += yg;
            }
        }
        if (lane == 63) {
            s_c[w] = ic;
            s_g[w] = ig;
        }
        __syncthreads();
        int64_t rc = cbase + ic - tc, rg = gbase + ig - tg, allc = 0, allg = 0;
#pragma unroll
        for (int ww = 0; ww < kWaves; ++ww) {
            if (ww < w) {
                rc += s_c[ww];
                rg += s_g[ww];
            }
            allc += s_c[ww];
            allg += s_g[ww];
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            if (first + q < big_count) {
                chunk_pref[first + q] = rc;
                gpref[first + q] = rg;
            }
            rc += (len[q] + kBigChunk - 1) / kBigChunk;
            rg += len[q];
        }
        cbase += allc;
        gbase += allg;
        __syncthreads();  // s_c, s_g are rewritten by the next group
    }
    if (threadIdx.x == 0) {
        chunk_pref[big_count] = cbase;
        gpref[big_count] = gbase;
    }
}

// One workgroup per `per` consecutive chunks: the LDS histogram of a
// range's slots is added to the range's global histogram once per range met,
// not once per chunk (a chunk holds 4096 keys over 2048 slots, so a flush per
// chunk costs about as many global atomics as it has keys).  `per` stays 1
// until there are enough chunks for 2048 workgroups, and is at most
// kGatherChunks.
constexpr int kGatherChunks = 8;

__global__ void __launch_bounds__(256) k_big_gather(const int32_t* __restrict__ bigbucket, int64_t big_count,
                                                    const int64_t* __restrict__ chunk_pref,
                                                    const int64_t* __restrict__ gpref,
                                                    const int64_t* __restrict__ start,
                                                    const uint64_t* __restrict__ K, const uint32_t* __restrict__ Sl,
                                                    uint32_t* hist, uint64_t* G, int per) {
    __shared__ uint32_t h[kBucketSlots];
    const int64_t total = chunk_pref[big_count];
    const int64_t first = (int64_t)blockIdx.x * per;
    if (first >= total) return;  // the grid is an upper bound
    const int64_t last = first + per < total ? first + per : total;
    // big range of the first chunk: last i with chunk_pref[i] <= first
    int64_t lo = 0, hi = big_count - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (chunk_pref[mid] <= first) lo = mid;
        else hi = mid - 1;
    }
    int64_t id = lo;
    for (int i = threadIdx.x; i < (int)kBucketSlots; i += blockDim.x) h[i] = 0;
    __syncthreads();
    for (int64_t chunk = first; chunk < last; ++chunk) {
        if (chunk >= chunk_pref[id + 1]) {  // a new range: flush the last one's counts (uniform branch)
            __syncthreads();
            for (int i = threadIdx.x; i < (int)kBucketSlots; i += blockDim.x)
                if (h[i]) {
                    atomicAdd(&hist[id * kBucketSlots + i], h[i]);
                    h[i] = 0;
                }
            __syncthreads();
            while (chunk >= chunk_pref[id + 1]) ++id;
        }
        const int32_t b = bigbucket[id];
        const int64_t s0 = start[b], len = start[b + 1] - s0;
        const int64_t c0 = (chunk - chunk_pref[id]) * kBigChunk;
        const int64_t c1 = c0 + kBigChunk < len ? c0 + kBigChunk : len;
        int64_t e = c0 + threadIdx.x;
        if (G) {
            for (; e < c1; e += blockDim.x) {
                G[gpref[id] + e] = K[s0 + e];
                atomicAdd(&h[Sl[s0 + e] & (kBucketSlots - 1)], 1u);
            }
        } else {  // the range is sorted where it is: slots only, four loads in flight
            for (; e + 3 * (int64_t)blockDim.x < c1; e += 4 * (int64_t)blockDim.x) {
                uint32_t v[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = Sl[s0 + e + q * (int64_t)blockDim.x];
#pragma unroll
                for (int q = 0; q < 4; ++q) atomicAdd(&h[v[q] & (kBucketSlots - 1)], 1u);
            }
            for (; e < c1; e += blockDim.x) atomicAdd(&h[Sl[s0 + e] & (kBucketSlots - 1)], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < (int)kBucketSlots; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[id * kBucketSlots + i], h[i]);
}

// Dense range id's sorted keys go to their place out[u_neg + start[b] ...]
// after the radix sort of the whole residue in G (ranges sorted one by one
// write their output themselves).  G in order is the keys without a slot
// whose order key has the top bit clear (negative NaN, -inf), then the dense
// ranges' keys, then the other keys without a slot.  Where f is monotone
// across ranges the middle part is the dense ranges one after another, so
// range id's slice is G[u_neg + gpref[id] ...]; the boundary check that
// follows catches any overlap.
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
    const int64_t c0 = (chunk - chunk_pref[id]) * kBigChunk;
    const int64_t c1 = c0 + kBigChunk < len ? c0 + kBigChunk : len;
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
    // the first passes take one bit fewer where the bits do not divide
    // evenly: fewer digits, longer runs per tile for the unstable first pass
    const int fewer = per * passes - bits;
    int shift = 0;
    for (int p = 0; p < passes; ++p) {
        const int w = per - (p < fewer ? 1 : 0);
        shifts[p] = shift;
        masks[p] = (1u << w) - 1u;
        widths[p] = w;
        shift += w;
    }
    return passes;
}

size_t partition_hist_words(int64_t n) { return lsd_hist_words(n); }

// Partition (keys, slots) by range id.  in_keys are caller bit patterns;
// result in (K[res], S[res]) as order keys; returns res via *which.
hipError_t partition_by_range(const uint64_t* in_keys, const uint32_t* in_slots, int64_t n, uint32_t NB, bool is_f64,
                              uint64_t* K0, uint32_t* S0, uint64_t* K1, uint32_t* S1, uint32_t* blockhist,
                              int* which, hipStream_t st, bool first_counted) {
    int shifts[4], widths[4];
    uint32_t masks[4];
    int passes = range_passes(NB, shifts, masks, widths);
    const int64_t ntiles = (n + kLsdTile - 1) / kLsdTile;
    const uint32_t* chunk = blockhist + 256 * ntiles;
    uint64_t* Kb[2] = {K0, K1};
    uint32_t* Sb[2] = {S0, S1};
    const uint64_t* kin = in_keys;
    const uint32_t* sin = in_slots;
    hipError_t e;
    for (int p = 0; p < passes; ++p) {
        uint64_t* ko = Kb[p & 1];
        uint32_t* so = Sb[p & 1];
        const RangeDigit dig{NB, shifts[p], masks[p]};
        const int im = p == 0 ? (is_f64 ? 1 : 2) : 0;
        if (p > 0 || !first_counted)  // else the map kernel counted the first pass's digits
            hipLaunchKernelGGL((k_lsd_upsweep<true, RangeDigit>), dim3((unsigned)ntiles), dim3(kLsdThreads), 0, st,
                               kin, sin, n, im, dig, blockhist);
        if ((e = launch_lsd_scan(blockhist, ntiles, st)) != hipSuccess) return e;
        if (p == 0)
            hipLaunchKernelGGL((k_lsd_downsweep<false, true, RangeDigit>), dim3((unsigned)ntiles), dim3(kLsdThreads),
                               0, st, kin, sin, ko, so, n, im, 0, dig, widths[p], blockhist, chunk, ntiles);
        else if (passes >= 3)
            hipLaunchKernelGGL((k_lsd_downsweep<true, true, RangeDigit, true>), dim3((unsigned)ntiles),
                               dim3(kLsdThreads), 0, st, kin, sin, ko, so, n, im, 0, dig, widths[p], blockhist, chunk,
                               ntiles);
        else
            hipLaunchKernelGGL((k_lsd_downsweep<true, true, RangeDigit>), dim3((unsigned)ntiles), dim3(kLsdThreads),
                               0, st, kin, sin, ko, so, n, im, 0, dig, widths[p], blockhist, chunk, ntiles);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        kin = ko;
        sin = so;
    }
    *which = (passes - 1) & 1;
    return hipSuccess;
}

hipError_t launch_range_bounds(const uint32_t* d_sorted_slots, int64_t n, uint32_t NB, int64_t* d_start,
                               hipStream_t st) {
    int64_t m = (int64_t)NB + 2;
    hipLaunchKernelGGL(k_range_bounds, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, d_sorted_slots, n, NB,
                       d_start);
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
    if (big_count <= 256)
        hipLaunchKernelGGL((k_big_chunks<256, 1>), dim3(1), dim3(256), 0, st, d_bigbucket, big_count, d_start,
                           d_chunk_pref, d_gpref);
    else
        hipLaunchKernelGGL((k_big_chunks<1024, 8>), dim3(1), dim3(1024), 0, st, d_bigbucket, big_count, d_start,
                           d_chunk_pref, d_gpref);
    return hipGetLastError();
}

hipError_t launch_big_gather(const int32_t* d_bigbucket, int64_t big_count, int64_t nchunks,
                             const int64_t* d_chunk_pref, const int64_t* d_gpref, const int64_t* d_start,
                             const uint64_t* d_K, const uint32_t* d_S, uint32_t* d_hist, uint64_t* d_G,
                             hipStream_t st) {
    if (nchunks <= 0) return hipSuccess;
    const int64_t per = std::min<int64_t>(kGatherChunks, std::max<int64_t>(1, nchunks / 2048));
    hipLaunchKernelGGL(k_big_gather, dim3((unsigned)((nchunks + per - 1) / per)), dim3(256), 0, st, d_bigbucket,
                       big_count, d_chunk_pref, d_gpref, d_start, d_K, d_S, d_hist, d_G, (int)per);
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
