// Sort of the dense ranges' keys, range by range (the conventional sort of
// the keys the LDS polish cannot hold; Sec. 2 sorts the last conflict array
// conventionally, and the dense ranges' keys are the part of it that this
// design routes here).  Segment id holds gpref[id + 1] - gpref[id] order keys
// starting at G[gpref[id]] (a compact buffer), or, when seg_range is given,
// at G[range_start[seg_range[id]]] (the range's own slice of the partition
// output, sorted in place); it is cut into chunks of kBigChunk keys
// (chunk_pref[id] = its first chunk).  Sorting each
// segment on its own gives every range exactly its own keys in order, the
// same state a small range reaches in LDS; the boundary check that follows
// treats both alike.
//
//  1. k_seg_sort_chunk: every run of run0 keys (one chunk, or two once the
//     dense keys are many) sorted in LDS (8 keys per thread by a sorting
//     network, then levels of merge path; one workgroup per run).
//  2. k_seg_merge, once per round r = 0, 1, ...: in every segment longer
//     than L = run0 2^r, the sorted runs of length L are merged in pairs
//     (merge path: each workgroup writes one chunk of output; a wave finds
//     where the chunk starts in the two runs by a 64-way search, then the
//     chunk's inputs are staged in LDS and every thread merges 16 outputs
//     into registers, which go back through LDS to be written out in
//     wave-contiguous order).  Round r reads one buffer and writes the other;
//     a segment that takes R rounds ends in buffer R mod 2 (G for even R).
// Where every thread reads or writes 8 or 16 consecutive keys in LDS, the
// index is swizzled (swz) so that neighbouring threads start in different
// banks.  Given an output (SegOut), the step that completes a segment (the
// run sort of a segment of at most one run, else its last merge round) writes
// it there as bit patterns instead of to the sort's buffers.
#include "nnsort_internal.h"

namespace nns {

constexpr int kMergeThreads = 256;
constexpr int kMergePer = kBigChunk / kMergeThreads;  // outputs per thread

// Segment of a chunk: the last id with chunk_pref[id] <= chunk.
__device__ __forceinline__ int64_t seg_of_chunk(const int64_t* __restrict__ chunk_pref, int64_t nseg,
                                                int64_t chunk) {
    int64_t lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (chunk_pref[mid] <= chunk) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Merge path, whole wave: the number of A's elements among the first d of
// the merge of sorted A[0, na) and B[0, nb) (ties from A first).  That is the
// first i in [max(0, d - nb), min(d, na)] where A[i] <= B[d - i - 1] fails;
// the predicate holds on a prefix, so 64 probes per step narrow the interval
// 65-fold.  Every probe index stays inside both arrays.
__device__ int64_t split_wave(const uint64_t* __restrict__ A, int64_t na, const uint64_t* __restrict__ B,
                              int64_t nb, int64_t d, int lane) {
    int64_t lo = d > nb ? d - nb : 0;
    int64_t hi = d < na ? d : na;
    while (hi > lo) {
        const int64_t w = hi - lo;
        if (w <= 64) {
            const bool p = lane < w && A[lo + lane] <= B[d - (lo + lane) - 1];
            return lo + __popcll(__ballot(p));
        }
        const int64_t m = lo + (w * (lane + 1)) / 65;  // lo <= m < hi, increasing in lane
        const int t = __popcll(__ballot(A[m] <= B[d - m - 1]));
        const int64_t nlo = t > 0 ? lo + (w * t) / 65 + 1 : lo;
        const int64_t nhi = t < 64 ? lo + (w * (t + 1)) / 65 : hi;
        lo = nlo;
        hi = nhi;
    }
    return lo;
}

// Same in LDS, one thread.
__device__ __forceinline__ int split_lds(const uint64_t* A, int na, const uint64_t* B, int nb, int d) {
    int lo = d > nb ? d - nb : 0;
    int hi = d < na ? d : na;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (A[mid] <= B[d - mid - 1]) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Block merge sort of one run of RUN keys (RUN / kBigChunk chunks, starting at
// a chunk whose index in its segment is a multiple of that).  Each thread
// sorts P keys in registers (P = 8: a 19-comparator network, Batcher's
// odd-even merge sort for 8 inputs; P = 16: that network on both halves, then
// a bitonic merge of the two); then runs of P, 2P, ..., RUN / 2 keys are
// merged in pairs in LDS: at every level a thread finds where its P outputs
// start in its pair of runs (merge path, ties from the left run) and merges
// them in registers.  Global memory is read and written in wave-contiguous
// order through LDS.  P = 16 for two-chunk runs (one LDS level fewer, and
// half as many merge-path searches; the runs are that long only when dense
// keys fill the GPU), 8 for one-chunk runs (twice the threads for few keys).
constexpr int kSortPerRun(int run) { return run >= 8192 ? 16 : 8; }

__device__ __forceinline__ void cswap(uint64_t& a, uint64_t& b) {
    const uint64_t lo = a < b ? a : b;
    b = a < b ? b : a;
    a = lo;
}

// LDS index of key i of a sorted run: the low four bits XORed with bits 4..7,
// a permutation within each 16-key row.  A thread's 8 consecutive keys
// (i = 8 t + r) then start in different banks for neighbouring threads, which
// the plain layout maps onto the same two banks.
__device__ __forceinline__ int swz(int i) { return i ^ ((i >> 4) & 15); }

// split_lds over runs held in swizzled LDS: A at s[swz(pa + i)], B at
// s[swz(pq + j)].
__device__ __forceinline__ int split_lds_swz(const uint64_t* s, int pa, int na, int pq, int nb, int d) {
    int lo = d > nb ? d - nb : 0;
    int hi = d < na ? d : na;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s[swz(pa + mid)] <= s[swz(pq + d - mid - 1)]) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// First key of segment id in G.
__device__ __forceinline__ int64_t seg_base(const int64_t* __restrict__ gpref, const int32_t* __restrict__ seg_range,
                                            const int64_t* __restrict__ range_start, int64_t id) {
    return seg_range ? range_start[seg_range[id]] : gpref[id];
}

template <int RUN, int kSortPer = kSortPerRun(RUN)>
__global__ void __launch_bounds__(RUN / kSortPer) k_seg_sort_chunk(const int64_t* __restrict__ chunk_pref,
                                                                  const int64_t* __restrict__ gpref, int64_t nseg,
                                                                  const int32_t* __restrict__ seg_range,
                                                                  const int64_t* __restrict__ range_start,
                                                                  uint64_t* G, SegOut fo) {
    constexpr int kThreads = RUN / kSortPer;
    constexpr int kChunksPerRun = RUN / kBigChunk;
    static_assert(RUN % kBigChunk == 0 && RUN <= 8192, "a run of whole chunks, in at most 64 KB of LDS");
    __shared__ uint64_t s[RUN];
    const int64_t chunk = blockIdx.x;
    if (chunk >= chunk_pref[nseg]) return;  // the grid is an upper bound
    const int64_t id = seg_of_chunk(chunk_pref, nseg, chunk);
    if ((chunk - chunk_pref[id]) % kChunksPerRun) return;  // sorted with the chunk before it
    const int64_t g0 = seg_base(gpref, seg_range, range_start, id), len = gpref[id + 1] - gpref[id];
    const int64_t c0 = (chunk - chunk_pref[id]) * kBigChunk;
    const int cnt = (int)(len - c0 < RUN ? len - c0 : RUN);
    uint64_t* p = G + g0 + c0;
    const int tid = threadIdx.x;
    // each thread loads its kSortPer consecutive keys straight into registers
    // (all loads in flight at once), padded with the largest order key: a
    // real key of that value is the same bit pattern, so the first cnt
    // outputs are right either way
    const int base = tid * kSortPer;
    uint64_t v[kSortPer];
#pragma unroll
    for (int r = 0; r < kSortPer; ++r) v[r] = base + r < cnt ? p[base + r] : ~0ull;
#pragma unroll
    for (int h = 0; h < kSortPer; h += 8) {
        cswap(v[h + 0], v[h + 2]); cswap(v[h + 1], v[h + 3]); cswap(v[h + 4], v[h + 6]); cswap(v[h + 5], v[h + 7]);
        cswap(v[h + 0], v[h + 4]); cswap(v[h + 1], v[h + 5]); cswap(v[h + 2], v[h + 6]); cswap(v[h + 3], v[h + 7]);
        cswap(v[h + 0], v[h + 1]); cswap(v[h + 2], v[h + 3]); cswap(v[h + 4], v[h + 5]); cswap(v[h + 6], v[h + 7]);
        cswap(v[h + 2], v[h + 4]); cswap(v[h + 3], v[h + 5]);
        cswap(v[h + 1], v[h + 4]); cswap(v[h + 3], v[h + 6]);
        cswap(v[h + 1], v[h + 2]); cswap(v[h + 3], v[h + 4]); cswap(v[h + 5], v[h + 6]);
    }
    if (kSortPer == 16) {
        // the two sorted halves as one bitonic sequence (second half
        // reversed), then half-cleaners at distances 8, 4, 2, 1
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint64_t t = v[8 + i];
            v[8 + i] = v[15 - i];
            v[15 - i] = t;
        }
#pragma unroll
        for (int dd = 8; dd > 0; dd >>= 1)
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if ((i & dd) == 0) cswap(v[i], v[i | dd]);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortPer; ++r) s[swz(base + r)] = v[r];
    __syncthreads();
    for (int run = kSortPer; run < RUN; run <<= 1) {
        const int pb = base & ~(2 * run - 1);  // this thread's pair of runs
        const int pa = pb, pq = pb + run;  // first keys of runs A and B
        const int d = base - pb;
        int ia = split_lds_swz(s, pa, run, pq, run, d);
        int ib = d - ia;
#pragma unroll
        for (int r = 0; r < kSortPer; ++r) {
            // both heads read in bounds (an exhausted run's last key, unused)
            const uint64_t a = s[swz(pa + (ia < run ? ia : run - 1))];
            const uint64_t b = s[swz(pq + (ib < run ? ib : run - 1))];
            const bool takeA = ib >= run || (ia < run && a <= b);
            v[r] = takeA ? a : b;
            ia += takeA ? 1 : 0;
            ib += takeA ? 0 : 1;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kSortPer; ++r) s[swz(base + r)] = v[r];
        __syncthreads();
    }
    if (fo.out && len <= RUN) {  // the whole segment: straight to its place in the output
        uint64_t* o = fo.out + fo.base + range_start[seg_range[id]];
        for (int i = tid; i < cnt; i += kThreads) o[i] = order_key_inverse(s[swz(i)], fo.is_f64 != 0);
    } else {
        for (int i = tid; i < cnt; i += kThreads) p[i] = s[swz(i)];
    }
}

__global__ void __launch_bounds__(kMergeThreads) k_seg_merge(const int64_t* __restrict__ chunk_pref,
                                                             const int64_t* __restrict__ gpref, int64_t nseg,
                                                             const int32_t* __restrict__ seg_range,
                                                             const int64_t* __restrict__ range_start,
                                                             int64_t L, const uint64_t* __restrict__ src,
                                                             uint64_t* __restrict__ dst, SegOut fo) {
    __shared__ uint64_t s[kBigChunk];
    __shared__ int64_t s_split[2];
    const int64_t chunk = blockIdx.x;
    if (chunk >= chunk_pref[nseg]) return;  // the grid is an upper bound
    const int64_t id = seg_of_chunk(chunk_pref, nseg, chunk);
    const int64_t g0 = seg_base(gpref, seg_range, range_start, id), len = gpref[id + 1] - gpref[id];
    if (len <= L) return;  // one run already: this segment is done
    const int64_t c0 = (chunk - chunk_pref[id]) * kBigChunk;
    const int64_t c1 = c0 + kBigChunk < len ? c0 + kBigChunk : len;
    const int64_t pb = (c0 / (2 * L)) * (2 * L);  // first output of this chunk's pair of runs
    const uint64_t* A = src + g0 + pb;
    const int64_t na = len - pb < L ? len - pb : L;
    const uint64_t* B = A + L;
    int64_t nb = len - pb - L;
    nb = nb < 0 ? 0 : (nb > L ? L : nb);
    // the round that completes the segment writes it to its place in the output
    const bool fin = fo.out != nullptr && len <= 2 * L;
    uint64_t* O = fin ? fo.out + fo.base + range_start[seg_range[id]] + pb : dst + g0 + pb;
    const bool f64 = fo.is_f64 != 0;
    const int64_t d0 = c0 - pb, d1 = c1 - pb;
    const int tid = threadIdx.x;
    if (nb == 0) {  // the segment's last run has no partner: carried over
        for (int64_t e = d0 + tid; e < d1; e += kMergeThreads) O[e] = fin ? order_key_inverse(A[e], f64) : A[e];
        return;
    }
    const int wv = tid >> 6, lane = tid & 63;
    if (wv < 2) {
        const int64_t sp = split_wave(A, na, B, nb, wv == 0 ? d0 : d1, lane);
        if (lane == 0) s_split[wv] = sp;
    }
    __syncthreads();
    const int64_t i0 = s_split[0], i1 = s_split[1];
    const int la = (int)(i1 - i0), lb = (int)((d1 - i1) - (d0 - i0));
    const uint64_t* Aw = A + i0;
    const uint64_t* Bw = B + (d0 - i0);
    {  // all of a thread's loads in flight before its LDS writes
        uint64_t t[kMergePer];
#pragma unroll
        for (int q = 0; q < kMergePer; ++q) {
            const int e = tid + q * kMergeThreads;
            t[q] = e < la ? Aw[e] : (e < la + lb ? Bw[e - la] : 0);
        }
#pragma unroll
        for (int q = 0; q < kMergePer; ++q) {
            const int e = tid + q * kMergeThreads;
            if (e < la + lb) s[e] = t[q];
        }
    }
    __syncthreads();
    // each thread merges kMergePer outputs into registers; they go back to
    // LDS (swizzled against bank conflicts) and out in wave-contiguous order
    const int tot = la + lb;
    const int t0 = tid * kMergePer;
    uint64_t v[kMergePer];
    if (t0 < tot) {
        const uint64_t* sa = s;
        const uint64_t* sb = s + la;
        int ia = split_lds(sa, la, sb, lb, t0);
        int ib = t0 - ia;
#pragma unroll
        for (int k = 0; k < kMergePer; ++k) {
            if (t0 + k < tot) {
                const bool takeA = ib >= lb || (ia < la && sa[ia] <= sb[ib]);
                v[k] = takeA ? sa[ia] : sb[ib];
                ia += takeA ? 1 : 0;
                ib += takeA ? 0 : 1;
            }
        }
    }
    __syncthreads();
    if (t0 < tot) {
#pragma unroll
        for (int k = 0; k < kMergePer; ++k)
            if (t0 + k < tot) s[swz(t0 + k)] = v[k];
    }
    __syncthreads();
    for (int e = tid; e < tot; e += kMergeThreads) {
        const uint64_t k = s[swz(e)];
        O[d0 + e] = fin ? order_key_inverse(k, f64) : k;
    }
}

int seg_rounds(int64_t max_len, int64_t run0) {
    int r = 0;
    for (int64_t L = run0; L < max_len; L <<= 1) ++r;
    return r;
}

// Sorts every segment of G; tmp holds as many keys as G, and a segment uses
// the same offsets in it.  A segment of len keys ends in
// (seg_rounds(len, run0) odd ? tmp : G).
hipError_t seg_sort(const int64_t* d_chunk_pref, const int64_t* d_gpref, int64_t nseg, int64_t nchunks,
                    int rounds, int64_t run0, uint64_t* d_G, uint64_t* d_tmp, hipStream_t st,
                    const int32_t* d_seg_range, const int64_t* d_range_start, SegOut fo) {
    if (fo.out && !(d_seg_range && d_range_start)) return hipErrorInvalidValue;
    if (nseg <= 0 || nchunks <= 0) return hipSuccess;
    if (run0 == kSortRun)
        hipLaunchKernelGGL(k_seg_sort_chunk<kSortRun>, dim3((unsigned)nchunks), dim3(kSortRun / kSortPerRun(kSortRun)), 0, st,
                           d_chunk_pref, d_gpref, nseg, d_seg_range, d_range_start, d_G, fo);
    else if (run0 == kBigChunk)
        hipLaunchKernelGGL(k_seg_sort_chunk<kBigChunk>, dim3((unsigned)nchunks), dim3(kBigChunk / kSortPerRun(kBigChunk)), 0, st,
                           d_chunk_pref, d_gpref, nseg, d_seg_range, d_range_start, d_G, fo);
    else
        return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint64_t* buf[2] = {d_G, d_tmp};
    for (int r = 0; r < rounds; ++r) {
        hipLaunchKernelGGL(k_seg_merge, dim3((unsigned)nchunks), dim3(kMergeThreads), 0, st, d_chunk_pref, d_gpref,
                           nseg, d_seg_range, d_range_start, run0 << r, buf[r & 1], buf[(r + 1) & 1], fo);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace nns
