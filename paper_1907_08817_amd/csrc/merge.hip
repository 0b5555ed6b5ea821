// Merge of two ascending order-key arrays (the polish phase's final merge of
// the bucket-sorted keys with the conventionally sorted remainder, Sec. 2,
// Algorithm polish).  Merge path: each workgroup owns 2048 consecutive
// outputs, finds its split of the two inputs by binary search, stages both
// slices in LDS and lets each thread merge 8 outputs.  Ties take the first
// array first.  Output is decoded to the caller's bit patterns.
#include "nnsort_internal.h"

namespace nns {

constexpr int kMergeThreads = 256;
constexpr int kMergeItems = 8;
constexpr int kMergeTile = kMergeThreads * kMergeItems;

__device__ __forceinline__ int64_t global_split(const uint64_t* a, int64_t na, const uint64_t* b, int64_t nb,
                                                int64_t diag) {
    int64_t lo = diag > nb ? diag - nb : 0;
    int64_t hi = diag < na ? diag : na;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] <= b[diag - 1 - mid]) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ void __launch_bounds__(kMergeThreads) k_merge(const uint64_t* __restrict__ a, int64_t na,
                                                         const uint64_t* __restrict__ b, int64_t nb,
                                                         uint64_t* __restrict__ out, int out_mode) {
    __shared__ uint64_t sa[kMergeTile];
    __shared__ uint64_t sb[kMergeTile];
    __shared__ int64_t split[2];
    const int64_t total = na + nb;
    const int64_t d0 = (int64_t)blockIdx.x * kMergeTile;
    const int64_t d1 = d0 + kMergeTile < total ? d0 + kMergeTile : total;
    if (threadIdx.x < 2) split[threadIdx.x] = global_split(a, na, b, nb, threadIdx.x ? d1 : d0);
    __syncthreads();
    const int64_t a0 = split[0], a1 = split[1];
    const int64_t b0 = d0 - a0, b1 = d1 - a1;
    const int la = (int)(a1 - a0), lb = (int)(b1 - b0);
    for (int i = threadIdx.x; i < la; i += kMergeThreads) sa[i] = a[a0 + i];
    for (int i = threadIdx.x; i < lb; i += kMergeThreads) sb[i] = b[b0 + i];
    __syncthreads();
    const int n = la + lb;
    int d = threadIdx.x * kMergeItems;
    if (d >= n) return;
    int lo = d > lb ? d - lb : 0, hi = d < la ? d : la;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (sa[mid] <= sb[d - 1 - mid]) lo = mid + 1;
        else hi = mid;
    }
    int ia = lo, ib = d - lo;
    const bool f64 = out_mode == 1;
    for (int k = 0; k < kMergeItems && d + k < n; ++k) {
        bool takeA = ib >= lb || (ia < la && sa[ia] <= sb[ib]);
        uint64_t v = takeA ? sa[ia] : sb[ib];
        ia += takeA ? 1 : 0;
        ib += takeA ? 0 : 1;
        out[d0 + d + k] = f64 ? order_key_inverse(v, true) : v;
    }
}

hipError_t launch_merge(const uint64_t* d_a, int64_t na, const uint64_t* d_b, int64_t nb, uint64_t* d_out,
                        int out_mode, hipStream_t st) {
    int64_t total = na + nb;
    if (total <= 0) return hipSuccess;
    int64_t blocks = (total + kMergeTile - 1) / kMergeTile;
    hipLaunchKernelGGL(k_merge, dim3((unsigned)blocks), dim3(kMergeThreads), 0, st, d_a, na, d_b, nb, d_out,
                       out_mode);
    return hipGetLastError();
}

}  // namespace nns
