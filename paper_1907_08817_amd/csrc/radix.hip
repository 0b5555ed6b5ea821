// The conventional sort of the procedure's last conflict array (Sec. 2:
// QuickSort(w) in the paper; here an LSD radix sort, which reaches the same
// unique result): 64-bit order keys, 8-bit digits.  One counting pass over
// all digit positions comes first, so that positions where every key has the
// same digit are skipped; each remaining position is one pass of the shared
// LSD scatter (lsd.h).
#include "lsd.h"

namespace nns {

hipError_t fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t st);

constexpr int kHistThreads = 256;

// Digit counts of all 8 byte positions.  High bytes are often the same for
// every key of a wave (keys of similar magnitude); then one lane adds the
// wave's count instead of 64 lanes hitting one LDS counter.
__global__ void __launch_bounds__(kHistThreads) k_hist_all(const uint64_t* __restrict__ in, int64_t n,
                                                           int in_mode, unsigned long long* hist8) {
    __shared__ uint32_t h[8][256];
    for (int i = threadIdx.x; i < 8 * 256; i += kHistThreads) (&h[0][0])[i] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    int64_t stride = (int64_t)gridDim.x * kHistThreads;
    for (int64_t base = (int64_t)blockIdx.x * kHistThreads; base < n; base += stride) {
        const int64_t i = base + threadIdx.x;
        const bool valid = i < n;
        const uint64_t k = valid ? to_order_key(in[i], in_mode) : 0;
        const unsigned long long act = __ballot(valid);
        const int leader = __ffsll((long long)act) - 1;
        const uint64_t k0 = __shfl(k, leader < 0 ? 0 : leader);
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const uint32_t d = (uint32_t)(k >> (8 * p)) & 255u;
            const uint32_t d0 = (uint32_t)(k0 >> (8 * p)) & 255u;
            const unsigned long long same = __ballot(valid && d == d0);
            if (same == act) {
                if (lane == leader) atomicAdd(&h[p][d0], (uint32_t)__popcll(act));
            } else if (valid) {
                atomicAdd(&h[p][d], 1u);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 8 * 256; i += kHistThreads) {
        uint32_t v = (&h[0][0])[i];
        if (v) atomicAdd(&hist8[i], (unsigned long long)v);
    }
}

__global__ void __launch_bounds__(256) k_convert(const uint64_t* __restrict__ in, uint64_t* out, int64_t n,
                                                 int in_mode, int out_mode) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = from_order_key(to_order_key(in[i], in_mode), out_mode);
}

hipError_t launch_convert(const uint64_t* d_in, uint64_t* d_out, int64_t n, int in_mode, int out_mode,
                          hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_convert, dim3((unsigned)blocks), dim3(256), 0, st, d_in, d_out, n, in_mode, out_mode);
    return hipGetLastError();
}

static size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t radix_ws_bytes(int64_t n) {
    const size_t nn = (size_t)(n > 0 ? n : 1);
    return a256(8 * 256 * 8) + a256(lsd_hist_words(n) * 4) + a256(nn * 8);
}

hipError_t radix_sort(const uint64_t* d_in, uint64_t* d_out, int64_t n, int in_mode, int out_mode,
                      void* d_ws, size_t ws_bytes, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (ws_bytes < radix_ws_bytes(n)) return hipErrorInvalidValue;
    const int64_t ntiles = (n + kLsdTile - 1) / kLsdTile;
    char* p = (char*)d_ws;
    unsigned long long* hist8 = (unsigned long long*)p;
    p += a256(8 * 256 * 8);
    uint32_t* hist = (uint32_t*)p;
    p += a256(lsd_hist_words(n) * 4);
    uint64_t* tmp = (uint64_t*)p;
    const uint32_t* chunk = hist + 256 * ntiles;

    hipError_t e = fill_u64((uint64_t*)hist8, 8 * 256, 0, st);
    if (e != hipSuccess) return e;
    int64_t hb = (n + kHistThreads - 1) / kHistThreads;
    if (hb > 2048) hb = 2048;
    hipLaunchKernelGGL(k_hist_all, dim3((unsigned)hb), dim3(kHistThreads), 0, st, d_in, n, in_mode, hist8);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    unsigned long long h[8 * 256];
    if ((e = hipMemcpyAsync(h, hist8, sizeof(h), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    int passes[8], np = 0;
    for (int ps = 0; ps < 8; ++ps) {
        bool trivial = false;
        for (int d = 0; d < 256; ++d)
            if (h[ps * 256 + d] == (unsigned long long)n) trivial = true;
        if (!trivial) passes[np++] = ps;
    }
    if (np == 0) return launch_convert(d_in, d_out, n, in_mode, out_mode, st);

    // ping-pong between d_out and tmp so that the last pass lands in d_out;
    // when sorting in place the first pass must not write over its source,
    // and a final copy moves the result where it belongs.
    uint64_t* bufs[2] = {d_out, tmp};
    int first = ((np - 1) % 2 == 0) ? 0 : 1;
    if (bufs[first] == d_in) first ^= 1;
    const uint64_t* src = d_in;
    for (int q = 0; q < np; ++q) {
        const bool last = q == np - 1;
        uint64_t* dst = bufs[(first + q) % 2];
        const KeyDigit dig{8 * passes[q]};
        const int im = q == 0 ? in_mode : 0;
        const int om = last ? out_mode : 0;
        hipLaunchKernelGGL((k_lsd_upsweep<false, KeyDigit>), dim3((unsigned)ntiles), dim3(kLsdThreads), 0, st, src,
                           nullptr, n, im, dig, hist);
        if ((e = launch_lsd_scan(hist, ntiles, st)) != hipSuccess) return e;
        if (q == 0)
            hipLaunchKernelGGL((k_lsd_downsweep<false, false, KeyDigit>), dim3((unsigned)ntiles), dim3(kLsdThreads),
                               0, st, src, nullptr, dst, nullptr, n, im, om, dig, 8, hist, chunk, ntiles);
        else
            hipLaunchKernelGGL((k_lsd_downsweep<true, false, KeyDigit>), dim3((unsigned)ntiles), dim3(kLsdThreads),
                               0, st, src, nullptr, dst, nullptr, n, im, om, dig, 8, hist, chunk, ntiles);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        src = dst;
    }
    if (src != d_out) return launch_convert(src, d_out, n, 0, 0, st);
    return hipSuccess;
}

}  // namespace nns
