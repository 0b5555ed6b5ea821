// The conventional sort of the procedure's last conflict array (Sec. 2:
// QuickSort(w) in the paper; here an LSD radix sort, which reaches the same
// unique result): 64-bit order keys, 8-bit digits, one counting pass over all
// digit positions first so that positions where every key has the same digit
// are skipped.  Each remaining pass is reduce-then-scan: per-tile digit
// histograms, one exclusive scan over (digit, tile), then a stable scatter
// where keys are ranked inside a wave with ballot-based digit matching.
#include "nnsort_internal.h"

namespace nns {

constexpr int kRadixThreads = 256;
constexpr int kRadixItems = 16;
constexpr int kRadixTile = kRadixThreads * kRadixItems;  // 4096
constexpr int kWaves = kRadixThreads / 64;

__device__ __forceinline__ uint64_t conv_in(uint64_t v, int mode) {
    return mode == 1 ? order_key(v, true) : v;  // mode 0 (order key) and 2 (u64) are identities
}
__device__ __forceinline__ uint64_t conv_out(uint64_t v, int mode) {
    return mode == 1 ? order_key_inverse(v, true) : v;
}

__global__ void __launch_bounds__(kRadixThreads) k_hist_all(const uint64_t* __restrict__ in, int64_t n,
                                                            int in_mode, unsigned long long* hist8) {
    __shared__ uint32_t h[8][256];
    for (int i = threadIdx.x; i < 8 * 256; i += kRadixThreads) (&h[0][0])[i] = 0;
    __syncthreads();
    int64_t stride = (int64_t)gridDim.x * kRadixThreads;
    for (int64_t i = (int64_t)blockIdx.x * kRadixThreads + threadIdx.x; i < n; i += stride) {
        uint64_t k = conv_in(in[i], in_mode);
#pragma unroll
        for (int p = 0; p < 8; ++p) atomicAdd(&h[p][(k >> (8 * p)) & 255], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 8 * 256; i += kRadixThreads) {
        uint32_t v = (&h[0][0])[i];
        if (v) atomicAdd(&hist8[i], (unsigned long long)v);
    }
}

__global__ void __launch_bounds__(kRadixThreads) k_upsweep(const uint64_t* __restrict__ in, int64_t n,
                                                           int in_mode, int shift, uint32_t* blockhist,
                                                           int64_t nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t t0 = (int64_t)blockIdx.x * kRadixTile;
#pragma unroll 4
    for (int k = 0; k < kRadixItems; ++k) {
        int64_t i = t0 + k * kRadixThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(conv_in(in[i], in_mode) >> shift) & 255], 1u);
    }
    __syncthreads();
    blockhist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// ---- exclusive scan of uint32 (values fit: totals <= n < 2^32) ----
constexpr int kScanChunk = 2048;  // 256 threads x 8

__global__ void __launch_bounds__(256) k_scan_chunks(uint32_t* data, int64_t len, uint32_t* sums) {
    __shared__ uint32_t s[256];
    int64_t base = (int64_t)blockIdx.x * kScanChunk + threadIdx.x * 8;
    uint32_t v[8], tot = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        v[k] = base + k < len ? data[base + k] : 0;
        tot += v[k];
    }
    s[threadIdx.x] = tot;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t y = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += y;
        __syncthreads();
    }
    uint32_t run = s[threadIdx.x] - tot;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (base + k < len) data[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 255) sums[blockIdx.x] = s[255];
}

__global__ void __launch_bounds__(1024) k_scan_top(uint32_t* sums, int64_t m) {
    __shared__ uint32_t s[1024];
    int64_t per = (m + 1023) / 1024;
    int64_t b0 = threadIdx.x * per;
    uint32_t tot = 0;
    for (int64_t i = b0; i < b0 + per && i < m; ++i) tot += sums[i];
    s[threadIdx.x] = tot;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t y = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += y;
        __syncthreads();
    }
    uint32_t run = s[threadIdx.x] - tot;
    for (int64_t i = b0; i < b0 + per && i < m; ++i) {
        uint32_t v = sums[i];
        sums[i] = run;
        run += v;
    }
}

__global__ void __launch_bounds__(256) k_scan_add(uint32_t* data, int64_t len, const uint32_t* sums) {
    int64_t base = (int64_t)blockIdx.x * kScanChunk;
    uint32_t add = sums[blockIdx.x];
    for (int k = threadIdx.x; k < kScanChunk; k += 256)
        if (base + k < len) data[base + k] += add;
}

hipError_t exclusive_scan_u32(uint32_t* data, int64_t len, uint32_t* sums, hipStream_t st) {
    int64_t chunks = (len + kScanChunk - 1) / kScanChunk;
    hipLaunchKernelGGL(k_scan_chunks, dim3((unsigned)chunks), dim3(256), 0, st, data, len, sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, sums, chunks);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)chunks), dim3(256), 0, st, data, len, sums);
    return hipGetLastError();
}

__global__ void __launch_bounds__(kRadixThreads) k_downsweep(const uint64_t* __restrict__ in,
                                                             uint64_t* __restrict__ out, int64_t n,
                                                             int in_mode, int out_mode, int shift,
                                                             const uint32_t* __restrict__ scanned,
                                                             int64_t nblocks) {
    __shared__ uint32_t wcnt[kWaves][256];
    __shared__ uint32_t gofs[256];
    const int lane = __lane_id();
    const int w = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < kWaves * 256; i += kRadixThreads) (&wcnt[0][0])[i] = 0;
    gofs[threadIdx.x] = scanned[(int64_t)threadIdx.x * nblocks + blockIdx.x];
    __syncthreads();

    const int64_t t0 = (int64_t)blockIdx.x * kRadixTile + (int64_t)w * (kRadixItems * 64);
    uint64_t key[kRadixItems];
    uint32_t rank[kRadixItems];
    const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int k = 0; k < kRadixItems; ++k) {
        int64_t i = t0 + k * 64 + lane;
        bool valid = i < n;
        key[k] = valid ? conv_in(in[i], in_mode) : 0;
        uint32_t d = (uint32_t)(key[k] >> shift) & 255u;
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            unsigned long long bb = __ballot(valid && ((d >> bit) & 1u));
            peers &= ((d >> bit) & 1u) ? bb : ~bb;
        }
        uint32_t base = valid ? wcnt[w][d] : 0;
        rank[k] = base + (uint32_t)__popcll(peers & lt);
        // the lowest lane of each digit group bumps the wave's counter
        if (valid && (peers & lt) == 0) wcnt[w][d] = base + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // per digit: exclusive prefix over waves, plus the tile's global offset
    {
        uint32_t d = threadIdx.x;
        uint32_t run = gofs[d];
#pragma unroll
        for (int ww = 0; ww < kWaves; ++ww) {
            uint32_t c = wcnt[ww][d];
            wcnt[ww][d] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRadixItems; ++k) {
        int64_t i = t0 + k * 64 + lane;
        if (i < n) {
            uint32_t d = (uint32_t)(key[k] >> shift) & 255u;
            out[wcnt[w][d] + rank[k]] = conv_out(key[k], out_mode);
        }
    }
}

__global__ void __launch_bounds__(256) k_convert(const uint64_t* __restrict__ in, uint64_t* out, int64_t n,
                                                 int in_mode, int out_mode) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = conv_out(conv_in(in[i], in_mode), out_mode);
}

hipError_t launch_convert(const uint64_t* d_in, uint64_t* d_out, int64_t n, int in_mode, int out_mode,
                          hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_convert, dim3((unsigned)blocks), dim3(256), 0, st, d_in, d_out, n, in_mode, out_mode);
    return hipGetLastError();
}

// Workspace: hist8 (8*256 u64) | blockhist (256 * nblocks u32) | sums | temp keys (n u64)
size_t radix_ws_bytes(int64_t n) {
    int64_t nblocks = (n + kRadixTile - 1) / kRadixTile;
    if (nblocks < 1) nblocks = 1;
    size_t a = 8 * 256 * 8;
    size_t b = ((size_t)256 * nblocks * 4 + 255) & ~(size_t)255;
    size_t c = (((size_t)(256 * nblocks + kScanChunk - 1) / kScanChunk) * 4 + 255) & ~(size_t)255;
    size_t d = ((size_t)(n > 0 ? n : 1) * 8 + 255) & ~(size_t)255;
    return a + b + c + d;
}

hipError_t radix_sort(const uint64_t* d_in, uint64_t* d_out, int64_t n, int in_mode, int out_mode,
                      void* d_ws, size_t ws_bytes, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (ws_bytes < radix_ws_bytes(n)) return hipErrorInvalidValue;
    int64_t nblocks = (n + kRadixTile - 1) / kRadixTile;
    char* p = (char*)d_ws;
    unsigned long long* hist8 = (unsigned long long*)p;
    p += 8 * 256 * 8;
    uint32_t* blockhist = (uint32_t*)p;
    p += ((size_t)256 * nblocks * 4 + 255) & ~(size_t)255;
    uint32_t* sums = (uint32_t*)p;
    p += (((size_t)(256 * nblocks + kScanChunk - 1) / kScanChunk) * 4 + 255) & ~(size_t)255;
    uint64_t* tmp = (uint64_t*)p;

    hipError_t e = hipMemsetAsync(hist8, 0, 8 * 256 * 8, st);
    if (e != hipSuccess) return e;
    int64_t hb = nblocks < 2048 ? nblocks : 2048;
    hipLaunchKernelGGL(k_hist_all, dim3((unsigned)hb), dim3(kRadixThreads), 0, st, d_in, n, in_mode, hist8);
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
        bool last = q == np - 1;
        uint64_t* dst = bufs[(first + q) % 2];
        int shift = 8 * passes[q];
        int im = q == 0 ? in_mode : 0;
        int om = last ? out_mode : 0;
        hipLaunchKernelGGL(k_upsweep, dim3((unsigned)nblocks), dim3(kRadixThreads), 0, st, src, n, im, shift,
                           blockhist, nblocks);
        if ((e = exclusive_scan_u32(blockhist, 256 * nblocks, sums, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_downsweep, dim3((unsigned)nblocks), dim3(kRadixThreads), 0, st, src, dst, n, im,
                           om, shift, blockhist, nblocks);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        src = dst;
    }
    if (src != d_out) return launch_convert(src, d_out, n, 0, 0, st);
    return hipSuccess;
}

}  // namespace nns
