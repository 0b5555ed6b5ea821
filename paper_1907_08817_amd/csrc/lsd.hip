// Host side of the shared LSD pass: the two-kernel scan of the tile
// histograms into output offsets.
#include "lsd.h"

namespace nns {

// Offsets from the tile histograms, in two coalesced passes.  Tiles are taken
// in chunks of kScanTiles: (1) per chunk and digit, the exclusive prefix over
// the chunk's tiles in place, and the chunk total; (2) per digit, the
// exclusive prefix over chunks plus the digit's start (all digits below it).
// A tile's output offset for digit d is then hist[t][d] + chunk[t / kScanTiles][d].
__global__ void __launch_bounds__(256) k_lsd_scan_chunks(uint32_t* hist, int64_t ntiles, uint32_t* chunk) {
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
__global__ void __launch_bounds__(1024) k_lsd_scan_top(uint32_t* chunk, int64_t nchunks) {
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

hipError_t launch_lsd_scan(uint32_t* hist, int64_t ntiles, hipStream_t st) {
    const int64_t nchunks = (ntiles + kScanTiles - 1) / kScanTiles;
    uint32_t* chunk = hist + 256 * ntiles;
    hipLaunchKernelGGL(k_lsd_scan_chunks, dim3((unsigned)nchunks), dim3(256), 0, st, hist, ntiles, chunk);
    hipLaunchKernelGGL(k_lsd_scan_top, dim3(1), dim3(1024), 0, st, chunk, nchunks);
    return hipGetLastError();
}

// Tile histograms followed by the chunk offsets.
size_t lsd_hist_words(int64_t n) {
    int64_t ntiles = (n + kLsdTile - 1) / kLsdTile;
    if (ntiles < 1) ntiles = 1;
    int64_t nchunks = (ntiles + kScanTiles - 1) / kScanTiles;
    return (size_t)256 * (ntiles + nchunks);
}

}  // namespace nns
