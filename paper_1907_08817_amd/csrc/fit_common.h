// Device helpers shared by the fit's kernels (fit.hip, fit_mfma.hip): the
// counter-based generator, the loss of one batch entry, the Adam update of one
// parameter and fixed-order column sums of per-workgroup partial gradients.
#pragma once
#include "nnsort_internal.h"

namespace nns {

// ---- Philox4x32-10 ----
__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint32_t hi0 = __umulhi(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
        uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
        uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

__device__ __forceinline__ uint64_t rand64(uint64_t seed, uint32_t stream, uint64_t a, uint32_t b) {
    uint32_t c[4] = {(uint32_t)a, (uint32_t)(a >> 32), b, stream};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    return (uint64_t)c[0] | ((uint64_t)c[1] << 32);
}

constexpr uint32_t kStreamSample = 1, kStreamInit = 2, kStreamBatch = 3;

// Loss of one entry and its dL/dF before the 1/B scale (MSE, or Huber with
// threshold delta).
__device__ __forceinline__ float loss_term(float e, int loss, float delta, float& g) {
    if (loss == 1) {
        if (fabsf(e) <= delta) {
            g = e;
            return 0.5f * e * e;
        }
        g = e > 0.0f ? delta : -delta;
        return delta * fabsf(e) - 0.5f * delta * delta;
    }
    g = 2.0f * e;
    return e * e;
}

// One Adam step of parameter p with gradient gv (bias corrections c1, c2).
// The step on one parameter held in registers: (th, m, v) -> updated.
__device__ __forceinline__ void adam_step(float gv, float& th, float& m1, float& m2, float b1, float b2, float c1,
                                          float c2, float lr, float eps) {
    const float m = b1 * m1 + (1.0f - b1) * gv;
    const float v = b2 * m2 + (1.0f - b2) * gv * gv;
    m1 = m;
    m2 = v;
    const float mh = m / c1, vh = v / c2;
    th = th - lr * mh / (sqrtf(vh) + eps);
}
__device__ __forceinline__ void adam_update(int64_t p, float gv, float* th, float* m1, float* m2, float b1, float b2,
                                            float c1, float c2, float lr, float eps) {
    float t = th[p], m = m1[p], v = m2[p];
    adam_step(gv, t, m, v, b1, b2, c1, c2, lr, eps);
    m1[p] = m;
    m2[p] = v;
    th[p] = t;
}

// Column sums of `part` (rows x P), in a fixed order: kSumCols columns per
// block, eight groups of rows summed side by side, then the eight group sums
// in order.  The result is valid in the threads of group 0 (column p).
constexpr int kSumCols = 32;
constexpr int kSumUnroll = 8;
__device__ __forceinline__ float column_sum(const float* __restrict__ part, int rows, int P, int p, int c, int grp,
                                            float (*s)[kSumCols]) {
    float acc = 0.0f;
    if (p < P) {
#pragma unroll kSumUnroll
        for (int r = grp; r < rows; r += 8) acc += part[(int64_t)r * P + p];
    }
    s[grp][c] = acc;
    __syncthreads();
    float t = 0.0f;
    if (grp == 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) t += s[q][c];
    }
    return t;
}

}  // namespace nns
