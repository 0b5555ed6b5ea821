// BF16 form of the model map: the hidden-to-hidden layer on the matrix cores
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation), the rest on the vector ALU.
//
// One wave maps 32 keys per tile.  Keys are the N dimension of the product
// Z2^T[H x 32] = W2[H x H] * H1^T[H x 32]: lane l holds key j = l % 32 and lane
// half g = l / 32, so both layers' data of a key stays in the two lanes that
// own it and no transpose is needed:
//  - layer 1 (VALU, FP32 form order with the two-float input): lane (j, g)
//    computes hidden-1 units 16 s + 8 g + t (k-step s, t = 0..7), which is
//    exactly its slice of the B operand of k-step s;
//  - each activation is split exactly into up to three bfloat16 terms
//    (truncation: h = hi + mid + lo, 8 significant bits each), one MFMA per
//    term, so the product is formed from a 24-bit input (the bf16x3 scheme of
//    Henry, Tang and Heinecke, 2019) while W2 itself is rounded to bfloat16;
//  - the accumulators start at b2; lane (j, g) ends with hidden-2 units
//    32 rb + 8 (v / 4) + 4 g + v % 4 (v = 0..15) of its key;
//  - layer 3: relu (on the bits), then the dot product with w3 accumulated in FP64 (each
//    FP32 x FP32 product is exact there), the two halves' sums added in FP64,
//    so that F keeps a resolution finer than one slot at n = 1e9.
// Compiled with -ffp-contract=off.
#include "infer_common.h"

namespace nns {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t bf16_rne_bits(float v) {
    uint32_t u = __float_as_uint(v);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}

// Upper halves of two floats packed as (lo16 = x, hi16 = y).
__device__ __forceinline__ uint32_t pack_hi(float x, float y) {
    return __builtin_amdgcn_perm(__float_as_uint(y), __float_as_uint(x), 0x07060302u);
}

__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// relu as an integer max of the bit pattern: equal to z > 0 ? z : 0 for every
// z that is not a NaN (negative values and -0 have the sign bit set).  One
// instruction, where the float form costs two on matrix-core results (the
// compiler first quiets a possible signalling NaN).  Inputs are translated
// into [0, 1], so an activation is NaN only for a model with non-finite
// weights or FP32 overflow.
__device__ __forceinline__ float relu_bits(float z) {
    const int b = __float_as_int(z);
    return __int_as_float(b > 0 ? b : 0);
}

template <int H, int T>
__global__ void __launch_bounds__(256, 3) k_infer_bf16(InferArgs a) {
    constexpr int RB = H / 32;  // 32-row blocks of hidden-2 units
    constexpr int KS = H / 16;  // k-steps of 16 hidden-1 units
    const DevModel* __restrict__ m = a.model;
    // Per-unit vectors live in LDS and are re-read every tile: held in
    // registers they would cost 128 VGPRs at H = 64 and cut occupancy to one
    // wave per SIMD, leaving no other wave to cover MFMA and load latency.
    // s_w1 / s_b1 in layer-1 lane order, s_b2 / s_w3 in accumulator order:
    // entry (g, rb, v) for unit 32 rb + 8 (v / 4) + 4 g + v % 4.
    __shared__ float s_w1[64], s_b1[64];
    __shared__ float s_b2[2][64];
    __shared__ double s_w3[2][64];
    for (int i = threadIdx.x; i < H; i += blockDim.x) {
        s_w1[i] = m->w1[i];
        s_b1[i] = m->b1[i];
    }
    for (int i = threadIdx.x; i < 2 * H; i += blockDim.x) {
        const int g = i / H, rb = (i % H) / 16, v = i % 16;
        const int u = 32 * rb + 8 * (v >> 2) + 4 * g + (v & 3);
        s_b2[g][i % H] = m->b2[u];
        s_w3[g][i % H] = (double)m->w3[u];
    }
    __syncthreads();
    const int lane = __lane_id();
    const int j = lane & 31;
    const int g = lane >> 5;

    // A operands: W2 rows 32 rb + j, columns 16 s + 8 g + t, rounded to bf16,
    // staged in LDS per (rb, s, lane) and read back before each product, so
    // that they do not hold 32 VGPRs for the whole kernel (more waves per SIMD
    // to cover latency)
    __shared__ u32x4 s_A[RB][KS][64];
    {
        const int wv = threadIdx.x >> 6;
        for (int idx = wv; idx < RB * KS; idx += 4) {
            const int rb = idx / KS, s = idx % KS;
            const float* row = m->w2 + (32 * rb + j) * H + 16 * s + 8 * g;
            u32x4 a;
#pragma unroll
            for (int q = 0; q < 4; ++q) a[q] = bf16_rne_bits(row[2 * q]) | (bf16_rne_bits(row[2 * q + 1]) << 16);
            s_A[rb][s][lane] = a;
        }
    }
    __syncthreads();
    const float b3 = m->b3;
    const double lo = m->lo, inv = m->inv_range;
    const float* __restrict__ w1g = s_w1 + 8 * g;
    const float* __restrict__ b1g = s_b1 + 8 * g;
    const float* __restrict__ b2g = s_b2[g];
    const double* __restrict__ w3g = s_w3[g];

    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t ntiles = (a.n + 31) >> 5;
    for (int64_t tile = wave; tile < ntiles; tile += nwaves) {
        // keeps the compiler from hoisting the LDS vectors into registers
        __asm__ volatile("" ::: "memory");
        const int64_t i = tile * 32 + j;
        const bool active = i < a.n;
        const uint64_t bits = active ? a.in[i] : 0;
        double x = 0.0;
        const bool mapped = active && translate_key(bits, a.is_f64, lo, inv, &x);
        const float xh = (float)x;
        const float xl = (float)(x - (double)xh);

        floatx16 acc[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[rb][v] = b2g[16 * rb + v];

#pragma unroll
        for (int s = 0; s < KS; ++s) {
            float h[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int u = 16 * s + t;
                float z = __builtin_fmaf(w1g[u], xh, b1g[u]);
                z = __builtin_fmaf(w1g[u], xl, z);
                h[t] = z > 0.0f ? z : 0.0f;
            }
            u32x4 B0, B1, B2;
            float r1[8], r2[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                float hi = __uint_as_float(__float_as_uint(h[t]) & 0xFFFF0000u);
                r1[t] = h[t] - hi;
                if (T >= 3) {
                    float mid = __uint_as_float(__float_as_uint(r1[t]) & 0xFFFF0000u);
                    r2[t] = r1[t] - mid;
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                B0[q] = pack_hi(h[2 * q], h[2 * q + 1]);
                if (T >= 2) B1[q] = pack_hi(r1[2 * q], r1[2 * q + 1]);
                if (T >= 3) B2[q] = pack_hi(r2[2 * q], r2[2 * q + 1]);
            }
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const bf16x8 av = as_bf16x8(s_A[rb][s][lane]);
                acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, as_bf16x8(B0), acc[rb], 0, 0, 0);
                if (T >= 2)
                    acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, as_bf16x8(B1), acc[rb], 0, 0, 0);
                if (T >= 3)
                    acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, as_bf16x8(B2), acc[rb], 0, 0, 0);
            }
        }

        // layer 3: w3 . relu(z2) accumulated in FP64.  A product of two FP32
        // values is exact in FP64, so the sum carries ~2^-53 relative error
        // per step: F keeps a resolution far below one slot at n = 1e9, at
        // three VALU operations per unit (relu, convert, FP64 FMA)
        double sum = g == 0 ? (double)b3 : 0.0;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const float h2 = relu_bits(acc[rb][v]);
                sum = __builtin_fma(w3g[16 * rb + v], (double)h2, sum);
            }
        const double F = sum + __shfl_xor(sum, 32);
        const uint32_t slot = mapped ? slot_of(F, a.M) : kUnmapped;
        if (active && g == 0) {
            if (a.slots_out) a.slots_out[i] = slot;
            if (a.F_out) a.F_out[i] = mapped ? F : __longlong_as_double(0x7FF8000000000000ll);
        }
    }
}

hipError_t launch_bf16_infer(const InferArgs& a, int H, int bf16_terms, hipStream_t st) {
    int64_t tiles = (a.n + 31) / 32;
    // grid-stride over 32-key tiles; 64 workgroups per CU (about ten times
    // what is resident at once) balances the waves' finishing times better
    // than fewer, longer-lived workgroups (measured: 6 per CU is 11% slower,
    // 16 per CU 4%, 256 per CU 2%)
    int64_t blocks = (tiles + 3) / 4;
    if (blocks > 256 * 64) blocks = 256 * 64;
    if (blocks < 1) blocks = 1;
    dim3 grid((unsigned)blocks), block(256);
#define NNS_BF16_CASE(HH, TT)                                                     \
    if (H == HH && bf16_terms == TT) {                                           \
        hipLaunchKernelGGL((k_infer_bf16<HH, TT>), grid, block, 0, st, a);       \
        return hipGetLastError();                                                \
    }
    NNS_BF16_CASE(32, 1)
    NNS_BF16_CASE(32, 2)
    NNS_BF16_CASE(32, 3)
    NNS_BF16_CASE(64, 1)
    NNS_BF16_CASE(64, 2)
    NNS_BF16_CASE(64, 3)
#undef NNS_BF16_CASE
    return hipErrorInvalidValue;
}

}  // namespace nns
