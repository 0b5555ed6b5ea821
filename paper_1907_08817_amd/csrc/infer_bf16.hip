// BF16 form of the model map: the hidden-to-hidden layer on the matrix cores
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation), the rest on the vector ALU.
//
// A wave takes 64 keys per step: lane l translates key l of the block, and
// the block is mapped as two 32-key tiles A (keys 0..31) and B (32..63).  In
// a tile, keys are the N dimension of the product
// Z2^T[H x 32] = W2[H x H] * H1^T[H x 32]: lane l holds key j = l % 32 and
// lane half g = l / 32, so both layers' data of a key stays in the two lanes
// that own it and no transpose is needed:
//  - layer 1 (VALU, FP32 form order with the two-float input): lane (j, g)
//    computes hidden-1 units 16 s + 8 g + t (k-step s, t = 0..7), which is
//    exactly its slice of the B operand of k-step s;
//  - each activation is split exactly into up to three bfloat16 terms
//    (truncation: h = hi + mid + lo, 8 significant bits each), one MFMA per
//    term, so the product is formed from a 24-bit input (the bf16x3 scheme of
//    Henry, Tang and Heinecke, 2019) while W2 itself is rounded to bfloat16;
//  - the accumulators start at b2; lane (j, g) ends with hidden-2 units
//    32 rb + 8 (v / 4) + 4 g + v % 4 (v = 0..15) of its key;
//  - layer 3: the dot product with w3 accumulated in FP64 (each FP32 x FP32
//    product is exact there), the two halves' sums added in FP64, so that F
//    keeps a resolution finer than one slot at n = 1e9.
// The two lane halves then swap one partial sum, so that lane l ends with F
// of its own key l; translate, slot and store run once per key.  The two
// tiles go through each k-step together: one read of the k-step's layer-1
// weights and W2 operands from LDS serves both (half the LDS traffic of
// mapping them one after the other).  Held to 4 waves per SIMD: 128 VGPRs at
// H = 64, one value spilled outside the block loop.
//
// A workgroup maps one partition tile (2048 keys, 8 blocks per wave) at a
// time; in a sort it also counts the tile's keys by the first partition
// pass's range digit in LDS and stores the tile's histogram, so the
// partition does not read the slots back to count them.
//
// Scaled operands (the host's bf16_operands()): with every pre-activation of
// the power-of-two-scaled network at most 1, relu(z) equals clamp(z, 0, 1),
// which the layer-1 FMA and the FP32 -> FP64 conversion of layer 3 apply
// through their output clamp bit: two VALU instructions per unit fewer.  When
// the host could not scale exactly, relu is applied explicitly (SCALED false).
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
// z that is not a NaN (negative values and -0 have the sign bit set).
__device__ __forceinline__ float relu_bits(float z) {
    const int b = __float_as_int(z);
    return __int_as_float(b > 0 ? b : 0);
}

// relu of a pre-activation known to be at most 1: the clamp folds into the
// producing instruction's output modifier.
__device__ __forceinline__ float clamp01(float z) { return __builtin_amdgcn_fmed3f(z, 0.0f, 1.0f); }
__device__ __forceinline__ double clamp01(double z) { return __builtin_fmin(__builtin_fmax(z, 0.0), 1.0); }

// Value of the other lane half (lane l ^ 32).
__device__ __forceinline__ float other_half(float v) { return __shfl_xor(v, 32); }
__device__ __forceinline__ double other_half(double v) { return __shfl_xor(v, 32); }

// Per-wave LDS view of the operands a tile reads.
struct TileOps {
    const float* w1g;   // layer-1 weights of this lane half, in k order
    const float* b1g;
    const float* b2g;   // b2 in accumulator order of this lane half
    const double* w3g;  // w3 in accumulator order of this lane half
};

// The bf16 terms of unit pair q of eight activations (truncation split):
// term 0 the heads, term 1 the first residuals, term 2 the second.
template <int T>
__device__ __forceinline__ void split_terms(const float (&h)[8], u32x4& t0, u32x4& t1, u32x4& t2) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float h0 = h[2 * q], h1 = h[2 * q + 1];
        t0[q] = pack_hi(h0, h1);
        if (T >= 2) {
            const float r0 = h0 - __uint_as_float(__float_as_uint(h0) & 0xFFFF0000u);
            const float r1 = h1 - __uint_as_float(__float_as_uint(h1) & 0xFFFF0000u);
            t1[q] = pack_hi(r0, r1);
            if (T >= 3) {
                const float q0 = r0 - __uint_as_float(__float_as_uint(r0) & 0xFFFF0000u);
                const float q1 = r1 - __uint_as_float(__float_as_uint(r1) & 0xFFFF0000u);
                t2[q] = pack_hi(q0, q1);
            }
        }
    }
}

// This lane's halves of the layer-3 sums of two tiles, A and B, whose keys'
// translated inputs are (xa, xla) and (xb, xlb): units of lane half g only,
// b3 included in half 0.  Each tile's products and sums run in the same order
// as for a tile alone; the two share every read of the per-unit vectors and
// of the W2 operands, so a 64-key block costs half the LDS traffic.
template <int H, int T, bool SCALED>
__device__ __forceinline__ void pair_half_sums(float xa, float xla, float xb, float xlb, int g, float b3,
                                               const TileOps& op, const u32x4 (*s_A)[H / 16][64], int lane,
                                               double& sumA, double& sumB) {
    constexpr int RB = H / 32;  // 32-row blocks of hidden-2 units
    constexpr int KS = H / 16;  // k-steps of 16 hidden-1 units
    // the accumulators start at b2: the first product of each tile takes it
    // as its C operand
    floatx16 b2v[RB], accA[RB], accB[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int v = 0; v < 16; ++v) b2v[rb][v] = op.b2g[16 * rb + v];

#pragma unroll
    for (int s = 0; s < KS; ++s) {
        // the k-step's layer-1 weights and W2 operands, read once for both tiles
        float w[8], c[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            w[t] = op.w1g[16 * s + t];
            c[t] = op.b1g[16 * s + t];
        }
        bf16x8 av[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) av[rb] = as_bf16x8(s_A[rb][s][lane]);
#pragma unroll
        for (int tile = 0; tile < 2; ++tile) {
            const float x0 = tile ? xb : xa, x1 = tile ? xlb : xla;
            float h[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                float z = __builtin_fmaf(w[t], x0, c[t]);
                z = __builtin_fmaf(w[t], x1, z);
                h[t] = SCALED ? clamp01(z) : (z > 0.0f ? z : 0.0f);
            }
            u32x4 B0, B1, B2;
            split_terms<T>(h, B0, B1, B2);
            floatx16* acc = tile ? accB : accA;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[rb], as_bf16x8(B0), s == 0 ? b2v[rb] : acc[rb], 0, 0, 0);
                if (T >= 2) acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[rb], as_bf16x8(B1), acc[rb], 0, 0, 0);
                if (T >= 3) acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[rb], as_bf16x8(B2), acc[rb], 0, 0, 0);
            }
        }
    }

    // layer 3: w3 . relu(z2) accumulated in FP64.  A product of two FP32
    // values is exact in FP64, so the sum carries ~2^-53 relative error per
    // step: F keeps a resolution far below one slot at n = 1e9
    double sa = g == 0 ? (double)b3 : 0.0, sb = sa;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const double w = op.w3g[16 * rb + v];
            const double ya = SCALED ? clamp01((double)accA[rb][v]) : (double)relu_bits(accA[rb][v]);
            const double yb = SCALED ? clamp01((double)accB[rb][v]) : (double)relu_bits(accB[rb][v]);
            sa = __builtin_fma(w, ya, sa);
            sb = __builtin_fma(w, yb, sb);
        }
    sumA = sa;
    sumB = sb;
}

template <int H, int T, bool SCALED>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) k_infer_bf16(InferArgs a) {
    constexpr int RB = H / 32;
    constexpr int KS = H / 16;
    const DevModel* __restrict__ m = a.model;
    // Per-unit vectors live in LDS and are re-read every 64 keys: held in
    // registers they would cost 128 VGPRs at H = 64 and cut occupancy to one
    // wave per SIMD, leaving no other wave to cover MFMA and load latency.
    // s_w1 / s_b1 in layer-1 lane order, s_b2 / s_w3 in accumulator order:
    // entry (g, rb, v) for unit 32 rb + 8 (v / 4) + 4 g + v % 4.
    __shared__ float s_w1[64], s_b1[64];
    __shared__ float s_b2[2][64];
    __shared__ double s_w3[2][64];
    for (int i = threadIdx.x; i < H; i += blockDim.x) {
        s_w1[i] = m->w1s[i];
        s_b1[i] = m->b1s[i];
    }
    for (int i = threadIdx.x; i < 2 * H; i += blockDim.x) {
        const int g = i / H, rb = (i % H) / 16, v = i % 16;
        const int u = 32 * rb + 8 * (v >> 2) + 4 * g + (v & 3);
        s_b2[g][i % H] = m->b2s[u];
        s_w3[g][i % H] = m->w3s[u];
    }
    __syncthreads();
    const int lane = __lane_id();
    const int j = lane & 31;
    const int g = lane >> 5;

    // A operands: W2 rows 32 rb + j, columns 16 s + 8 g + t (bf16 values,
    // scaled), staged in LDS per (rb, s, lane) and read back before each
    // product, so that they do not hold 32 VGPRs for the whole kernel (more
    // waves per SIMD to cover latency)
    __shared__ u32x4 s_A[RB][KS][64];
    {
        const int wv = threadIdx.x >> 6;
        for (int idx = wv; idx < RB * KS; idx += 4) {
            const int rb = idx / KS, s = idx % KS;
            const float* row = m->w2s + (32 * rb + j) * H + 16 * s + 8 * g;
            u32x4 av;
#pragma unroll
            for (int q = 0; q < 4; ++q) av[q] = bf16_rne_bits(row[2 * q]) | (bf16_rne_bits(row[2 * q + 1]) << 16);
            s_A[rb][s][lane] = av;
        }
    }
    __syncthreads();
    const float b3 = m->b3;
    const double lo = m->lo, inv = m->inv_range;
    const TileOps op{s_w1 + 8 * g, s_b1 + 8 * g, s_b2[g], s_w3[g]};

    const int64_t nblocks = (a.n + 63) >> 6;
    // Maps block blk (keys 64 blk .. 64 blk + 63; the whole wave calls it
    // with the same blk) and returns the slot of the lane's key.
    auto map_block = [&](int64_t blk) -> uint32_t {
        // keeps the compiler from hoisting the LDS vectors into registers
        __asm__ volatile("" ::: "memory");
        const int64_t i = blk * 64 + lane;
        const bool active = i < a.n;
        const uint64_t bits = active ? a.in[i] : 0;
        double x = 0.0;
        const bool mapped = active && translate_key(bits, a.is_f64, lo, inv, &x);
        const float xh = (float)x;
        const float xl = (float)(x - (double)xh);
        // tile A maps keys 0..31 of the block (lane half 0's own keys), tile B
        // keys 32..63: each lane takes the other half's input for one of them
        const float xh_o = other_half(xh), xl_o = other_half(xl);
        double sA, sB;
        pair_half_sums<H, T, SCALED>(g ? xh_o : xh, g ? xl_o : xl, g ? xh : xh_o, g ? xl : xl_o, g, b3, op, s_A, lane,
                                     sA, sB);
        // F of key l: lane half 0 adds half 1's sum of tile A, lane half 1
        // half 0's sum of tile B (the same two terms a sum over both halves
        // of one tile adds)
        const double F = (g ? sB : sA) + other_half(g ? sA : sB);
        uint32_t slot = kUnmapped;
        if (active) {
            slot = mapped ? slot_of(F, a.M) : kUnmapped;
            if (a.slots_out) a.slots_out[i] = slot;
            if (a.F_out) a.F_out[i] = mapped ? F : __longlong_as_double(0x7FF8000000000000ll);
        }
        return slot;
    };

    // Tiles of kPartTile keys, one per workgroup at a time: wave w maps
    // blocks 8w .. 8w + 7 of the tile.  With tile_hist, the keys' first-pass
    // digits are counted in LDS and the tile's histogram stored as the
    // partition's count kernel would store it.
    static_assert(kPartTile == 4 * 8 * 64, "a tile is 8 blocks per wave of a 256-thread workgroup");
    __shared__ uint32_t s_h[256];
    const int wv = threadIdx.x >> 6;
    const int64_t ntiles = (a.n + kPartTile - 1) / kPartTile;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        if (a.tile_hist) {
            s_h[threadIdx.x] = 0;
            __syncthreads();
        }
#pragma unroll 1
        for (int k = 0; k < 8; ++k) {
            const int64_t blk = t * 32 + wv * 8 + k;
            if (blk < nblocks) {
                const uint32_t sl = map_block(blk);
                if (a.tile_hist && blk * 64 + lane < a.n) atomicAdd(&s_h[range_of(sl, a.NB) & a.dmask], 1u);
            }
        }
        if (a.tile_hist) {
            __syncthreads();
            a.tile_hist[t * 256 + threadIdx.x] = s_h[threadIdx.x];
        }
    }
}

hipError_t launch_bf16_infer(const InferArgs& a, int H, int bf16_terms, bool scaled, hipStream_t st) {
    // grid-stride over tiles; up to 64 workgroups per CU (about ten times
    // what is resident at once) balances the waves' finishing times better
    // than fewer, longer-lived workgroups
    int64_t blocks = (a.n + kPartTile - 1) / kPartTile;
    if (blocks > 256 * 64) blocks = 256 * 64;
    if (blocks < 1) blocks = 1;
    dim3 grid((unsigned)blocks), block(256);
#define NNS_BF16_CASE(HH, TT)                                                          \
    if (H == HH && bf16_terms == TT) {                                                 \
        if (scaled)                                                                    \
            hipLaunchKernelGGL((k_infer_bf16<HH, TT, true>), grid, block, 0, st, a);   \
        else                                                                           \
            hipLaunchKernelGGL((k_infer_bf16<HH, TT, false>), grid, block, 0, st, a);  \
        return hipGetLastError();                                                      \
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
