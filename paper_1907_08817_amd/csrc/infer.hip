// Input and sorting phases' map (Sec. 2, Procedure NN-sort): translate each
// key, evaluate the learned model f and round F * m * n to a slot.  The keys
// themselves move in the partition by slot range that follows.
//
// FP32 form: one thread per key, weights read as wave-uniform scalars, the
// operation order fixed exactly as below so that the slot can be reproduced
// bit for bit on a CPU:
//   xh = fl32(x), xl = fl32(x - xh)
//   z1_j = fma(w1_j, xl, fma(w1_j, xh, b1_j));  h1_j = z1_j > 0 ? z1_j : 0
//   z2_i = b2_i; for j ascending z2_i = fma(W2_ij, h1_j, z2_i);  h2 = relu
//   F = b3 + sum_i w3_i h2_i as a compensated dot product (Dot2: Ogita, Rump
//       and Oishi 2005), i ascending, returned as double(sum) + double(err)
//   slot = round-half-away(clamp(F * M, 0, M)) in FP64.
// This translation unit is compiled with -ffp-contract=off.
#include "infer_common.h"

namespace nns {

template <int H>
__device__ __forceinline__ double model_fp32(const DevModel* __restrict__ m, double xhat) {
    float xh = (float)xhat;
    float xl = (float)(xhat - (double)xh);
    float h1[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
        float z = __builtin_fmaf(m->w1[j], xh, m->b1[j]);
        z = __builtin_fmaf(m->w1[j], xl, z);
        h1[j] = z > 0.0f ? z : 0.0f;
    }
    float p = m->b3, s = 0.0f;
    for (int i = 0; i < H; ++i) {
        float z = m->b2[i];
        const float* w = m->w2 + i * H;
#pragma unroll
        for (int j = 0; j < H; ++j) z = __builtin_fmaf(w[j], h1[j], z);
        float h2 = z > 0.0f ? z : 0.0f;
        float w3 = m->w3[i];
        float pr = w3 * h2;
        float r = __builtin_fmaf(w3, h2, -pr);
        float q;
        p = two_sum(p, pr, q);
        s = s + (q + r);
    }
    return (double)p + (double)s;
}

template <int H>
__global__ void __launch_bounds__(256) k_infer_fp32(InferArgs a) {
    const DevModel* __restrict__ m = a.model;
    const double lo = m->lo, inv = m->inv_range;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        const uint64_t bits = a.in[i];
        uint32_t slot = kUnmapped;
        double F = __longlong_as_double(0x7FF8000000000000ll);
        double x;
        if (translate_key(bits, a.is_f64, lo, inv, &x)) {
            F = model_fp32<H>(m, x);
            slot = slot_of(F, a.M);
        }
        if (a.slots_out) a.slots_out[i] = slot;
        if (a.F_out) a.F_out[i] = F;
    }
}

// Sum over sorted positions p of |F_p n - p| for mappable keys (F not NaN):
// how far the model's expected position is from the true rank.
__global__ void __launch_bounds__(256) k_pos_err(const double* __restrict__ F, int64_t n, double* sum,
                                                 unsigned long long* count) {
    __shared__ double s_sum[256];
    __shared__ unsigned long long s_cnt[256];
    double acc = 0.0;
    unsigned long long c = 0;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        double f = F[p];
        if (f == f) {
            acc += fabs(f * (double)n - (double)p);
            ++c;
        }
    }
    s_sum[threadIdx.x] = acc;
    s_cnt[threadIdx.x] = c;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < (unsigned)off) {
            s_sum[threadIdx.x] += s_sum[threadIdx.x + off];
            s_cnt[threadIdx.x] += s_cnt[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(sum, s_sum[0]);
        atomicAdd(count, s_cnt[0]);
    }
}

hipError_t launch_pos_err_sum(const double* d_F, int64_t n, double* d_sum, hipStream_t st) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_pos_err, dim3((unsigned)blocks), dim3(256), 0, st, d_F, n, d_sum,
                       (unsigned long long*)(d_sum + 1));
    return hipGetLastError();
}

hipError_t launch_bf16_infer(const InferArgs& a, int H, int bf16_terms, bool scaled, hipStream_t st);
hipError_t launch_pwl_infer(const InferArgs& a, int H, hipStream_t st);

static int grid_for(int64_t n, int threads, int max_blocks) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return (int)b;
}

hipError_t launch_infer(const InferArgs& a, int H, int form, int bf16_terms, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    if (form == NNSORT_FORM_BF16) return launch_bf16_infer(a, H, bf16_terms, a.bf16_scaled != 0, st);
    if (form == NNSORT_FORM_PWL) return launch_pwl_infer(a, H, st);
    int grid = grid_for(a.n, 256, 256 * 64);
    if (H == 32)
        hipLaunchKernelGGL(k_infer_fp32<32>, dim3(grid), dim3(256), 0, st, a);
    else if (H == 64)
        hipLaunchKernelGGL(k_infer_fp32<64>, dim3(grid), dim3(256), 0, st, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace nns
