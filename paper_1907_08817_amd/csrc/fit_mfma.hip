// One training step of the fit (Sec. 2, Training) on the FP32 matrix cores,
// for widths H = 32 and 64: the batch draw, the forward pass, the loss, the
// backward pass and each workgroup's partial gradient in one kernel, so no
// activation goes through memory; then one kernel that adds the partial
// gradients in a fixed order, keeps the parameters when the batch loss is the
// lowest so far, and applies the Adam step.
//
// A wave maps 32 batch entries at a time (lane l: entry n = l % 32, lane half
// g = l / 32).  The three products of a step run on v_mfma_f32_32x32x2_f32
// (32 x 32 output, two terms of the sum per instruction, FP32):
//   forward   Z2^T [H x 32]  = W2    [H x H] * H1^T  [H x 32]
//   backward  dZ1^T[H x 32]  = W2^T  [H x H] * dZ2^T [H x 32]
//   weights   dW2  [H x H]  += dZ2^T [H x 32] * H1   [32 x H]
// In the first two the entries are the N dimension: lane (n, g) holds, in
// accumulator slot v of row block r, unit u(q, g) = 32 r + 8 (v / 4) + 4 g +
// v % 4 of entry n (q = 16 r + v).  Their sums run over units in the order
// k-step q, term g: the lane's own activation at slot q is its B operand, so
// neither product needs data from another lane, and the activation a lane
// feeds in at step q is the one the other product returns at slot q.  The
// weight product sums over entries, so its operands are transposed through
// LDS (entry-major rows), which also serve the vector gradients.
//
// A workgroup holds eight waves (two per SIMD, so one wave's matrix work
// overlaps the other's vector and LDS work) and one LDS copy of the
// parameters, read by both W2 products; apart from that copy each wave works
// on its own tiles and LDS arrays, ordered by waits on its own LDS traffic,
// so only the parameter load and the final reduction use workgroup barriers.
// A 65,536-entry batch is one 32-entry tile per wave over 256 workgroups.
//
// Every sum has a fixed order, so a step does not depend on scheduling.  The
// products are FP32 with the matrix cores' accumulation order (not the FP32
// form's FMA chains); F is accumulated in FP64.
// Compiled with -ffp-contract=off.
#include "fit_common.h"

namespace nns {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kStepWaves = 8;
constexpr int kMaxStepGroups = 256;  // partial rows per step

struct FitStepArgs {
    const float* th;       // parameters theta (packed)
    const double* x;       // the fit sample's translated keys
    const float* y;        // their labels
    int64_t k;             // sample size
    int64_t B;             // batch size
    uint64_t seed;
    int64_t step;          // 1-based
    int loss;              // 0 MSE, 1 Huber
    float delta;
    float* part;           // out: one partial gradient row of P floats per workgroup
    float* loss_part;      // out: one partial loss sum per workgroup
};

// Hidden unit at accumulator slot q of lane half g (see above).
__host__ __device__ __forceinline__ int slot_unit(int q, int g) {
    return 32 * (q >> 4) + 8 * ((q & 15) >> 2) + 4 * g + (q & 3);
}

// Orders a wave's LDS stores before its later LDS loads (and the reverse):
// the wave's own LDS operations complete in issue order, so it is enough to
// drain them and keep the compiler from moving memory accesses across.
__device__ __forceinline__ void wave_lds_sync() { __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

template <int H>
__global__ void __launch_bounds__(64 * kStepWaves) k_fit_step(FitStepArgs a) {
    constexpr int RB = H / 32;     // 32-row blocks
    constexpr int NQ = H / 2;      // accumulator slots per lane = k-steps of an H-deep product
    constexpr int P = H * H + 4 * H + 1;
    constexpr int LD = H + 1;      // padded rows
    static_assert(NQ == 16 * RB, "slots");
    // W2 row-major: the forward product's A operand at (row block r, k-step
    // q, lane (n, g)) is W2[32 r + n][u(q, g)], the backward one's
    // W2[u(q, g)][32 r + n]
    __shared__ float sW2[H * LD];
    // per-slot vectors, [lane half][slot]
    __shared__ float sw1[2][NQ], sb1[2][NQ], sb2[2][NQ], sw3f[2][NQ];
    __shared__ double sw3[2][NQ];
    // per-wave transposes: two entry-major [32][H] arrays, then the entries'
    // x; reused by the final reduction
    __shared__ float str[kStepWaves][2][32][LD];
    __shared__ float sx[kStepWaves][32];
    __shared__ float svec[kStepWaves][4][H];
    __shared__ float sscal[kStepWaves][2];

    const float* __restrict__ th = a.th;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, n = lane & 31, g = lane >> 5;
    const int64_t tiles = (a.B + 31) / 32;
    const int64_t per_round = (int64_t)gridDim.x * kStepWaves;
    const int64_t rounds = (tiles + per_round - 1) / per_round;
    // batch entry b of round rd: draw its sample index and load (x, y)
    auto fetch = [&](int64_t rd, double& xv, float& yv) {
        const int64_t b = ((rd * gridDim.x + blockIdx.x) * kStepWaves + w) * 32 + n;
        xv = 0.0;
        yv = 0.0f;
        if (b < a.B) {
            const uint64_t j = rand64(a.seed, kStreamBatch, (uint64_t)b, (uint32_t)a.step) % (uint64_t)a.k;
            xv = a.x[j];
            yv = a.y[j];
        }
    };
    // the thread's W2 loads go out first, the batch draw runs while they are
    // in flight, then the first entry's loads follow before any LDS store
    const float* W2 = th + 2 * H;
    double xv;
    float yv;
    {
        constexpr int kPer = (H * H + 64 * kStepWaves - 1) / (64 * kStepWaves);
        float v[kPer];
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = tid + 64 * kStepWaves * i;
            v[i] = e < H * H ? W2[e] : 0.0f;
        }
        fetch(0, xv, yv);
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = tid + 64 * kStepWaves * i;
            if (e < H * H) sW2[(e / H) * LD + e % H] = v[i];
        }
    }
    for (int e = tid; e < 2 * NQ; e += 64 * kStepWaves) {
        const int gg = e / NQ, q = e % NQ, u = slot_unit(q, gg);
        sw1[gg][q] = th[u];
        sb1[gg][q] = th[H + u];
        sb2[gg][q] = th[2 * H + H * H + u];
        sw3f[gg][q] = th[3 * H + H * H + u];
        sw3[gg][q] = (double)th[3 * H + H * H + u];
    }
    __syncthreads();
    const float b3 = th[4 * H + H * H];
    const float invB = 1.0f / (float)a.B;
    // lane bases of the A operands (the k-step and row block add constants)
    const float* Af = &sW2[n * LD + 4 * g];
    const float* Ab = &sW2[4 * g * LD + n];

    floatx16 accW[RB][RB];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < RB; ++c)
#pragma unroll
            for (int v = 0; v < 16; ++v) accW[r][c][v] = 0.0f;
    float vdb2[RB], vdw3[RB], vdb1[RB], vdw1[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) vdb2[r] = vdw3[r] = vdb1[r] = vdw1[r] = 0.0f;
    float vdb3 = 0.0f, vloss = 0.0f;

    float* T0 = &str[w][0][0][0];
    float* T1 = &str[w][1][0][0];
    // the waves share only the parameters in LDS, so each runs its rounds on
    // its own (entries past the batch contribute nothing)
    for (int64_t rd = 0; rd < rounds; ++rd) {
        const bool ok = ((rd * gridDim.x + blockIdx.x) * kStepWaves + w) * 32 + n < a.B;
        const float xh = (float)xv;
        const float xl = (float)(xv - (double)xh);
        const float ycur = yv;
        if (rd + 1 < rounds) fetch(rd + 1, xv, yv);  // the next round's entry, in flight meanwhile

        // ---- forward: h1 at each slot, z2 = W2 h1 + b2 on the matrix cores
        floatx16 acc[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[r][v] = sb2[g][16 * r + v];
        float h1[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            float z = __builtin_fmaf(sw1[g][q], xh, sb1[g][q]);
            z = __builtin_fmaf(sw1[g][q], xl, z);
            h1[q] = z > 0.0f ? z : 0.0f;
            const int cu = slot_unit(q, 0);
#pragma unroll
            for (int r = 0; r < RB; ++r)
                acc[r] = __builtin_amdgcn_mfma_f32_32x32x2f32(Af[32 * r * LD + cu], h1[q], acc[r], 0, 0, 0);
        }
        // ---- h2, F (FP64 sum over the lane's units, then the two halves), loss
        float h2[NQ];
        double s = g == 0 ? (double)b3 : 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const float z = acc[q >> 4][q & 15];
            h2[q] = z > 0.0f ? z : 0.0f;
            s = __builtin_fma(sw3[g][q], (double)h2[q], s);
        }
        const double F = s + __shfl_xor(s, 32);
        float gv = 0.0f;
        if (ok) {
            float gg;
            const float l = loss_term((float)F - ycur, a.loss, a.delta, gg);
            gv = gg * invB;
            if (g == 0) {
                vloss += l;
                vdb3 += gv;
            }
        }
        // ---- backward: dz2 = g w3 [h2 > 0]; h1 and dz2 transposed for dW2
        float dz2[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            dz2[q] = h2[q] > 0.0f ? gv * sw3f[g][q] : 0.0f;
            const int u = slot_unit(q, g);
            T0[n * LD + u] = h1[q];
            T1[n * LD + u] = dz2[q];
        }
        // dz1 = W2^T dz2 on the matrix cores, masked by h1 > 0 (slot q of the
        // output is the unit whose h1 the lane computed at step q)
        floatx16 acc1[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc1[r][v] = 0.0f;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int cu = slot_unit(q, 0);
#pragma unroll
            for (int r = 0; r < RB; ++r)
                acc1[r] = __builtin_amdgcn_mfma_f32_32x32x2f32(Ab[cu * LD + 32 * r], dz2[q], acc1[r], 0, 0, 0);
        }
        wave_lds_sync();
        // dW2 += dz2^T h1 over the 32 entries, two per step (lane: unit
        // 32 r + l % 32 of entry 2 p + g); db2 from the same reads
#pragma unroll
        for (int p = 0; p < 16; ++p) {
            const int e = 2 * p + g;
            float av[RB], bv[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                av[r] = T1[e * LD + 32 * r + n];
                bv[r] = T0[e * LD + 32 * r + n];
                vdb2[r] += av[r];
            }
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int c = 0; c < RB; ++c)
                    accW[r][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[r], bv[c], accW[r][c], 0, 0, 0);
        }
        wave_lds_sync();
        // ---- vector gradients: g h2 and dz1 transposed, with x
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int u = slot_unit(q, g);
            T0[n * LD + u] = gv * h2[q];
            T1[n * LD + u] = h1[q] > 0.0f ? acc1[q >> 4][q & 15] : 0.0f;
        }
        if (g == 0) sx[w][n] = xh;
        wave_lds_sync();
#pragma unroll 4
        for (int p = 0; p < 16; ++p) {
            const int e = 2 * p + g;
            const float xe = sx[w][e];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const float d1 = T1[e * LD + 32 * r + n];
                vdb1[r] += d1;
                vdw1[r] = __builtin_fmaf(d1, xe, vdw1[r]);
                vdw3[r] += T0[e * LD + 32 * r + n];
            }
        }
        wave_lds_sync();
    }

    // ---- the workgroup's partial gradient: waves in order, lane halves added
    float* row = a.part + (int64_t)blockIdx.x * P;
    float* Wsum = &str[w][0][0][0];  // H * H <= 2 * 32 * LD floats
    static_assert(H * H <= 2 * 32 * LD, "a wave's dW2 fits its transpose arrays");
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < RB; ++c)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int i = 32 * r + 8 * (v >> 2) + 4 * g + (v & 3);
                Wsum[i * H + 32 * c + n] = accW[r][c][v];
            }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const float d1 = vdw1[r] + __shfl_xor(vdw1[r], 32);
        const float e1 = vdb1[r] + __shfl_xor(vdb1[r], 32);
        const float e2 = vdb2[r] + __shfl_xor(vdb2[r], 32);
        const float d3 = vdw3[r] + __shfl_xor(vdw3[r], 32);
        if (g == 0) {
            svec[w][0][32 * r + n] = d1;
            svec[w][1][32 * r + n] = e1;
            svec[w][2][32 * r + n] = e2;
            svec[w][3][32 * r + n] = d3;
        }
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        vdb3 += __shfl_xor(vdb3, off);
        vloss += __shfl_xor(vloss, off);
    }
    if (lane == 0) {
        sscal[w][0] = vdb3;
        sscal[w][1] = vloss;
    }
    __syncthreads();
    for (int e = tid; e < H * H; e += 64 * kStepWaves) {
        float t = 0.0f;
#pragma unroll
        for (int ww = 0; ww < kStepWaves; ++ww) t += (&str[ww][0][0][0])[e];
        row[2 * H + e] = t;
    }
    for (int e = tid; e < 4 * H; e += 64 * kStepWaves) {
        const int kind = e / H, u = e % H;
        float t = 0.0f;
#pragma unroll
        for (int ww = 0; ww < kStepWaves; ++ww) t += svec[ww][kind][u];
        const int at = kind == 0 ? u : kind == 1 ? H + u : kind == 2 ? 2 * H + H * H + u : 3 * H + H * H + u;
        row[at] = t;
    }
    if (tid == 0) {
        float t = 0.0f, l = 0.0f;
#pragma unroll
        for (int ww = 0; ww < kStepWaves; ++ww) {
            t += sscal[ww][0];
            l += sscal[ww][1];
        }
        row[P - 1] = t;
        a.loss_part[blockIdx.x] = l;
    }
}

// The step's update: the batch loss (the workgroups' partial sums added in a
// fixed order, over B), the keep-best test against the lowest loss before this
// step (best_loss[(t - 1) & 1]; workgroup 0 writes best_loss[t & 1]), the copy
// of the parameters to `best` when this loss is lower, then each parameter's
// gradient (its column of the partial rows, fixed order) into one Adam step.
// A workgroup takes 8 columns; 32 row groups add rows grp, grp + 32, ...
constexpr int kUpdCols = 8, kUpdGroups = 32;
__global__ void __launch_bounds__(kUpdCols * kUpdGroups) k_fit_update(const float* __restrict__ part, int rows, int P,
                                                                      const float* __restrict__ loss_part, int64_t B,
                                                                      int64_t t, float* th, float* m1, float* m2,
                                                                      float b1, float b2, float c1, float c2, float lr,
                                                                      float eps, float* best, float* best_loss,
                                                                      float* loss_out) {
    __shared__ float s[kUpdGroups][kUpdCols];
    __shared__ float s_part[kMaxStepGroups];
    __shared__ int better;
    const int tid = threadIdx.x;
    for (int i = tid; i < kMaxStepGroups; i += blockDim.x) s_part[i] = i < rows ? loss_part[i] : 0.0f;
    const int c = tid % kUpdCols, grp = tid / kUpdCols;
    const int p = blockIdx.x * kUpdCols + c;
    // the parameter's state and the lowest loss so far, loaded alongside the rows
    const bool mine = grp == 0 && p < P;
    float th_p = mine ? th[p] : 0.0f, m1_p = mine ? m1[p] : 0.0f, m2_p = mine ? m2[p] : 0.0f;
    const float prev = best_loss[(t - 1) & 1];
    // every row load of the thread in flight at once, then added in row order
    constexpr int kRowsPer = kMaxStepGroups / kUpdGroups;
    float v[kRowsPer];
#pragma unroll
    for (int i = 0; i < kRowsPer; ++i) {
        const int r = grp + kUpdGroups * i;
        v[i] = (p < P && r < rows) ? part[(int64_t)r * P + p] : 0.0f;
    }
    float acc = 0.0f;
#pragma unroll
    for (int i = 0; i < kRowsPer; ++i) acc += v[i];
    s[grp][c] = acc;
    __syncthreads();
    if (tid < 32) {  // the loss: 32 runs of consecutive partials, then a butterfly over the 32 run sums
        float q = 0.0f;
        for (int i = 0; i < kMaxStepGroups / 32; ++i) q += s_part[(kMaxStepGroups / 32) * tid + i];
        float L = q;
        for (int off = 1; off < 32; off <<= 1) L += __shfl_xor(L, off, 32);
        if (tid == 0) {
            L /= (float)B;
            better = L < prev ? 1 : 0;
            if (blockIdx.x == 0) {
                loss_out[0] = L;
                best_loss[t & 1] = better ? L : prev;
            }
        }
    }
    __syncthreads();
    if (mine) {
        float gsum = 0.0f;
        for (int i = 0; i < kUpdGroups; ++i) gsum += s[i][c];
        if (better) best[p] = th_p;
        adam_step(gsum, th_p, m1_p, m2_p, b1, b2, c1, c2, lr, eps);
        m1[p] = m1_p;
        m2[p] = m2_p;
        th[p] = th_p;
    }
}

// Column sums of the partial rows into gtheta (fixed order).
__global__ void __launch_bounds__(8 * kSumCols) k_grad_sums(const float* __restrict__ part, int rows, int P,
                                                            float* out) {
    __shared__ float s[8][kSumCols];
    const int c = threadIdx.x % kSumCols, grp = threadIdx.x / kSumCols;
    const int p = blockIdx.x * kSumCols + c;
    const float t = column_sum(part, rows, P, p, c, grp, s);
    if (grp == 0 && p < P) out[p] = t;
}

// The batch loss: the workgroups' partial sums in order, over B.
__global__ void k_loss_total(const float* __restrict__ loss_part, int rows, int64_t B, float* loss_out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        float L = 0.0f;
        for (int i = 0; i < rows; ++i) L += loss_part[i];
        loss_out[0] = L / (float)B;
    }
}

// Workgroups of one step: at most 256 (partial rows), one 32-entry tile per
// wave up to a 65,536 batch.
int fit_step_groups(int64_t B) {
    const int64_t tiles = (B + 31) / 32;
    int64_t g = (tiles + kStepWaves - 1) / kStepWaves;
    if (g > kMaxStepGroups) g = kMaxStepGroups;
    return (int)(g < 1 ? 1 : g);
}

bool fit_step_mfma(int H) { return H == 32 || H == 64; }

// One fused training step t (1-based) for H = 32 or 64.  part: 256 x P
// floats; loss_part: 256 floats; best_loss: two floats (slot 0 = +inf before
// step 1).
hipError_t launch_fit_step_mfma(int H, float* d_theta, const double* d_x, const float* d_y, int64_t k, int64_t B,
                                uint64_t seed, int64_t t, int loss, float delta, float lr, float b1, float b2,
                                float eps, float* d_part, float* d_loss_part, float* d_m1, float* d_m2, float* d_best,
                                float* d_best_loss, float* d_loss, hipStream_t st) {
    const int G = fit_step_groups(B);
    const int P = H * H + 4 * H + 1;
    FitStepArgs a{d_theta, d_x, d_y, k, B, seed, t, loss, delta, d_part, d_loss_part};
    if (H == 64)
        hipLaunchKernelGGL(k_fit_step<64>, dim3(G), dim3(64 * kStepWaves), 0, st, a);
    else if (H == 32)
        hipLaunchKernelGGL(k_fit_step<32>, dim3(G), dim3(64 * kStepWaves), 0, st, a);
    else
        return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const float c1 = (float)(1.0 - pow((double)b1, (double)t));
    const float c2 = (float)(1.0 - pow((double)b2, (double)t));
    hipLaunchKernelGGL(k_fit_update, dim3((P + kUpdCols - 1) / kUpdCols), dim3(kUpdCols * kUpdGroups), 0, st, d_part,
                       G, P, d_loss_part, B, t, d_theta, d_m1, d_m2, b1, b2, c1, c2, lr, eps, d_best, d_best_loss,
                       d_loss);
    return hipGetLastError();
}

// One fused step's gradient and loss without the update (a test hook: the
// same kernel as the fit's step, then plain column sums).
hipError_t launch_fit_gradient(int H, const float* d_theta, const double* d_x, const float* d_y, int64_t k,
                               int64_t B, uint64_t seed, int64_t t, int loss, float delta, float* d_part,
                               float* d_loss_part, float* d_gtheta, float* d_loss, hipStream_t st) {
    const int G = fit_step_groups(B);
    const int P = H * H + 4 * H + 1;
    FitStepArgs a{d_theta, d_x, d_y, k, B, seed, t, loss, delta, d_part, d_loss_part};
    if (H == 64)
        hipLaunchKernelGGL(k_fit_step<64>, dim3(G), dim3(64 * kStepWaves), 0, st, a);
    else if (H == 32)
        hipLaunchKernelGGL(k_fit_step<32>, dim3(G), dim3(64 * kStepWaves), 0, st, a);
    else
        return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_grad_sums, dim3((P + kSumCols - 1) / kSumCols), dim3(8 * kSumCols), 0, st, d_part, G, P,
                       d_gtheta);
    hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(256), 0, st, d_loss_part, G, B, d_loss);
    return hipGetLastError();
}

}  // namespace nns
