// On-device fit of the CDF model (Sec. 2, Training; Sec. 4.1, Training
// details: a regression network trained with Adam, here on the normalised rank
// of a random sample of the keys).
//
// Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC
// 2011) keyed by the seed: stream 1 draws the sample, stream 2 the uniform
// initial weights, stream 3 the batches.  The forward pass uses the FP32
// form's operation order; the backward pass is hand-written: per-sample
// deltas, then batch reductions in fixed blocks summed in a fixed order, so a
// gradient does not depend on scheduling.  This translation unit is compiled
// with -ffp-contract=off.
#include "fit_common.h"

namespace nns {


// Sample k keys with replacement; keep the finite ones (order keys) in G.
// Each workgroup draws kSampleItems x 256 keys and reserves their place in G
// with one atomic; the order of G is arbitrary (it is sorted next).
constexpr int kSampleItems = 8;
__global__ void __launch_bounds__(256) k_sample(const uint64_t* __restrict__ in, int64_t n, int is_f64,
                                                uint64_t seed, int64_t k, uint64_t* out,
                                                unsigned long long* count) {
    __shared__ uint32_t s_w[4];
    __shared__ unsigned long long s_base;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t per_block = 256 * kSampleItems;
    for (int64_t base = (int64_t)blockIdx.x * per_block; base < k; base += (int64_t)gridDim.x * per_block) {
        uint64_t okey[kSampleItems];
        uint32_t okm = 0;
#pragma unroll
        for (int q = 0; q < kSampleItems; ++q) {
            const int64_t j = base + q * 256 + tid;
            okey[q] = 0;
            if (j < k) {
                const uint64_t r = rand64(seed, kStreamSample, (uint64_t)j, 0);
                const uint64_t bits = in[r % (uint64_t)n];
                const bool ok = !is_f64 || (bits & 0x7FF0000000000000ull) != 0x7FF0000000000000ull;
                okey[q] = order_key(bits, is_f64);
                okm |= ok ? 1u << q : 0u;
            }
        }
        const uint32_t c = (uint32_t)__popc(okm);
        uint32_t inc = c;  // inclusive prefix over the wave
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(inc, o);
            if (lane >= o) inc += y;
        }
        if (lane == 63) s_w[wv] = inc;
        __syncthreads();
        if (tid == 0) s_base = atomicAdd(count, (unsigned long long)(s_w[0] + s_w[1] + s_w[2] + s_w[3]));
        __syncthreads();
        unsigned long long pos = s_base + (inc - c);
        for (int w = 0; w < wv; ++w) pos += s_w[w];
#pragma unroll
        for (int q = 0; q < kSampleItems; ++q)
            if ((okm >> q) & 1u) out[pos++] = okey[q];
        __syncthreads();  // s_w and s_base are rewritten by the next round
    }
}

__device__ __forceinline__ double key_value(uint64_t okey, int is_f64) {
    const uint64_t bits = order_key_inverse(okey, is_f64);
    return is_f64 ? __longlong_as_double((long long)bits) : __ull2double_rn(bits);
}

// Training inputs: x_j = clamp((key_j - lo) * inv, 0, 1), y_j = (j + 0.5)/k,
// with lo and hi the sample's extremes (its first and last sorted keys) and
// inv = 1 / (hi - lo) (0 if they are equal); lohi receives (lo, inv) for the
// model the host returns.
__global__ void __launch_bounds__(256) k_make_xy(const uint64_t* __restrict__ sorted_okeys, int64_t k, int is_f64,
                                                 double* x, float* y, double* lohi) {
    const double lo = key_value(sorted_okeys[0], is_f64), hi = key_value(sorted_okeys[k - 1], is_f64);
    const double inv = hi > lo ? 1.0 / (hi - lo) : 0.0;
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j == 0) {
        lohi[0] = lo;
        lohi[1] = inv;
    }
    if (j >= k) return;
    double t = (key_value(sorted_okeys[j], is_f64) - lo) * inv;
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    x[j] = t;
    y[j] = (float)(((double)j + 0.5) / (double)k);
}

// ---- knots of the piecewise-linear CDF interpolant ----
// Greedy maximum-deviation splitting over the sorted sample x[0..k) with ranks
// y_j = (j + 0.5)/k: split the piece whose points lie farthest (in rank) from
// the chord between its ends, at the farthest point, until H pieces.  Ties:
// larger deviation first, then the smaller start / smaller point index.  A
// piece with < 3 points, zero width, or no point more than 1/k off its chord
// is final.
// Each split rescans only the two new pieces.  A scan is spread over
// kKnotBlocks workgroups per piece, each keeping its first largest deviation
// (the reduction prefers the larger deviation, then the smaller index, so
// the result is the first maximum whatever the split into blocks).  Split t
// is one launch: every workgroup first applies the previous scan's result to
// its own LDS copy of the piece table (all copies come out identical, and
// workgroup 0 stores its copy for the next launch), then scans its share of
// the two pieces the table names.  State and partial results alternate
// between two buffers, so a launch never writes what it reads.  The host
// launches H steps and a finish that applies the last result; once no piece
// can be split, the steps only carry the table over.
constexpr int kKnotBlocks = 256;
constexpr int kKnotThreads = 256;

struct KnotState {
    int32_t np, best, done, pad;
    int64_t ra[2], rb[2];  // the two pieces the next scan covers
    int64_t pa[NNSORT_MAX_HIDDEN], pb[NNSORT_MAX_HIDDEN], pj[NNSORT_MAX_HIDDEN];
    double pd[NNSORT_MAX_HIDDEN];
};
struct KnotWork {
    KnotState s[2];
    double part_d[2][2][kKnotBlocks];
    int64_t part_j[2][2][kKnotBlocks];
};
static_assert(sizeof(KnotState) % 8 == 0, "copied as 64-bit words");

size_t knot_ws_bytes() { return sizeof(KnotWork); }

__device__ __forceinline__ double rank_of(int64_t j, int64_t k) { return ((double)j + 0.5) / (double)k; }

// (d, j) pairs: larger deviation wins, then the smaller valid index.
__device__ __forceinline__ void arg_max_reduce(double* s_d, int64_t* s_j) {
    for (int off = kKnotThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < (unsigned)off) {
            const double d2 = s_d[threadIdx.x + off];
            const int64_t j2 = s_j[threadIdx.x + off];
            const double d1 = s_d[threadIdx.x];
            const int64_t j1 = s_j[threadIdx.x];
            if (d2 > d1 || (d2 == d1 && j2 >= 0 && (j1 < 0 || j2 < j1))) {
                s_d[threadIdx.x] = d2;
                s_j[threadIdx.x] = j2;
            }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ void copy_state(KnotState* dst, const KnotState* src) {
    const uint64_t* a = (const uint64_t*)src;
    uint64_t* b = (uint64_t*)dst;
    for (int i = threadIdx.x; i < (int)(sizeof(KnotState) / 8); i += blockDim.x) b[i] = a[i];
}

__global__ void k_knot_start(int64_t k, KnotWork* w) {
    if (threadIdx.x != 0) return;
    KnotState& S = w->s[0];
    S.np = 0;
    S.best = -1;
    S.done = 0;
    S.ra[0] = 0;
    S.rb[0] = k - 1;
    S.ra[1] = 0;  // no second piece in the first scan
    S.rb[1] = 0;
}

// Apply a scan's result (per piece r, kKnotBlocks partial (d, j)) to the
// table S in LDS: the first piece, or the split of the chosen one; then
// choose the next piece to split: the valid piece (a split point, a positive
// deviation) of largest deviation, ties to the leftmost start.  Piece starts
// are distinct, so that order is strict and a butterfly over one wave finds
// the same piece as a scan in index order.  All kKnotThreads threads call it.
__device__ void knot_apply(int64_t k, int H, KnotState& S, const double (*part_d)[kKnotBlocks],
                           const int64_t (*part_j)[kKnotBlocks], double* s_d, int64_t* s_j) {
    static_assert(kKnotBlocks == kKnotThreads, "one thread per scan block");
    static_assert(NNSORT_MAX_HIDDEN <= 64, "one lane per piece");
    __shared__ double r_d[2];
    __shared__ int64_t r_j[2];
    if (S.done) return;
    const int t = threadIdx.x;
    for (int r = 0; r < 2; ++r) {
        s_d[t] = part_d[r][t];
        s_j[t] = part_j[r][t];
        __syncthreads();
        arg_max_reduce(s_d, s_j);
        if (t == 0) {
            double d = s_d[0];
            int64_t j = s_j[0];
            if (!(d > 1.0 / (double)k)) {  // within one rank step of linear: final
                d = 0.0;
                j = -1;
            }
            r_d[r] = d;
            r_j[r] = j;
        }
        __syncthreads();
    }
    if (t == 0) {
        const int np0 = S.np;
        int np = np0;
        if (np == 0) {
            S.pa[0] = 0;
            S.pb[0] = k - 1;
            np = 1;
        } else {
            const int bst = S.best;
            const int64_t b = S.pb[bst], sj = S.pj[bst];
            S.pb[bst] = sj;
            S.pa[np] = sj;
            S.pb[np] = b;
            S.pd[bst] = r_d[0];
            S.pj[bst] = r_j[0];
            ++np;
        }
        const int nw = np - 1;  // the new piece (or the first one)
        S.pd[nw] = r_d[np0 == 0 ? 0 : 1];
        S.pj[nw] = r_j[np0 == 0 ? 0 : 1];
        S.np = np;
    }
    __syncthreads();
    if (t < 64) {
        const int np = S.np;
        const bool ok = np < H && t < np && S.pj[t] >= 0 && S.pd[t] > 0.0;
        double d = ok ? S.pd[t] : 0.0;
        int64_t a = ok ? S.pa[t] : 0;
        int best = ok ? t : -1;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double d2 = __shfl_xor(d, off);
            const int64_t a2 = __shfl_xor(a, off);
            const int b2 = __shfl_xor(best, off);
            if (b2 >= 0 && (best < 0 || d2 > d || (d2 == d && a2 < a))) {
                d = d2;
                a = a2;
                best = b2;
            }
        }
        if (t == 0) {
            S.best = best;
            if (best < 0) {
                S.done = 1;
            } else {
                S.ra[0] = S.pa[best];
                S.rb[0] = S.pj[best];
                S.ra[1] = S.pj[best];
                S.rb[1] = S.pb[best];
            }
        }
    }
    __syncthreads();
}

// Split t: block (blockIdx.x, r = blockIdx.y) applies split t - 1's result
// (t > 0), then scans its share of the points a+1 .. b-1 of piece r.
__global__ void __launch_bounds__(kKnotThreads) k_knot_step(const double* __restrict__ x, int64_t k, int H, int t,
                                                            KnotWork* w) {
    __shared__ KnotState S;
    __shared__ double s_d[kKnotThreads];
    __shared__ int64_t s_j[kKnotThreads];
    copy_state(&S, &w->s[t == 0 ? 0 : (t - 1) & 1]);
    __syncthreads();
    if (t > 0) {
        knot_apply(k, H, S, w->part_d[(t - 1) & 1], w->part_j[(t - 1) & 1], s_d, s_j);
        if (blockIdx.x == 0 && blockIdx.y == 0) copy_state(&w->s[t & 1], &S);
    }
    if (S.done) return;
    const int r = blockIdx.y;
    const int64_t a = S.ra[r], b = S.rb[r];
    double best = -1.0;
    int64_t bj = -1;
    if (b - a >= 2) {
        const double xa = x[a], xb = x[b];
        if (xb != xa) {
            const double ya = rank_of(a, k), yb = rank_of(b, k);
            const int64_t stride = (int64_t)gridDim.x * kKnotThreads;
            for (int64_t j = a + 1 + (int64_t)blockIdx.x * kKnotThreads + threadIdx.x; j < b; j += stride) {
                const double lin = ya + ((yb - ya) * (x[j] - xa)) / (xb - xa);
                const double d = fabs(rank_of(j, k) - lin);
                if (d > best) {
                    best = d;
                    bj = j;
                }
            }
        }
    }
    s_d[threadIdx.x] = best;
    s_j[threadIdx.x] = bj;
    __syncthreads();
    arg_max_reduce(s_d, s_j);
    if (threadIdx.x == 0) {
        w->part_d[t & 1][r][blockIdx.x] = s_d[0];
        w->part_j[t & 1][r][blockIdx.x] = s_j[0];
    }
}

// The last split's result applied (after steps 0 .. H - 1), then the piece
// starts in ascending order (distinct: each piece begins where its left
// neighbour ends) and the last sample index.
__global__ void __launch_bounds__(kKnotThreads) k_knot_finish(int64_t k, int H, KnotWork* __restrict__ w,
                                                              int64_t* knots) {
    __shared__ KnotState S;
    __shared__ double s_d[kKnotThreads];
    __shared__ int64_t s_j[kKnotThreads];
    __shared__ int64_t s_st[NNSORT_MAX_HIDDEN];
    copy_state(&S, &w->s[(H - 1) & 1]);
    __syncthreads();
    knot_apply(k, H, S, w->part_d[(H - 1) & 1], w->part_j[(H - 1) & 1], s_d, s_j);
    const int n = S.np;
    const int t = threadIdx.x;
    if (t < n) {
        const int64_t v = S.pa[t];
        int rk = 0;
        for (int i = 0; i < n; ++i) rk += S.pa[i] < v ? 1 : 0;
        s_st[rk] = v;
    }
    __syncthreads();
    if (t <= H) knots[t] = t < n ? s_st[t] : k - 1;
}

__global__ void k_quantile_knots(int64_t k, int H, int64_t* knots) {
    int i = threadIdx.x;
    if (i <= H) knots[i] = (int64_t)i * (k - 1) / H;
}

// Initial weights (packed theta of width H).
// init 1 / 2: ramps through the knots (q_i, F_i) of the sample CDF:
//   u_i = relu(s_i (x - q_i)), s_i = 1/max(q_{i+1} - q_i, 2^-40);
//   v_i = relu(1 - u_i);  F = F_H - sum_i (F_{i+1} - F_i) v_i.
// init 0: uniform(+-1/sqrt(fan_in)).
__global__ void k_init(float* theta, int H, int init, uint64_t seed, const double* __restrict__ x, int64_t k,
                       const int64_t* __restrict__ knots) {
    int P = H * H + 4 * H + 1;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        double v = 0.0;
        if (init == 1 || init == 2) {
            if (p < 2 * H) {
                int i = p < H ? p : p - H;
                double q0 = x[knots[i]], q1 = x[knots[i + 1]];
                double w = q1 - q0;
                w = w > 0x1p-40 ? w : 0x1p-40;
                double s = 1.0 / w;
                v = p < H ? s : -s * q0;
            } else if (p < 2 * H + H * H) {
                int e = p - 2 * H;
                v = (e / H == e % H) ? -1.0 : 0.0;
            } else if (p < 3 * H + H * H) {
                v = 1.0;
            } else if (p < 4 * H + H * H) {
                int i = p - 3 * H - H * H;
                v = -(rank_of(knots[i + 1], k) - rank_of(knots[i], k));
            } else {
                v = rank_of(knots[H], k);
            }
        } else {
            double bound = p < 2 * H ? 1.0 : 1.0 / sqrt((double)H);
            uint64_t r = rand64(seed, kStreamInit, (uint64_t)p, 0);
            double u = (double)(uint32_t)(r >> 40) * (1.0 / 16777216.0);
            v = bound * (2.0 * u - 1.0);
        }
        theta[p] = (float)v;
    }
}

// ---- forward (FP32 form order), saving h1 and h2 ----
__device__ __forceinline__ float two_sum_f(float a, float b, float& err) {
    float s = a + b;
    float bb = s - a;
    err = (a - (s - bb)) + (b - bb);
    return s;
}

template <int H>
__global__ void __launch_bounds__(256) k_fwd(const float* __restrict__ th, const double* __restrict__ x,
                                             int64_t B, float* F, float* saved) {
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const float* w1 = th;
    const float* b1 = th + H;
    const float* W2 = th + 2 * H;
    const float* b2 = th + 2 * H + H * H;
    const float* w3 = th + 3 * H + H * H;
    double xv = x[b];
    float xh = (float)xv;
    float xl = (float)(xv - (double)xh);
    float h1[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
        float z = __builtin_fmaf(w1[j], xh, b1[j]);
        z = __builtin_fmaf(w1[j], xl, z);
        h1[j] = z > 0.0f ? z : 0.0f;
    }
    float p = th[4 * H + H * H], s = 0.0f;
    // saved activations unit-major, saved[u * B + b] (h1 then h2): the
    // threads of a wave write consecutive addresses
    float* sh1 = saved ? saved + b : nullptr;
    // four outputs at a time: their FMA chains are independent, which keeps
    // the ALU busy at one wave per SIMD; each z_i still sums over j in order
    static_assert(H % 4 == 0, "outputs in groups of four");
    for (int i0 = 0; i0 < H; i0 += 4) {
        float z[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) z[q] = b2[i0 + q];
#pragma unroll
        for (int j = 0; j < H; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) z[q] = __builtin_fmaf(W2[(i0 + q) * H + j], h1[j], z[q]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = i0 + q;
            float h2 = z[q] > 0.0f ? z[q] : 0.0f;
            if (sh1) sh1[(int64_t)(H + i) * B] = h2;
            float pr = w3[i] * h2;
            float r = __builtin_fmaf(w3[i], h2, -pr);
            float e;
            p = two_sum_f(p, pr, e);
            s = s + (e + r);
        }
    }
    if (sh1) {
#pragma unroll
        for (int j = 0; j < H; ++j) sh1[(int64_t)j * B] = h1[j];
    }
    F[b] = p + s;
}

// One training step's batch, drawn and scored inside the fit's forward.
struct FitBatch {
    const float* y;   // labels of the sample
    int64_t k;        // sample size
    uint64_t seed;
    int64_t step;
    double* bx;       // out: the batch's inputs, for the backward
    int loss;         // 0 MSE, 1 Huber
    float delta;
    float* gF;        // out: dL/dF per batch entry
    float* partial;   // out: the loss summed over each workgroup's 64 entries
};


// The same forward pass for the fit, spread over four waves per 64 samples:
// wave q computes hidden-2 units [q H/4, (q+1) H/4) of its samples (lane =
// sample), each z2_i the same FMA chain over j in order as above; the
// activations meet in LDS and the compensated layer-3 sum runs over i in
// order as above.  h1, h2 and F are therefore the same bit for bit, with four
// times as many waves to cover latency.
//
// x is the fit sample and entry b of the batch is x[idx], idx = Philox(step,
// b) mod k (stream kStreamBatch); the kernel also writes bx, and in place of F
// the loss terms: dL/dF and one partial loss sum per 64 entries (a butterfly
// over the wave, so the order is fixed).
template <int H>
__global__ void __launch_bounds__(256) k_fwd_fit(const float* __restrict__ th, const double* __restrict__ x,
                                                 int64_t B, float* saved, FitBatch fb) {
    constexpr int Q = H / 4;  // hidden-2 units per wave
    __shared__ float s_h2[64][H + 1];
    // the wave index, known wave-uniform so that W2 is read by scalar loads
    const int lane = threadIdx.x & 63, q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t b = (int64_t)blockIdx.x * 64 + lane;
    const bool ok = b < B;
    const float* w1 = th;
    const float* b1 = th + H;
    const float* W2 = th + 2 * H;
    const float* b2 = th + 2 * H + H * H;
    const float* w3 = th + 3 * H + H * H;
    // wave 0 draws the entries and hands the inputs to the other waves
    __shared__ double s_x[64];
    float yv = 0.0f;
    if (q == 0) {
        double v = 0.0;
        if (ok) {
            const uint64_t j = rand64(fb.seed, kStreamBatch, (uint64_t)b, (uint32_t)fb.step) % (uint64_t)fb.k;
            v = x[j];
            yv = fb.y[j];
            fb.bx[b] = v;
        }
        s_x[lane] = v;
    }
    __syncthreads();
    const double xv = s_x[lane];
    const float xh = (float)xv;
    const float xl = (float)(xv - (double)xh);
    float h1[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
        float z = __builtin_fmaf(w1[j], xh, b1[j]);
        z = __builtin_fmaf(w1[j], xl, z);
        h1[j] = z > 0.0f ? z : 0.0f;
    }
    static_assert(Q % 4 == 0 || Q < 4, "outputs in groups of four");
    constexpr int G = Q < 4 ? Q : 4;
    for (int i0 = q * Q; i0 < (q + 1) * Q; i0 += G) {
        float z[G];
#pragma unroll
        for (int k = 0; k < G; ++k) z[k] = b2[i0 + k];
#pragma unroll
        for (int j = 0; j < H; ++j)
#pragma unroll
            for (int k = 0; k < G; ++k) z[k] = __builtin_fmaf(W2[(i0 + k) * H + j], h1[j], z[k]);
#pragma unroll
        for (int k = 0; k < G; ++k) {
            const float h2 = z[k] > 0.0f ? z[k] : 0.0f;
            s_h2[lane][i0 + k] = h2;
            if (saved && ok) saved[(int64_t)(H + i0 + k) * B + b] = h2;
        }
    }
    if (saved && ok) {  // h1: a quarter of the units per wave
#pragma unroll
        for (int j = 0; j < H; ++j)
            if (j / Q == q) saved[(int64_t)j * B + b] = h1[j];
    }
    __syncthreads();
    if (q != 0) return;
    float p = th[4 * H + H * H], s = 0.0f;
    for (int i = 0; i < H; ++i) {
        const float h2 = s_h2[lane][i];
        float pr = w3[i] * h2;
        float r = __builtin_fmaf(w3[i], h2, -pr);
        float e;
        p = two_sum_f(p, pr, e);
        s = s + (e + r);
    }
    const float Fb = p + s;
    float l = 0.0f;
    if (ok) {
        float g;
        l = loss_term(Fb - yv, fb.loss, fb.delta, g);
        fb.gF[b] = g * (1.0f / (float)B);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off);
    if (lane == 0) fb.partial[blockIdx.x] = l;
}

// ---- loss and dL/dF ----
constexpr int kLossBlocks = 256;
__global__ void __launch_bounds__(256) k_loss(const float* __restrict__ F, const float* __restrict__ y, int64_t B,
                                              int loss, float delta, float* gF, float* partial) {
    __shared__ float s[256];
    float acc = 0.0f;
    float invB = 1.0f / (float)B;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < B; b += (int64_t)gridDim.x * blockDim.x) {
        float g;
        const float l = loss_term(F[b] - y[b], loss, delta, g);
        gF[b] = g * invB;
        acc += l;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < (unsigned)off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

__global__ void __launch_bounds__(kLossBlocks) k_loss_final(const float* __restrict__ partial, int nb, int64_t B,
                                                          float* loss_out) {
    __shared__ float s_p[kLossBlocks];
    for (int i = threadIdx.x; i < nb; i += blockDim.x) s_p[i] = partial[i];  // nb <= kLossBlocks
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.0f;
        for (int i = 0; i < nb; ++i) s += s_p[i];
        loss_out[0] = s / (float)B;
    }
}

// The fit's loss total with the keep-best step: the nb partial sums of the
// step's forward are added in 256 groups of ceil(nb / 256) consecutive ones,
// those sums in 16 groups of 16, and those 16 in order (a fixed order); then
// the parameters are kept when this batch's loss is the lowest so far (a
// step's loss is measured before its update).
__global__ void __launch_bounds__(kLossBlocks) k_loss_final_keep(const float* __restrict__ partial, int nb,
                                                               int64_t B, float* loss_out,
                                                               const float* __restrict__ th, float* best, int P,
                                                               float* best_loss) {
    static_assert(kLossBlocks == 256, "16 groups of 16");
    __shared__ float s_p[kLossBlocks], s_q[16];
    __shared__ float s_l;
    __shared__ int better;
    {
        const int c = (nb + kLossBlocks - 1) / kLossBlocks;
        const int i0 = threadIdx.x * c, i1 = i0 + c < nb ? i0 + c : nb;
        float g = 0.0f;
        for (int i = i0; i < i1; ++i) g += partial[i];
        s_p[threadIdx.x] = g;
    }
    __syncthreads();
    if (threadIdx.x < 16) {
        float g = 0.0f;
        for (int i = 0; i < 16; ++i) g += s_p[16 * threadIdx.x + i];
        s_q[threadIdx.x] = g;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.0f;
        for (int i = 0; i < 16; ++i) s += s_q[i];
        const float l = s / (float)B;
        loss_out[0] = l;
        s_l = l;
        better = l < best_loss[0] ? 1 : 0;
    }
    __syncthreads();
    if (!better) return;
    for (int p = threadIdx.x; p < P; p += blockDim.x) best[p] = th[p];
    if (threadIdx.x == 0) best_loss[0] = s_l;
}

// ---- backward ----
// Per sample: dz2_i = g w3_i [h2_i > 0]; dz1_j = [h1_j > 0] sum_i dz2_i W2_ij,
// computed inside the batch reduction below from the saved (h1, h2).

// Batch reductions: block c sums samples [c*chunk, (c+1)*chunk) into its row
// of `part` (P floats): dW2_ij = sum dz2_i h1_j, dw3_i = sum g h2_i,
// db2 = sum dz2, dw1_j = sum dz1_j x, db1 = sum dz1, db3 = sum g.  Samples
// are staged in LDS 16 or 32 at a time; their dz2 and dz1 are formed there (W2 in
// LDS, each dz1_j one FMA chain over i in order), so they never go through
// memory.  dW2 is a product [H x chunk] x [chunk x H]: each thread keeps a
// T x T tile of it in registers (T = 4 at H = 64), two 16-byte LDS reads per
// sample for T^2 FMAs.  Every sum runs over the samples in order, so the
// result does not depend on scheduling.
constexpr int kRedChunk = 64;  // 1024 workgroups at a 65,536 batch
template <int H>
__global__ void __launch_bounds__(256) k_bwd_reduce(const float* __restrict__ th, const double* __restrict__ x,
                                                    int64_t B, const float* __restrict__ saved,
                                                    const float* __restrict__ gF, float* part) {
    constexpr int P = H * H + 4 * H + 1;
    // samples staged at a time: 16 keeps the workgroup at 32 KB of LDS at
    // H = 64, so that all 1024 workgroups of a 65,536 batch are resident at
    // once (five per CU; 32 samples need 48 KB, three per CU, and a second
    // round of workgroups)
    constexpr int kRedSub = H >= 32 ? 16 : 32;
    constexpr int T = H >= 64 ? 4 : (H >= 32 ? 2 : 1);  // tile edge
    constexpr int NBK = H / T;                          // tiles per dimension (<= 16)
    static_assert(NBK * NBK <= 256, "one tile per thread");
    // Rows padded against LDS bank conflicts: the staging writes put
    // consecutive samples in consecutive lanes, and the dz1 loop reads four
    // samples' dz2 at one unit.  sh1 and sdz2 rows stay 16-byte aligned for
    // the tile loop's vector reads.
    __shared__ __align__(16) float sh1[kRedSub][H + 4];
    __shared__ __align__(16) float sdz2[kRedSub][H + 4];
    __shared__ float sh2[kRedSub][H + 4], sdz1[kRedSub][H + 1];
    __shared__ float sW2[H][H];  // row i: hidden-2 unit i
    __shared__ float sw3[H];
    __shared__ float sx[kRedSub], sg[kRedSub];
    const int tid = threadIdx.x;
    for (int e = tid; e < H * H; e += 256) sW2[e / H][e % H] = th[2 * H + e];
    for (int e = tid; e < H; e += 256) sw3[e] = th[3 * H + H * H + e];
    // dz1 outputs per thread: kJ consecutive units of one sample
    constexpr int kJ = H * kRedSub / 256;
    static_assert(kJ >= 1 && H % kJ == 0, "dz1 outputs split evenly over the threads");
    const bool tile_on = tid < NBK * NBK;
    const int i0 = (tid / NBK) * T, j0 = (tid % NBK) * T;
    float acc[T][T];
#pragma unroll
    for (int a = 0; a < T; ++a)
#pragma unroll
        for (int c = 0; c < T; ++c) acc[a][c] = 0.0f;
    float accv = 0.0f;   // one of the 4H vector gradients per thread (tid < 4H)
    float accb3 = 0.0f;  // db3, thread 0
    const int64_t c0 = (int64_t)blockIdx.x * kRedChunk;
    for (int64_t s0 = c0; s0 < c0 + kRedChunk && s0 < B; s0 += kRedSub) {
        // unit-major sources: consecutive threads read consecutive samples
        for (int e = tid; e < kRedSub * H; e += 256) {
            int r = e % kRedSub, c = e / kRedSub;
            int64_t b = s0 + r;
            const bool ok = b < B;
            sh1[r][c] = ok ? saved[(int64_t)c * B + b] : 0.0f;
            sh2[r][c] = ok ? saved[(int64_t)(H + c) * B + b] : 0.0f;
        }
        if (tid < kRedSub) {
            int64_t b = s0 + tid;
            sx[tid] = b < B ? (float)x[b] : 0.0f;
            sg[tid] = b < B ? gF[b] : 0.0f;
        }
        __syncthreads();
        // dz2_i = g w3_i [h2_i > 0] (samples past B were staged as zeros)
        for (int e = tid; e < kRedSub * H; e += 256) {
            const int r = e / H, i = e % H;
            sdz2[r][i] = sh2[r][i] > 0.0f ? sg[r] * sw3[i] : 0.0f;
        }
        __syncthreads();
        // dz1_j = [h1_j > 0] sum_i dz2_i W2_ij, one FMA chain per output
        {
            const int r = tid / (H / kJ), j0 = (tid % (H / kJ)) * kJ;
            float a1[kJ];
#pragma unroll
            for (int q = 0; q < kJ; ++q) a1[q] = 0.0f;
            for (int i = 0; i < H; ++i) {
                const float dz = sdz2[r][i];
#pragma unroll
                for (int q = 0; q < kJ; ++q) a1[q] = __builtin_fmaf(dz, sW2[i][j0 + q], a1[q]);
            }
#pragma unroll
            for (int q = 0; q < kJ; ++q) sdz1[r][j0 + q] = sh1[r][j0 + q] > 0.0f ? a1[q] : 0.0f;
        }
        __syncthreads();
        if (tile_on) {
            for (int r = 0; r < kRedSub; ++r) {
                float u[T], w[T];
#pragma unroll
                for (int a = 0; a < T; ++a) {
                    u[a] = sdz2[r][i0 + a];
                    w[a] = sh1[r][j0 + a];
                }
#pragma unroll
                for (int a = 0; a < T; ++a)
#pragma unroll
                    for (int c = 0; c < T; ++c) acc[a][c] = __builtin_fmaf(u[a], w[c], acc[a][c]);
            }
        }
        if (tid == 0)
            for (int r = 0; r < kRedSub; ++r) accb3 += sg[r];
        if (tid < 4 * H) {
            for (int r = 0; r < kRedSub; ++r) {
                int64_t b = s0 + r;
                if (b >= B) break;
                float v;
                if (tid < H) {  // dw1_j = dz1_j x
                    v = sdz1[r][tid] * sx[r];
                } else if (tid < 2 * H) {  // db1_j = dz1_j
                    v = sdz1[r][tid - H];
                } else if (tid < 3 * H) {  // db2_i = dz2_i
                    v = sdz2[r][tid - 2 * H];
                } else {  // dw3_i = g h2_i
                    v = sg[r] * sh2[r][tid - 3 * H];
                }
                accv += v;
            }
        }
        __syncthreads();
    }
    float* row = part + (int64_t)blockIdx.x * P;
    if (tile_on) {
#pragma unroll
        for (int a = 0; a < T; ++a)
#pragma unroll
            for (int c = 0; c < T; ++c) row[2 * H + (i0 + a) * H + (j0 + c)] = acc[a][c];
    }
    if (tid < 4 * H) {
        int p;
        if (tid < 2 * H) p = tid;                                 // w1, b1
        else if (tid < 3 * H) p = 2 * H + H * H + (tid - 2 * H);  // b2
        else p = 3 * H + H * H + (tid - 3 * H);                   // w3
        row[p] = accv;
    }
    if (tid == 0) row[4 * H + H * H] = accb3;
}



__global__ void __launch_bounds__(8 * kSumCols) k_sum_rows(const float* __restrict__ part, int rows, int P,
                                                           float* out) {
    __shared__ float s[8][kSumCols];
    const int c = threadIdx.x % kSumCols, grp = threadIdx.x / kSumCols;
    const int p = blockIdx.x * kSumCols + c;
    const float t = column_sum(part, rows, P, p, c, grp, s);
    if (grp == 0 && p < P) out[p] = t;
}

// The fit's update: the same column sums, each fed straight into its
// parameter's Adam step (the gradient never goes through memory).
__global__ void __launch_bounds__(8 * kSumCols) k_sum_rows_adam(const float* __restrict__ part, int rows, int P,
                                                                float* th, float* m1, float* m2, float b1, float b2,
                                                                float c1, float c2, float lr, float eps) {
    __shared__ float s[8][kSumCols];
    const int c = threadIdx.x % kSumCols, grp = threadIdx.x / kSumCols;
    const int p = blockIdx.x * kSumCols + c;
    const float t = column_sum(part, rows, P, p, c, grp, s);
    if (grp == 0 && p < P) adam_update(p, t, th, m1, m2, b1, b2, c1, c2, lr, eps);
}


// Disorder of a model over the sorted sample: sum_j max(0, F_j - F_{j+1}),
// how far F moves backwards along keys that are in order (0 for a monotone
// model).  Partial sums per block (fixed order), then one block adds them.
__global__ void __launch_bounds__(256) k_disorder_partial(const double* __restrict__ F, int64_t k, double* part) {
    __shared__ double s[256];
    double acc = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j + 1 < k; j += (int64_t)gridDim.x * blockDim.x) {
        const double d = F[j] - F[j + 1];
        acc += d > 0.0 ? d : 0.0;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < (unsigned)off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void k_disorder_final(const double* __restrict__ part, int nb, double* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < nb; ++i) t += part[i];
        out[0] = t;
    }
}

constexpr int kDisorderBlocks = 512;
size_t disorder_ws_doubles() { return kDisorderBlocks + 1; }

hipError_t launch_disorder(const double* d_F, int64_t k, double* d_ws, hipStream_t st) {
    hipLaunchKernelGGL(k_disorder_partial, dim3(kDisorderBlocks), dim3(256), 0, st, d_F, k, d_ws);
    hipLaunchKernelGGL(k_disorder_final, dim3(1), dim3(64), 0, st, d_ws, kDisorderBlocks, d_ws + kDisorderBlocks);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_adam(float* th, const float* __restrict__ g, float* m1, float* m2,
                                              int64_t count, float b1, float b2, float c1, float c2, float lr,
                                              float eps) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= count) return;
    adam_update(p, g[p], th, m1, m2, b1, b2, c1, c2, lr, eps);
}

// ---- launchers ----
static unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

hipError_t launch_sample(const void* d_in, int64_t n, bool is_f64, uint64_t seed, int64_t k, uint64_t* d_out,
                         uint64_t* d_count, hipStream_t st) {
    unsigned g = nblk(k, 256 * kSampleItems);
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_sample, dim3(g), dim3(256), 0, st, (const uint64_t*)d_in, n, is_f64 ? 1 : 0, seed, k,
                       d_out, (unsigned long long*)d_count);
    return hipGetLastError();
}

// The sample as the one segment of the chunk sort: chunk prefix {0, nchunks}
// and key prefix {0, k}, written by one small launch.
__global__ void k_one_segment(int64_t* seg, int64_t nchunks, int64_t k) {
    if (threadIdx.x == 0) {
        seg[0] = 0;
        seg[1] = nchunks;
        seg[2] = 0;
        seg[3] = k;
    }
}

hipError_t launch_one_segment(int64_t* d_seg, int64_t nchunks, int64_t k, hipStream_t st) {
    hipLaunchKernelGGL(k_one_segment, dim3(1), dim3(64), 0, st, d_seg, nchunks, k);
    return hipGetLastError();
}

hipError_t launch_make_xy(const uint64_t* d_sorted, int64_t k, bool is_f64, double* d_x, float* d_y, double* d_lohi,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_make_xy, dim3(nblk(k, 256)), dim3(256), 0, st, d_sorted, k, is_f64 ? 1 : 0, d_x, d_y,
                       d_lohi);
    return hipGetLastError();
}

hipError_t launch_init(float* d_theta, int H, int init, uint64_t seed, const double* d_x, int64_t k,
                       int64_t* d_knots, void* d_knotws, hipStream_t st) {
    if (init == 1) {
        KnotWork* w = (KnotWork*)d_knotws;
        hipLaunchKernelGGL(k_knot_start, dim3(1), dim3(64), 0, st, k, w);
        for (int it = 0; it < H; ++it)  // the first piece, then at most H - 1 splits
            hipLaunchKernelGGL(k_knot_step, dim3(kKnotBlocks, 2), dim3(kKnotThreads), 0, st, d_x, k, H, it, w);
        hipLaunchKernelGGL(k_knot_finish, dim3(1), dim3(kKnotThreads), 0, st, k, H, w, d_knots);
    } else if (init == 2)
        hipLaunchKernelGGL(k_quantile_knots, dim3(1), dim3(128), 0, st, k, H, d_knots);
    hipLaunchKernelGGL(k_init, dim3(nblk(H * H + 4 * H + 1, 256)), dim3(256), 0, st, d_theta, H, init, seed,
                       d_x, k, (const int64_t*)d_knots);
    return hipGetLastError();
}

template <int H>
static hipError_t fwd_h(const float* th, const double* x, int64_t B, float* F, float* saved, hipStream_t st) {
    hipLaunchKernelGGL(k_fwd<H>, dim3(nblk(B, 256)), dim3(256), 0, st, th, x, B, F, saved);
    return hipGetLastError();
}

template <int H>
static hipError_t fwd_step_h(const float* th, const double* x, int64_t B, float* saved, const FitBatch& fb,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_fwd_fit<H>, dim3(nblk(B, 64)), dim3(256), 0, st, th, x, B, saved, fb);
    return hipGetLastError();
}

size_t fit_loss_ws_floats(int64_t B) {
    const int64_t nb = (B + 63) / 64;
    return (size_t)(nb > kLossBlocks ? nb : kLossBlocks);
}

// One training step's batch, forward and loss: the batch drawn from the
// sample (x, y of k entries) with replacement, h1 and h2 saved for
// the backward, dL/dF into gF, the batch loss into loss_out; the parameters
// are copied to `best` when that loss is the lowest so far.  partial holds
// fit_loss_ws_floats(B) floats.
hipError_t launch_fit_step_forward(int H, const float* d_theta, const double* d_x, const float* d_y, int64_t k,
                                   uint64_t seed, int64_t step, int64_t B, double* d_bx, float* d_saved, int loss,
                                   float delta, float* d_gF, float* d_loss, float* d_partial, float* d_best, int P,
                                   float* d_best_loss, hipStream_t st) {
    const FitBatch fb{d_y, k, seed, step, d_bx, loss, delta, d_gF, d_partial};
    hipError_t e;
    switch (H) {
    case 8: e = fwd_step_h<8>(d_theta, d_x, B, d_saved, fb, st); break;
    case 16: e = fwd_step_h<16>(d_theta, d_x, B, d_saved, fb, st); break;
    case 32: e = fwd_step_h<32>(d_theta, d_x, B, d_saved, fb, st); break;
    case 64: e = fwd_step_h<64>(d_theta, d_x, B, d_saved, fb, st); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_loss_final_keep, dim3(1), dim3(kLossBlocks), 0, st, d_partial, (int)nblk(B, 64), B, d_loss,
                       d_theta, d_best, P, d_best_loss);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(int H, const float* d_theta, const double* d_x, int64_t B, float* d_F,
                              float* d_saved, hipStream_t st) {
    switch (H) {
    case 8: return fwd_h<8>(d_theta, d_x, B, d_F, d_saved, st);
    case 16: return fwd_h<16>(d_theta, d_x, B, d_F, d_saved, st);
    case 32: return fwd_h<32>(d_theta, d_x, B, d_F, d_saved, st);
    case 64: return fwd_h<64>(d_theta, d_x, B, d_F, d_saved, st);
    default: return hipErrorInvalidValue;
    }
}

size_t mlp_backward_ws_floats(int H, int64_t B) {
    int64_t rows = (B + kRedChunk - 1) / kRedChunk;
    return (size_t)rows * (H * H + 4 * H + 1);
}

// Backward pass: per-chunk partial gradients into ws, then either their sums
// (gtheta) or, when `adam` is given, their sums applied as one Adam step.
struct AdamStep {
    float* m1;
    float* m2;
    float b1, b2, c1, c2, lr, eps;
};

template <int H>
static hipError_t bwd_h(const float* th, const double* x, int64_t B, const float* saved, const float* gF,
                        float* gtheta, float* ws, const AdamStep* adam, float* th_update, hipStream_t st) {
    constexpr int P = H * H + 4 * H + 1;
    float* part = ws;
    int rows = (int)((B + kRedChunk - 1) / kRedChunk);
    hipLaunchKernelGGL(k_bwd_reduce<H>, dim3(rows), dim3(256), 0, st, th, x, B, saved, gF, part);
    if (adam)
        hipLaunchKernelGGL(k_sum_rows_adam, dim3((P + kSumCols - 1) / kSumCols), dim3(8 * kSumCols), 0, st, part,
                           rows, P, th_update,
                           adam->m1, adam->m2, adam->b1, adam->b2, adam->c1, adam->c2, adam->lr, adam->eps);
    else
        hipLaunchKernelGGL(k_sum_rows, dim3((P + kSumCols - 1) / kSumCols), dim3(8 * kSumCols), 0, st, part, rows,
                           P, gtheta);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(int H, const float* d_theta, const double* d_x, int64_t B, const float* d_saved,
                               const float* d_gF, float* d_gtheta, float* d_ws, hipStream_t st) {
    switch (H) {
    case 8: return bwd_h<8>(d_theta, d_x, B, d_saved, d_gF, d_gtheta, d_ws, nullptr, nullptr, st);
    case 16: return bwd_h<16>(d_theta, d_x, B, d_saved, d_gF, d_gtheta, d_ws, nullptr, nullptr, st);
    case 32: return bwd_h<32>(d_theta, d_x, B, d_saved, d_gF, d_gtheta, d_ws, nullptr, nullptr, st);
    case 64: return bwd_h<64>(d_theta, d_x, B, d_saved, d_gF, d_gtheta, d_ws, nullptr, nullptr, st);
    default: return hipErrorInvalidValue;
    }
}

// The fit's backward and update: gradients of d_theta applied to it by one
// Adam step t (the same arithmetic as launch_mlp_backward then launch_adam).
hipError_t launch_mlp_backward_adam(int H, float* d_theta, const double* d_x, int64_t B, const float* d_saved,
                                    const float* d_gF, float* d_ws, float* d_m1, float* d_m2, int64_t t, float lr,
                                    float b1, float b2, float eps, hipStream_t st) {
    const AdamStep a{d_m1, d_m2, b1, b2, (float)(1.0 - pow((double)b1, (double)t)),
                     (float)(1.0 - pow((double)b2, (double)t)), lr, eps};
    switch (H) {
    case 8: return bwd_h<8>(d_theta, d_x, B, d_saved, d_gF, nullptr, d_ws, &a, d_theta, st);
    case 16: return bwd_h<16>(d_theta, d_x, B, d_saved, d_gF, nullptr, d_ws, &a, d_theta, st);
    case 32: return bwd_h<32>(d_theta, d_x, B, d_saved, d_gF, nullptr, d_ws, &a, d_theta, st);
    case 64: return bwd_h<64>(d_theta, d_x, B, d_saved, d_gF, nullptr, d_ws, &a, d_theta, st);
    default: return hipErrorInvalidValue;
    }
}

size_t loss_ws_floats() { return kLossBlocks; }

hipError_t launch_loss_grad(const float* d_F, const float* d_y, int64_t B, int loss, float delta, float* d_gF,
                            float* d_loss, float* d_partial, hipStream_t st) {
    hipLaunchKernelGGL(k_loss, dim3(kLossBlocks), dim3(256), 0, st, d_F, d_y, B, loss, delta, d_gF, d_partial);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(kLossBlocks), 0, st, d_partial, kLossBlocks, B, d_loss);
    return hipGetLastError();
}

hipError_t launch_adam(float* d_theta, const float* d_g, float* d_m1, float* d_m2, int64_t count, int64_t t,
                       float lr, float b1, float b2, float eps, hipStream_t st) {
    float c1 = (float)(1.0 - pow((double)b1, (double)t));
    float c2 = (float)(1.0 - pow((double)b2, (double)t));
    hipLaunchKernelGGL(k_adam, dim3(nblk(count, 256)), dim3(256), 0, st, d_theta, d_g, d_m1, d_m2, count, b1, b2,
                       c1, c2, lr, eps);
    return hipGetLastError();
}

}  // namespace nns
