// Piecewise-linear form of the model map.  A network with one input and ReLU
// units computes a continuous piecewise-linear function: layer-1 unit k is
// active on one side of x = -b1_k / w1_k, so those knots cut [0, 1] into at
// most H + 1 intervals on which the active set, and hence every layer-2
// pre-activation z2_i = A_i x + B_i, is fixed; z2_i changes sign at most once
// inside an interval, at -B_i / A_i, and between consecutive such roots the
// output F = b3 + sum_i w3_i relu(z2_i) is affine.  The function is the same
// as the direct evaluation of the same weights; only the rounding differs.
//
// Compiled on the device from the FP32 weights in FP64, in two launches:
//  1. k_pwl_intervals, one workgroup per interval: the sorted layer-1 knots
//     (every workgroup ranks them the same way), A and B of the interval, and
//     its layer-2 roots sorted;
//  2. k_pwl_pieces, one workgroup per interval: the interval's first piece
//     index (from the root counts), then per piece its left edge xq, slope
//     alpha and value Fq at xq.
// The map kernel's workgroups each index the pieces by 1024 cells of [0, 1],
// then find each key's piece (two index entries bracket it, a binary search
// between them settles it) and evaluate one FP64 fma.
#include "infer_common.h"

namespace nns {

template <int H>
__global__ void __launch_bounds__(64) k_pwl_intervals(const DevModel* __restrict__ m, PwlTable* __restrict__ t) {
    __shared__ double s_w1[64], s_b1[64];
    __shared__ double s_c[64];
    __shared__ int s_ok[64];
    __shared__ double s_e[kPwlMaxIntervals + 1];
    const int lane = threadIdx.x;
    // W2 row `lane` in registers: independent 16-byte loads, all in flight
    // together
    float w2r[H];
    if (lane < H) {
        const float4* row = reinterpret_cast<const float4*>(m->w2 + lane * H);
#pragma unroll
        for (int q = 0; q < H / 4; ++q) {
            const float4 v = row[q];
            w2r[4 * q] = v.x;
            w2r[4 * q + 1] = v.y;
            w2r[4 * q + 2] = v.z;
            w2r[4 * q + 3] = v.w;
        }
    }
    const double w1l = lane < H ? (double)m->w1[lane] : 0.0;
    const double b1l = lane < H ? (double)m->b1[lane] : 0.0;
    s_w1[lane] = w1l;
    s_b1[lane] = b1l;
    // layer-1 knots strictly inside (0, 1), ranked with ties by unit index
    double c = 0.0;
    bool ok = false;
    if (lane < H && w1l != 0.0) {
        c = -b1l / w1l;
        ok = c > 0.0 && c < 1.0;
    }
    s_c[lane] = c;
    s_ok[lane] = ok ? 1 : 0;
    const int nk = __popcll(__ballot(ok));
    __syncthreads();
    if (ok) {
        int r = 0;
        for (int k = 0; k < H; ++k) r += (s_ok[k] && (s_c[k] < c || (s_c[k] == c && k < lane))) ? 1 : 0;
        s_e[1 + r] = c;
    }
    if (lane == 0) {
        s_e[0] = 0.0;
        s_e[nk + 1] = 1.0;
    }
    __syncthreads();
    const int nint = nk + 1;
    const int j = blockIdx.x;
    if (j == 0) {
        for (int e = lane; e <= nint; e += 64) t->edge[e] = s_e[e];
        if (lane == 0) t->nint = nint;
    }
    if (j >= nint) return;
    const double l = s_e[j], r = s_e[j + 1], mid = 0.5 * (l + r);
    // the layer-1 units active at the interval's midpoint are active on all
    // of it; z2 of unit `lane` there is A x + B
    const unsigned long long act = __ballot(lane < H && fma(w1l, mid, b1l) > 0.0);
    double A = 0.0, B = 0.0;
    if (lane < H) {
        B = (double)m->b2[lane];
#pragma unroll
        for (int k = 0; k < H; ++k) {
            if ((act >> k) & 1ull) {
                const double w = w2r[k];
                A = fma(w, s_w1[k], A);
                B = fma(w, s_b1[k], B);
            }
        }
    }
    t->A[j][lane] = A;
    t->B[j][lane] = B;
    // the units whose z2 changes sign strictly inside, in order of the root
    double rho = 0.0;
    bool in = false;
    if (A != 0.0) {
        rho = -B / A;
        in = rho > l && rho < r;
    }
    const int cnt = __popcll(__ballot(in));
    int rank = 0;
    for (int q = 0; q < 64; ++q) {
        const double rq = __shfl(rho, q);
        const int iq = __shfl(in ? 1 : 0, q);
        rank += (iq && (rq < rho || (rq == rho && q < lane))) ? 1 : 0;
    }
    double* sub = t->sub[j];
    if (in) sub[1 + rank] = rho;
    if (lane == 0) {
        sub[0] = l;
        sub[cnt + 1] = r;
        t->nroots[j] = cnt;
    }
}

__global__ void __launch_bounds__(64) k_pwl_pieces(const DevModel* __restrict__ m, PwlTable* __restrict__ t) {
    __shared__ double s_A[64], s_B[64], s_w3[64];
    const int j = blockIdx.x, lane = threadIdx.x;
    const int nint = t->nint;
    if (j >= nint) return;
    const int H = m->H;
    int off = 0, tot = 0;
    for (int q = lane; q < nint; q += 64) {
        const int c = t->nroots[q] + 1;
        tot += c;
        off += q < j ? c : 0;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        off += __shfl_xor(off, o);
        tot += __shfl_xor(tot, o);
    }
    if (j == 0 && lane == 0) t->npieces = tot;
    s_A[lane] = t->A[j][lane];
    s_B[lane] = t->B[j][lane];
    s_w3[lane] = lane < H ? (double)m->w3[lane] : 0.0;
    __syncthreads();
    const int cnt = t->nroots[j];
    const double* sub = t->sub[j];
    for (int p = lane; p <= cnt; p += 64) {
        // the layer-2 units active at the piece's midpoint are active on all
        // of it; F is taken at the left edge
        const double pl = sub[p], pr = sub[p + 1], pm = 0.5 * (pl + pr);
        double alpha = 0.0, F = (double)m->b3;
        for (int i = 0; i < H; ++i) {
            const double Ai = s_A[i], Bi = s_B[i];
            if (fma(Ai, pm, Bi) > 0.0) {
                alpha = fma(s_w3[i], Ai, alpha);
                F = fma(s_w3[i], fma(Ai, pl, Bi), F);
            }
        }
        t->xq[off + p] = pl;
        t->alpha[off + p] = alpha;
        t->Fq[off + p] = F;
    }
}

// F at x in [0, 1]: the last piece with xq <= x lies in [first[c],
// first[c + 1]] for the cell c of x (c = kPwlGrid - 1 for x = 1), where
// first[c] is the last piece starting at or before c / kPwlGrid.
__device__ __forceinline__ double pwl_eval(double x, const double* X, const double* Al, const double* Fq,
                                           const uint16_t* first) {
    int c = (int)(x * (double)kPwlGrid);
    c = c < kPwlGrid ? c : kPwlGrid - 1;
    int lo = first[c], hi = first[c + 1];
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (X[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return fma(Al[lo], x - X[lo], Fq[lo]);
}

// Keys per workgroup and step: each thread keeps kPwlPer independent loads
// in flight (measured at 1e8 keys: 2 per thread +48%, 4 per thread +6%
// against 8).
constexpr int kPwlThreads = 256;
constexpr int kPwlPer = 8;

__device__ __forceinline__ void pwl_map(const InferArgs& a, const double* X, const double* Al, const double* Fq,
                                        const uint16_t* first) {
    const double lo = a.model->lo, inv = a.model->inv_range;
    constexpr int kTile = kPwlThreads * kPwlPer;
    for (int64_t base = (int64_t)blockIdx.x * kTile; base < a.n; base += (int64_t)gridDim.x * kTile) {
        uint64_t bits[kPwlPer];
#pragma unroll
        for (int k = 0; k < kPwlPer; ++k) {
            const int64_t i = base + k * kPwlThreads + threadIdx.x;
            bits[k] = i < a.n ? a.in[i] : 0;
        }
#pragma unroll
        for (int k = 0; k < kPwlPer; ++k) {
            const int64_t i = base + k * kPwlThreads + threadIdx.x;
            if (i >= a.n) break;
            uint32_t slot = kUnmapped;
            double F = __longlong_as_double(0x7FF8000000000000ll);
            double x;
            if (translate_key(bits[k], a.is_f64, lo, inv, &x)) {
                F = pwl_eval(x, X, Al, Fq, first);
                slot = slot_of(F, a.M);
            }
            if (a.slots_out) a.slots_out[i] = slot;
            if (a.F_out) a.F_out[i] = F;
        }
    }
}

// Tables of up to kPwlLds pieces are read from LDS, larger ones from global
// memory (the fitted models seen here have about 2H pieces; the bound is
// (H + 1)^2).  A 512-piece table (14 KB of LDS with the index) leaves room
// for more workgroups per CU than a 1024-piece one: 0.30 vs 0.32 ms at 1e8.
// Every workgroup builds the piece index for itself.
constexpr int kPwlLds = 512;

__global__ void __launch_bounds__(kPwlThreads) k_infer_pwl(InferArgs a) {
    __shared__ double s_x[kPwlLds], s_a[kPwlLds], s_f[kPwlLds];
    __shared__ uint16_t s_first[kPwlGrid + 1];
    const PwlTable* __restrict__ t = a.pwl;
    const int np = t->npieces;
    const bool lds = np <= kPwlLds;
    if (lds) {
        for (int i = threadIdx.x; i < np; i += kPwlThreads) {
            s_x[i] = t->xq[i];
            s_a[i] = t->alpha[i];
            s_f[i] = t->Fq[i];
        }
        __syncthreads();
    }
    const double* X = lds ? s_x : t->xq;
    for (int c = threadIdx.x; c <= kPwlGrid; c += kPwlThreads) {
        const double v = c * (1.0 / kPwlGrid);
        int lo = 0, hi = np - 1;  // xq[0] = 0 <= v
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (X[mid] <= v) lo = mid;
            else hi = mid - 1;
        }
        s_first[c] = (uint16_t)lo;
    }
    __syncthreads();
    if (lds) pwl_map(a, s_x, s_a, s_f, s_first);
    else pwl_map(a, t->xq, t->alpha, t->Fq, s_first);
}

hipError_t launch_pwl_infer(const InferArgs& a, int H, hipStream_t st) {
    if (!a.pwl) return hipErrorInvalidValue;
    if (H == 32)
        hipLaunchKernelGGL(k_pwl_intervals<32>, dim3(kPwlMaxIntervals), dim3(64), 0, st, a.model, a.pwl);
    else if (H == 64)
        hipLaunchKernelGGL(k_pwl_intervals<64>, dim3(kPwlMaxIntervals), dim3(64), 0, st, a.model, a.pwl);
    else
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pwl_pieces, dim3(kPwlMaxIntervals), dim3(64), 0, st, a.model, a.pwl);
    constexpr int kTile = kPwlThreads * kPwlPer;
    int64_t blocks = (a.n + kTile - 1) / kTile;
    if (blocks > 256 * 24) blocks = 256 * 24;  // measured: 8 per CU +9%, 64 per CU +5%
    hipLaunchKernelGGL(k_infer_pwl, dim3((unsigned)blocks), dim3(kPwlThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace nns
