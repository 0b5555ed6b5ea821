/*
 * NN-sort oracle: TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, deliberately unoptimised CPU statement of what the NN-sort
 * hot path computes ("Deep Learning Service for Efficient Data Distribution
 * Aware Sorting", Zhu et al., arXiv 1907.08817).  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or helper with the HIP library; the two meet only through
 * plain arrays handed over by the tests.
 *
 * Arithmetic: FP64 everywhere the paper leaves precision open, except the
 * "canonical FP32" model evaluator, which fixes one FP32 operation order so
 * that a GPU kernel taking the same decision (key -> integer slot) in FP32 can
 * be checked slot for slot.  Build with -ffp-contract=off: every fused
 * multiply-add below is an explicit fma()/fmaf() call.
 *
 * Parity pins (what checks this file against something other than itself) live
 * in tests/test_oracle_pins.py.  Parity unpinned: the worked example's
 * intermediate conflict arrays (Sec. 2, Example) -- the example's model f and
 * figure are not given and its first conflict array contradicts the
 * first-arrival rule of the Sorting Phase.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_UNMAPPED 0xFFFFFFFFu

/* ------------------------------------------------------------------------ */
/* Order key: IEEE 754-2019 totalOrder for binary64, identity for uint64.   */
/* The paper sorts 64-bit floats (Sec. 4.1, Datasets); it does not discuss  */
/* -0, NaN or infinities, so the total order of the IEEE standard is taken. */
/* ------------------------------------------------------------------------ */
uint64_t orc_order_key(uint64_t bits, int is_f64)
{
    if (!is_f64) return bits;
    if (bits >> 63) return ~bits;            /* negative: reverse magnitude */
    return bits | 0x8000000000000000ull;     /* positive: above all negatives */
}

uint64_t orc_order_key_inverse(uint64_t key, int is_f64)
{
    if (!is_f64) return key;
    if (key >> 63) return key & 0x7FFFFFFFFFFFFFFFull;
    return ~key;
}

static double bits_to_f64(uint64_t b)
{
    double d;
    memcpy(&d, &b, 8);
    return d;
}

static int cmp_u64(const void* a, const void* b)
{
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return (x > y) - (x < y);
}

/* The plain definition of the result: the input sorted by order key. */
void orc_sort_bits(const uint64_t* in, int64_t n, int is_f64, uint64_t* out)
{
    uint64_t* k = (uint64_t*)malloc((size_t)(n > 0 ? n : 1) * 8);
    for (int64_t i = 0; i < n; ++i) k[i] = orc_order_key(in[i], is_f64);
    qsort(k, (size_t)n, 8, cmp_u64);
    for (int64_t i = 0; i < n; ++i) out[i] = orc_order_key_inverse(k[i], is_f64);
    free(k);
}

/* ------------------------------------------------------------------------ */
/* Input phase, translate(A) (Sec. 2, Input Phase): encode a key as the     */
/* model's input.  The paper names only string->ASCII; for numbers the      */
/* reading taken is an FP64 affine min-max map onto [0,1] with (lo,         */
/* inv_range) stored in the model.  Non-finite keys are unmappable and go   */
/* straight to the conflict array every round.                              */
/* ------------------------------------------------------------------------ */
int orc_translate(uint64_t bits, int is_f64, double lo, double inv_range, double* xhat)
{
    double x = is_f64 ? bits_to_f64(bits) : (double)bits;
    if (!isfinite(x)) return 0;
    double t = (x - lo) * inv_range;
    if (t != t) return 0;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    *xhat = t;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* The learned model f (Sec. 2, Sorting Phase; Sec. 4.1 Training details): */
/* a regression MLP 1 -> H -> H -> 1 with ReLU, returning F in ~[0,1], the  */
/* normalised expected position of the key.                                 */
/*                                                                          */
/* Packed parameter vector theta (length H*H + 4H + 1):                      */
/*   w1[H] | b1[H] | W2[H*H] (row i = hidden-2 unit i, column j = hidden-1  */
/*   unit j) | b2[H] | w3[H] | b3                                           */
/* ------------------------------------------------------------------------ */
#define W1(t, H) (t)
#define B1(t, H) ((t) + (H))
#define W2(t, H) ((t) + 2 * (H))
#define B2(t, H) ((t) + 2 * (H) + (H) * (H))
#define W3(t, H) ((t) + 3 * (H) + (H) * (H))
#define B3(t, H) ((t)[4 * (H) + (H) * (H)])

/* FP64 evaluation of the graph (weights widened exactly from FP32). */
double orc_f_fp64(int H, const float* th, double x)
{
    double h1[64], F;
    for (int j = 0; j < H; ++j) {
        double z = (double)W1(th, H)[j] * x + (double)B1(th, H)[j];
        h1[j] = z > 0.0 ? z : 0.0;
    }
    F = (double)B3(th, H);
    for (int i = 0; i < H; ++i) {
        double z = (double)B2(th, H)[i];
        for (int j = 0; j < H; ++j) z += (double)W2(th, H)[i * H + j] * h1[j];
        double h2 = z > 0.0 ? z : 0.0;
        F += (double)W3(th, H)[i] * h2;
    }
    return F;
}

/* Round an FP32 value to the nearest bfloat16, ties to even. */
float orc_round_bf16(float v)
{
    uint32_t u;
    memcpy(&u, &v, 4);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return v; /* NaN */
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    u &= 0xFFFF0000u;
    float r;
    memcpy(&r, &u, 4);
    return r;
}

/* FP64 evaluation of the "BF16 model": the hidden-to-hidden matrix W2 rounded
 * to bfloat16 (the operand the matrix cores consume), everything else as in
 * orc_f_fp64. */
double orc_f_bf16w(int H, const float* th, double x)
{
    double h1[64], F;
    for (int j = 0; j < H; ++j) {
        double z = (double)W1(th, H)[j] * x + (double)B1(th, H)[j];
        h1[j] = z > 0.0 ? z : 0.0;
    }
    F = (double)B3(th, H);
    for (int i = 0; i < H; ++i) {
        double z = (double)B2(th, H)[i];
        for (int j = 0; j < H; ++j) z += (double)orc_round_bf16(W2(th, H)[i * H + j]) * h1[j];
        double h2 = z > 0.0 ? z : 0.0;
        F += (double)W3(th, H)[i] * h2;
    }
    return F;
}

/* Canonical FP32 evaluation.  One fixed order of FP32 operations, so that an
 * FP32 implementation elsewhere can reproduce the slot bit for bit:
 *   xh = fl32(x), xl = fl32(x - xh)                      (two-float input)
 *   z1_j = fma(w1_j, xl, fma(w1_j, xh, b1_j)),  h1 = relu
 *   z2_i = b2_i; for j ascending: z2_i = fma(W2_ij, h1_j, z2_i),  h2 = relu
 *   F = b3 + sum_i w3_i h2_i, compensated (Dot2 of Ogita, Rump and Oishi,
 *       "Accurate sum and dot product", 2005: TwoProduct by FMA + TwoSum), i
 *       ascending, returned as (double)sum + (double)correction.
 * relu(z) = z > 0 ? z : 0 (a NaN maps to 0). */
static inline float two_sum(float a, float b, float* err)
{
    float s = a + b;
    float bb = s - a;
    *err = (a - (s - bb)) + (b - bb);
    return s;
}

double orc_f_fp32c(int H, const float* th, double x)
{
    float h1[64];
    float xh = (float)x;
    float xl = (float)(x - (double)xh);
    for (int j = 0; j < H; ++j) {
        float z = fmaf(W1(th, H)[j], xh, B1(th, H)[j]);
        z = fmaf(W1(th, H)[j], xl, z);
        h1[j] = z > 0.0f ? z : 0.0f;
    }
    float p = B3(th, H), s = 0.0f;
    for (int i = 0; i < H; ++i) {
        float z = B2(th, H)[i];
        for (int j = 0; j < H; ++j) z = fmaf(W2(th, H)[i * H + j], h1[j], z);
        float h2 = z > 0.0f ? z : 0.0f;
        float w = W3(th, H)[i];
        float pr = w * h2;
        float r = fmaf(w, h2, -pr);
        float q;
        p = two_sum(p, pr, &q);
        s = s + (q + r);
    }
    return (double)p + (double)s;
}

enum { ORC_FORM_FP32C = 0, ORC_FORM_FP64 = 1, ORC_FORM_BF16W = 2 };

static double eval_form(int form, int H, const float* th, double x)
{
    if (form == ORC_FORM_FP32C) return orc_f_fp32c(H, th, x);
    if (form == ORC_FORM_BF16W) return orc_f_bf16w(H, th, x);
    return orc_f_fp64(H, th, x);
}

/* ------------------------------------------------------------------------ */
/* Slot: pos <- round(w_pos * m) (Sec. 2, Sorting Phase).  f returns the    */
/* normalised position F, so w_pos = F*n and pos = round(F * M), M = m*n,   */
/* in FP64, clamped to [0, M], rounded half away from zero.  A NaN F is     */
/* unmappable.  The slot array o_i has S = round(M) + 1 entries.            */
/* ------------------------------------------------------------------------ */
uint32_t orc_slot(double F, double M)
{
    if (F != F) return ORC_UNMAPPED;
    double v = F * M;
    if (v < 0.0) v = 0.0;
    if (v > M) v = M;
    double t = trunc(v);
    if (v - t >= 0.5) t += 1.0;
    return (uint32_t)t;
}

int64_t orc_num_slots(int64_t n, double m)
{
    double M = m * (double)n;
    double t = trunc(M);
    if (M - t >= 0.5) t += 1.0;
    return (int64_t)t + 1;
}

/* A model with a non-finite parameter (weights, lo or inv_range) maps no
 * key: the paper does not consider such models; the reading taken is that
 * every key then stays in the conflict arrays and the residue sort orders
 * them all. */
int orc_model_finite(int H, const float* th, double lo, double inv_range)
{
    if (!isfinite(lo) || !isfinite(inv_range)) return 0;
    for (int p = 0; p < H * H + 4 * H + 1; ++p)
        if (!isfinite(th[p])) return 0;
    return 1;
}

/* Slots of every key (the map w.map(f) followed by the rounding). */
void orc_predict_slots(const uint64_t* bits, int64_t n, int is_f64, int H, const float* th,
                       double lo, double inv_range, double m, int form, uint32_t* slots)
{
    double M = m * (double)n;
    if (!orc_model_finite(H, th, lo, inv_range)) {
        for (int64_t i = 0; i < n; ++i) slots[i] = ORC_UNMAPPED;
        return;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double x;
        if (!orc_translate(bits[i], is_f64, lo, inv_range, &x)) {
            slots[i] = ORC_UNMAPPED;
            continue;
        }
        slots[i] = orc_slot(eval_form(form, H, th, x), M);
    }
}

void orc_translate_many(const uint64_t* bits, int64_t n, int is_f64, double lo, double inv_range,
                        double* xhat, uint8_t* ok)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double x = 0.0;
        ok[i] = (uint8_t)orc_translate(bits[i], is_f64, lo, inv_range, &x);
        xhat[i] = x;
    }
}

void orc_eval_many(const double* xhat, int64_t n, int H, const float* th, int form, double* F)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) F[i] = eval_form(form, H, th, xhat[i]);
}

/* ------------------------------------------------------------------------ */
/* The method: Procedure NN-sort (Sec. 2, Figure "Algorithm NN-sort") with  */
/* polish (Figure "Algorithm polish").                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    int64_t rounds;          /* t, completed iterations */
    int64_t collided[8];     /* |c_r| after round r (conflict array size) */
    int64_t placed[8];       /* keys stored in o_r */
    int64_t extracted[8];    /* e_r: o_r entries below the running maximum */
    int64_t residue;         /* size of the last conflict array w */
    double pos_err;          /* mean |F(out[p]) * n - p| / n over mappable keys */
} orc_stats;

/* Merge two ascending arrays of order keys. */
static void merge2(const uint64_t* a, int64_t na, const uint64_t* b, int64_t nb, uint64_t* out)
{
    int64_t i = 0, j = 0, k = 0;
    while (i < na && j < nb) out[k++] = (b[j] < a[i]) ? b[j++] : a[i++];
    while (i < na) out[k++] = a[i++];
    while (j < nb) out[k++] = b[j++];
}

/*
 * slots[i] must be the slot of key i (orc_predict_slots); passing them in keeps
 * the model evaluation in one place.  f is a fixed function, so mapping the
 * conflict array again in a later round gives every key the same slot it had
 * before: the round loop below therefore looks the slot up instead of
 * re-evaluating f.
 */
int orc_nnsort(const uint64_t* bits, int64_t n, int is_f64, const uint32_t* slots,
               double m, int eps, int64_t tau, uint64_t* out_bits, orc_stats* st)
{
    memset(st, 0, sizeof(*st));
    st->n = n;
    if (eps < 0 || eps > 8) return -1;
    int64_t S = orc_num_slots(n, m);
    for (int64_t i = 0; i < n; ++i)
        if (slots[i] != ORC_UNMAPPED && (int64_t)slots[i] >= S) return -2;

    /* w <- translate(A): w holds input indices, in processing order. */
    int64_t* w = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * 8);
    int64_t* c = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * 8);
    for (int64_t i = 0; i < n; ++i) w[i] = i;
    int64_t nw = n;

    /* O <- {}; o_i kept as the occupied slots in slot order (order keys). */
    uint64_t* O[8] = {0};
    int64_t On[8] = {0};
    int t = 0;

    /* while i < eps and count(w) > tau (the printed guard 0 < i < eps with
     * i <- 0 would never run; read as 0 <= i < eps). */
    uint32_t* owner = NULL;
    while (t < eps && nw > tau) {
        if (!owner) owner = (uint32_t*)malloc((size_t)S * 4);
        for (int64_t s = 0; s < S; ++s) owner[s] = ORC_UNMAPPED;
        int64_t nc = 0;
        for (int64_t idx = 0; idx < nw; ++idx) {
            int64_t key = w[idx];
            uint32_t pos = slots[key];
            if (pos != ORC_UNMAPPED && owner[pos] == ORC_UNMAPPED)
                owner[pos] = (uint32_t)key;      /* o_i[pos] is empty: store */
            else
                c[nc++] = key;                   /* conflict: c.append */
        }
        int64_t np = nw - nc;
        O[t] = (uint64_t*)malloc((size_t)(np > 0 ? np : 1) * 8);
        int64_t k = 0;
        for (int64_t s = 0; s < S; ++s)
            if (owner[s] != ORC_UNMAPPED) O[t][k++] = orc_order_key(bits[owner[s]], is_f64);
        On[t] = k;
        st->placed[t] = k;
        st->collided[t] = nc;
        int64_t* tmp = w; w = c; c = tmp;        /* w <- c */
        nw = nc;
        ++t;
    }
    free(owner);
    st->rounds = t;
    st->residue = nw;

    /* QuickSort(w): any correct comparison sort of the last conflict array. */
    uint64_t* A = (uint64_t*)malloc((size_t)(n > 0 ? n : 1) * 8);
    uint64_t* B = (uint64_t*)malloc((size_t)(n > 0 ? n : 1) * 8);
    for (int64_t i = 0; i < nw; ++i) A[i] = orc_order_key(bits[w[i]], is_f64);
    qsort(A, (size_t)nw, 8, cmp_u64);
    int64_t nA = nw;

    /* polish(O, w): A' <- w; for o_i in O: A' <- InsertSort(A', o_i).
     * Entries of o_i that are in order (not below the running maximum of the
     * entries before them) are the ones appended; the others are inserted.
     * The result of inserting each out-of-order entry at its place equals
     * merging A' with the in-order run and with the sorted out-of-order set,
     * which is what is done here (avoiding the quadratic insertion cost). */
    for (int r = 0; r < t; ++r) {
        int64_t np = On[r];
        uint64_t* R = (uint64_t*)malloc((size_t)(np > 0 ? np : 1) * 8);
        uint64_t* X = (uint64_t*)malloc((size_t)(np > 0 ? np : 1) * 8);
        int64_t nR = 0, nX = 0;
        uint64_t runmax = 0;
        int have = 0;
        for (int64_t p = 0; p < np; ++p) {
            uint64_t v = O[r][p];
            if (!have || v >= runmax) {
                R[nR++] = v;
                runmax = v;
                have = 1;
            } else {
                X[nX++] = v;
            }
        }
        st->extracted[r] = nX;
        qsort(X, (size_t)nX, 8, cmp_u64);
        merge2(A, nA, R, nR, B);
        merge2(B, nA + nR, X, nX, A);
        nA += nR + nX;
        free(R);
        free(X);
        free(O[r]);
    }
    for (int64_t i = 0; i < n; ++i) out_bits[i] = orc_order_key_inverse(A[i], is_f64);
    free(A);
    free(B);
    free(w);
    free(c);
    return 0;
}

/* Mean |F(out[p]) * n - p| / n over the mappable keys of a sorted output: how
 * far the model's expected position is from the true rank (ties ranked by
 * output position). */
double orc_pos_err(const uint64_t* sorted_bits, int64_t n, int is_f64, int H, const float* th,
                   double lo, double inv_range, int form, int64_t* counted)
{
    double acc = 0.0;
    int64_t cnt = 0;
#pragma omp parallel for reduction(+ : acc, cnt) schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        double x;
        if (!orc_translate(sorted_bits[p], is_f64, lo, inv_range, &x)) continue;
        double F = eval_form(form, H, th, x);
        acc += fabs(F * (double)n - (double)p);
        cnt += 1;
    }
    if (counted) *counted = cnt;
    return cnt ? acc / (double)cnt / (double)n : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Training (Sec. 2, Training; Sec. 4.1, Training details): Adam on a       */
/* regression loss.  FP64 forward/backward of the MLP for a batch.          */
/* loss 0: mean squared error; loss 1: Huber with threshold delta, the      */
/* paper's Eq. (loss), averaged over the batch.                              */
/* grad has the packed theta layout.  Returns the loss.                     */
/* ------------------------------------------------------------------------ */
static double loss_grad_chunk(int H, const double* th, const double* x, const double* y,
                              int64_t b0, int64_t b1_, double invB, int loss, double delta,
                              double* grad)
{
    const double *w1 = th, *b1 = th + H, *W2 = th + 2 * H, *b2 = th + 2 * H + H * H,
                 *w3 = th + 3 * H + H * H;
    double b3 = th[4 * H + H * H];
    double *gw1 = grad, *gb1 = grad + H, *gW2 = grad + 2 * H, *gb2 = grad + 2 * H + H * H,
           *gw3 = grad + 3 * H + H * H;
    double L = 0.0;
    for (int64_t b = b0; b < b1_; ++b) {
        double z1[64], h1[64], z2[64], h2[64], dz2[64];
        for (int j = 0; j < H; ++j) {
            z1[j] = w1[j] * x[b] + b1[j];
            h1[j] = z1[j] > 0.0 ? z1[j] : 0.0;
        }
        double F = b3;
        for (int i = 0; i < H; ++i) {
            double z = b2[i];
            for (int j = 0; j < H; ++j) z += W2[i * H + j] * h1[j];
            z2[i] = z;
            h2[i] = z > 0.0 ? z : 0.0;
            F += w3[i] * h2[i];
        }
        double e = F - y[b], g;
        if (loss == 1) {
            if (fabs(e) <= delta) {
                L += 0.5 * e * e;
                g = e;
            } else {
                L += delta * fabs(e) - 0.5 * delta * delta;
                g = e > 0 ? delta : -delta;
            }
        } else {
            L += e * e;
            g = 2.0 * e;
        }
        g *= invB;
        grad[4 * H + H * H] += g;
        for (int i = 0; i < H; ++i) {
            gw3[i] += g * h2[i];
            dz2[i] = z2[i] > 0.0 ? g * w3[i] : 0.0;
            gb2[i] += dz2[i];
            for (int j = 0; j < H; ++j) gW2[i * H + j] += dz2[i] * h1[j];
        }
        for (int j = 0; j < H; ++j) {
            if (!(z1[j] > 0.0)) continue;
            double dh = 0.0;
            for (int i = 0; i < H; ++i) dh += dz2[i] * W2[i * H + j];
            gw1[j] += dh * x[b];
            gb1[j] += dh;
        }
    }
    return L;
}

#define ORC_GRAD_CHUNKS 64
double orc_loss_grad_f64(int H, const double* th, const double* x, const double* y, int64_t B,
                         int loss, double delta, double* grad)
{
    int P = H * H + 4 * H + 1;
    double* part = (double*)calloc((size_t)ORC_GRAD_CHUNKS * P, sizeof(double));
    double Lpart[ORC_GRAD_CHUNKS];
    double invB = 1.0 / (double)B;
    /* Fixed chunks summed in chunk order: the result does not depend on the
     * number of threads. */
#pragma omp parallel for schedule(static)
    for (int c = 0; c < ORC_GRAD_CHUNKS; ++c) {
        int64_t b0 = B * c / ORC_GRAD_CHUNKS, b1_ = B * (c + 1) / ORC_GRAD_CHUNKS;
        Lpart[c] = loss_grad_chunk(H, th, x, y, b0, b1_, invB, loss, delta, part + (size_t)c * P);
    }
    double L = 0.0;
    for (int p = 0; p < P; ++p) grad[p] = 0.0;
    for (int c = 0; c < ORC_GRAD_CHUNKS; ++c) {
        L += Lpart[c];
        for (int p = 0; p < P; ++p) grad[p] += part[(size_t)c * P + p];
    }
    free(part);
    return L * invB;
}

/* FP64 forward only, same graph, for finite differences in double params. */
double orc_loss_f64(int H, const double* th, const double* x, const double* y, int64_t B, int loss,
                    double delta)
{
    double L = 0.0;
    const double *w1 = th, *b1 = th + H, *W2 = th + 2 * H, *b2 = th + 2 * H + H * H,
                 *w3 = th + 3 * H + H * H;
    for (int64_t b = 0; b < B; ++b) {
        double h1[64];
        for (int j = 0; j < H; ++j) {
            double z = w1[j] * x[b] + b1[j];
            h1[j] = z > 0.0 ? z : 0.0;
        }
        double F = th[4 * H + H * H];
        for (int i = 0; i < H; ++i) {
            double z = b2[i];
            for (int j = 0; j < H; ++j) z += W2[i * H + j] * h1[j];
            F += w3[i] * (z > 0.0 ? z : 0.0);
        }
        double e = F - y[b];
        if (loss == 1)
            L += fabs(e) <= delta ? 0.5 * e * e : delta * fabs(e) - 0.5 * delta * delta;
        else
            L += e * e;
    }
    return L / (double)B;
}

/* Adam (Kingma and Ba, the optimiser the paper names), with bias correction.
 * t is the 1-based step number. */
void orc_adam_step(double* th, const double* g, double* mom1, double* mom2, int P, int64_t t,
                   double lr, double beta1, double beta2, double eps)
{
    double c1 = 1.0 - pow(beta1, (double)t);
    double c2 = 1.0 - pow(beta2, (double)t);
    for (int p = 0; p < P; ++p) {
        mom1[p] = beta1 * mom1[p] + (1.0 - beta1) * g[p];
        mom2[p] = beta2 * mom2[p] + (1.0 - beta2) * g[p] * g[p];
        double mh = mom1[p] / c1;
        double vh = mom2[p] / c2;
        th[p] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers:  */
/* as easy as 1, 2, 3", SC 2011): the counter-based generator both the      */
/* device fit and this oracle draw the fit's random numbers from.           */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 64 random bits for (stream, a, b) under a 64-bit seed. */
static uint64_t rand64(uint64_t seed, uint32_t stream, uint64_t a, uint32_t b)
{
    uint32_t ctr[4] = {(uint32_t)a, (uint32_t)(a >> 32), b, stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    orc_philox4x32_10(ctr, key, o);
    return (uint64_t)o[0] | ((uint64_t)o[1] << 32);
}

enum { ORC_STREAM_SAMPLE = 1, ORC_STREAM_INIT = 2, ORC_STREAM_BATCH = 3 };

/* Indices of the fit sample: k draws with replacement, draw j = r(j) mod n. */
void orc_sample_indices(uint64_t seed, int64_t n, int64_t k, int64_t* idx)
{
    for (int64_t j = 0; j < k; ++j) idx[j] = (int64_t)(rand64(seed, ORC_STREAM_SAMPLE, (uint64_t)j, 0) % (uint64_t)n);
}

/* Batch of a training step: B draws with replacement from [0, k). */
void orc_batch_indices(uint64_t seed, int64_t step, int64_t k, int64_t B, int64_t* idx)
{
    for (int64_t b = 0; b < B; ++b)
        idx[b] = (int64_t)(rand64(seed, ORC_STREAM_BATCH, (uint64_t)b, (uint32_t)step) % (uint64_t)k);
}

/* Uniform [-bound, bound) initial weight for packed parameter p. */
double orc_init_uniform(uint64_t seed, int64_t p, double bound)
{
    uint64_t r = rand64(seed, ORC_STREAM_INIT, (uint64_t)p, 0);
    double u = (double)(uint32_t)(r >> 40) * (1.0 / 16777216.0); /* 24 bits */
    return bound * (2.0 * u - 1.0);
}

/* Slot of each normalised position F (orc_slot applied elementwise). */
void orc_slots_from_F(const double* F, int64_t n, double M, uint32_t* slots)
{
    for (int64_t i = 0; i < n; ++i) slots[i] = orc_slot(F[i], M);
}
