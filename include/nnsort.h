/*
 * nnsort.h -- C ABI of an MI355X (gfx950) implementation of NN-sort, the
 * learned sort of Zhu, Zhang, Zhou and Liu, "Deep Learning Service for
 * Efficient Data Distribution Aware Sorting" (arXiv 1907.08817).
 *
 * Problem statement (Sec. 2, Procedure NN-sort): given an array A, a learned
 * model f, a relaxation factor m, an iteration limit eps and a threshold tau,
 * produce A' = A in ascending order.  f maps each key to its expected
 * position; keys are placed at round(f * m) (first arrival wins), conflicts are
 * re-mapped for at most eps rounds while more than tau remain, the remainder is
 * sorted conventionally and everything is merged by the polish phase.
 *
 * Conventions shared by every entry point
 *  - Keys are 64-bit: IEEE binary64 (NNSORT_F64) or unsigned 64-bit integers
 *    (NNSORT_U64).  Output order is the IEEE 754-2019 totalOrder for binary64
 *    (-NaN < -Inf < ... < -0 < +0 < ... < +Inf < +NaN) and numeric order for
 *    uint64; the output holds the input's bit patterns.
 *  - Pointers named d_* are device pointers on the current HIP device; the
 *    caller owns them.  nnsort_model and nnsort_stats live in host memory.
 *  - Work is ordered on `stream` (a hipStream_t, NULL = the null stream).
 *    Calls that report statistics, or that need a device count to decide the
 *    next step (the tau test, a fallback), synchronise that stream before
 *    returning.
 *  - The library never allocates device memory: every call that needs scratch
 *    takes a caller-provided workspace d_ws of at least the size that
 *    nnsort_workspace_size() reports, aligned to 256 bytes.  Calls on one
 *    workspace must not overlap.  The sorts keep, per host thread and device,
 *    until the process ends: a 256-byte pinned host buffer (hipHostMalloc) and
 *    an event for reading back counters mid-sort, a pinned copy of the device
 *    model (about 35 KB) and an event for its upload, and twenty timing
 *    events; and per host thread the last model they prepared (about 52 KB
 *    of host memory), reused when the next model has the same bytes.  The
 *    no-allocation entry point uses none of them.
 *  - Every function returns an nnsort_status; no exception crosses the ABI.
 *    nnsort_strerror() describes a status.  On error the output is
 *    unspecified.
 */
#ifndef NNSORT_H
#define NNSORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NNSORT_ABI_VERSION 1
#define NNSORT_MAX_HIDDEN 64
#define NNSORT_MAX_EPS 8

typedef enum { NNSORT_F64 = 0, NNSORT_U64 = 1 } nnsort_dtype;

typedef enum {
    NNSORT_OK = 0,
    NNSORT_EINVAL = -1,      /* bad argument (null pointer, size, range) */
    NNSORT_EWORKSPACE = -2,  /* workspace smaller than nnsort_workspace_size(), or not 256-byte aligned */
    NNSORT_EHIP = -3,        /* a HIP runtime call failed */
    NNSORT_EMODEL = -4,      /* malformed model (hidden width, version) */
    NNSORT_EIO = -5,         /* model file could not be read or written */
    NNSORT_EINTERNAL = -6,   /* a device-side consistency check failed */
    NNSORT_ETOOBIG = -7      /* input beyond the static scratch of nnsort_sort_with_model_noalloc */
} nnsort_status;

typedef enum { NNSORT_FORM_FP32 = 0, NNSORT_FORM_BF16 = 1, NNSORT_FORM_PWL = 2 } nnsort_form;

/* Parameters of the sorting procedure (Sec. 2, Procedure NN-sort).
 *  m          relaxation factor; slots = round(F * m * n), S = round(m n) + 1
 *             slots (the paper uses m = 1.25, Sec. 4.1).
 *  eps        maximum number of mapping rounds, 1..8 (the paper finds 2 or 3
 *             best, Sec. 2 Sorting Phase and Sec. 4.2 Exp-4).
 *  tau        a round runs only while the conflict array holds more than tau
 *             keys; n <= tau sorts conventionally.
 *  form       model inference arithmetic: NNSORT_FORM_FP32 (FP32 vector ALU,
 *             one fixed operation order), NNSORT_FORM_BF16 (hidden layer on
 *             bf16 matrix cores, FP32 accumulation) or NNSORT_FORM_PWL (the
 *             FP64 model through its piecewise-linear form: a one-input ReLU
 *             network is affine between at most (H + 1)^2 breakpoints, which
 *             the call computes from the weights on the device; each key then
 *             costs a search among the breakpoints and one FP64 fma).
 *  bf16_terms number of bf16 terms each hidden-1 activation is split into
 *             for the matrix product (1..3).
 *  stats_level 0: none; 1: round counts and phase times; 2: also the mean
 *             |F n - rank| / n of the model over the sorted output. */
typedef struct {
    double m;
    int32_t eps;
    int32_t form;
    int64_t tau;
    int32_t bf16_terms;
    int32_t stats_level;
} nnsort_sort_params;

/* Parameters of the on-device fit of f (Sec. 2, Training; Sec. 4.1,
 * Training details: a regression MLP trained with Adam).
 *  hidden       width H of both hidden layers (1..64).
 *  sample_frac  fraction of n drawn (with replacement) as the training sample.
 *  batch, steps Adam mini-batch size and number of steps.
 *  lr           Adam learning rate (beta1 0.9, beta2 0.999, eps 1e-8).
 *  seed         seed of the Philox4x32-10 streams (sample, init, batches).
 *  loss         0: mean squared error; 1: Huber with threshold huber_delta.
 *  init         0: uniform(+-1/sqrt(fan_in)); 1 and 2: ramps forming the
 *               piecewise-linear interpolant of the sample CDF through H+1
 *               knots, placed by greedy maximum-deviation splitting (1) or at
 *               the quantiles j/H (2). */
typedef struct {
    int32_t hidden;
    int32_t batch;
    double sample_frac;
    int32_t steps;
    float lr;
    uint64_t seed;
    int32_t loss;
    float huber_delta;
    int32_t init;
    int32_t reserved;
} nnsort_fit_params;

/* The model f: F(x) = w3 . relu(W2 relu(w1 x + b1) + b2) + b3 with
 * x = clamp((key - lo) * inv_range, 0, 1) computed in FP64 (the input phase,
 * Sec. 2).  w2[i * hidden + j] is the weight from hidden-1 unit j to hidden-2
 * unit i; entries beyond hidden are ignored.  Host memory. */
typedef struct {
    int32_t version;  /* NNSORT_ABI_VERSION */
    int32_t hidden;
    double lo;
    double inv_range;
    float w1[NNSORT_MAX_HIDDEN];
    float b1[NNSORT_MAX_HIDDEN];
    float w2[NNSORT_MAX_HIDDEN * NNSORT_MAX_HIDDEN];
    float b2[NNSORT_MAX_HIDDEN];
    float w3[NNSORT_MAX_HIDDEN];
    float b3;
    float reserved[3];
} nnsort_model;

/* Statistics of one sort.  collided[r] is |c_{r+1}|, the conflict array after
 * round r+1; residue = |last conflict array|, so residue / n is the paper's
 * traditional sorting rate (Sec. 4.1, Eq. (ratio)).  Times are milliseconds
 * between HIP events on the call's stream.
 * Not reported: the out-of-order count e_r of each o_r (Sec. 3).  Here a
 * slot range's keys reach its workgroup in the order of the partition's
 * atomic ranks, not in input order, so which of a slot's keys sits in which
 * o_r (and so e_r) is not the paper's first-arrival assignment; the round
 * counts, which depend only on each slot's multiplicity, are. */
typedef struct {
    int64_t n;
    int32_t rounds;
    int32_t form;
    int64_t collided[NNSORT_MAX_EPS];
    int64_t placed[NNSORT_MAX_EPS];
    int64_t residue;
    int64_t unmapped;        /* keys with no slot (F not a number, or a
                                caller-given 0xFFFFFFFF) */
    int64_t big_buckets;     /* slot ranges too dense for one LDS tile */
    int64_t big_bucket_keys; /* keys sorted by the residue path for that reason */
    int64_t boundary_keys;   /* keys moved by the tile-boundary fix-up */
    int32_t fallback;        /* 0: the boundary fix-up settled every overlap;
                                1: overlaps beyond neighbouring ranges (or a
                                zone over 4096 keys); 2: blocks out of order
                                after the fix-up (ranges far out of value
                                order, keys without a slot that are not the
                                extremes).  In both cases the whole output
                                was then sorted by radix. */
    int32_t range_resorts;   /* slot ranges sorted whole in LDS: those with a
                                slot of more than 32 keys, and those whose
                                neighbour-tile merges did not settle */
    double pos_err;          /* stats_level 2: mean |F(key) n - rank| / n */
    /* stats_level >= 1: t_infer = the map kernel; t_place = the partition of
     * keys by slot range and the gather of dense ranges; t_polish = rounds and
     * polish of every range in LDS; t_residue = the conventional sort of the
     * residue path and its placement; t_merge = the check and repair of the
     * boundaries between neighbouring ranges; t_total = the whole call. */
    double t_infer_ms, t_place_ms, t_polish_ms, t_residue_ms, t_merge_ms, t_total_ms;
    double t_fit_ms;         /* nnsort_sort: the fit that preceded the sort (0 otherwise) */
} nnsort_stats;

/* Default parameters (m 1.25, eps 3, tau 1024, FP32 form, 3 bf16 terms;
 * hidden 32, sample 1%, batch 65536, 200 steps, lr 1e-7, MSE, ramp init). */
void nnsort_default_params(nnsort_sort_params* sort_params, nnsort_fit_params* fit_params);

/* Bytes of device workspace needed to sort (and, if fit_params is not NULL,
 * also fit) n keys.  Pure host computation. */
int nnsort_workspace_size(int64_t n, nnsort_dtype dtype, const nnsort_sort_params* sort_params,
                          const nnsort_fit_params* fit_params, size_t* bytes);

/* Fit f on the device from a random sample of d_keys[0..n) (Sec. 2,
 * Training): Philox4x32-10 sample with replacement, sort of the sample,
 * labels (j + 0.5)/k for the j-th smallest of the k finite sampled keys,
 * lo/inv_range from the sample's extremes, then `steps` Adam steps on
 * batches drawn with replacement.  Writes the model to *out (host): the
 * parameters with the lowest batch loss seen, unless the FP64 model with
 * them moves F backwards along the sorted sample more than with the initial
 * parameters (then those).  Synchronises the stream.  EINVAL: n < 1, null
 * pointers, hidden not 8, 16, 32 or 64, sample_frac <= 0, batch < 1,
 * steps < 0, sample_frac * n >= 2^32 - 1.  EWORKSPACE: d_ws smaller than nnsort_workspace_size() with
 * these fit parameters, or not 256-byte aligned. */
int nnsort_fit(const void* d_keys, int64_t n, nnsort_dtype dtype, const nnsort_fit_params* params,
               nnsort_model* out, void* d_ws, size_t ws_bytes, void* stream);

/* nnsort_fit that also copies the batch loss before each Adam step into
 * loss_history[0 .. min(steps, history_len)) (host memory, FP32). */
int nnsort_fit_history(const void* d_keys, int64_t n, nnsort_dtype dtype,
                       const nnsort_fit_params* params, nnsort_model* out, void* d_ws,
                       size_t ws_bytes, float* loss_history, int history_len, void* stream);

/* Sort d_in[0..n) into d_out[0..n) with a given model (Sec. 2, Procedure
 * NN-sort: input, sorting and polish phases).  d_in is read only; d_in and
 * d_out must not overlap (EINVAL).  n = 0 is a no-op.  stats may be NULL.
 * EINVAL: n < 0, null pointers with n > 0, m <= 0, eps outside 1..8,
 * tau < 0, m * n >= 2^32 - 1. */
int nnsort_sort_with_model(const nnsort_model* model, const void* d_in, void* d_out, int64_t n,
                           nnsort_dtype dtype, const nnsort_sort_params* params, void* d_ws,
                           size_t ws_bytes, nnsort_stats* stats, void* stream);

/* nnsort_sort_with_model without a caller workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  The sort runs in a static 64 MiB device
 * array of the library (one per GPU, held until the process ends): n may be
 * at most the largest count whose nnsort_workspace_size(n, dtype, params,
 * NULL) is at most 64 MiB (about 1.5 million keys at m = 1.25); larger inputs
 * return NNSORT_ETOOBIG before any device work.  The call allocates nothing:
 * no device memory, no events (stats carries counts but no phase times).
 * Every call on one GPU shares that GPU's array, which keeps the previous
 * call's contents (each call initialises what it reads): calls that overlap
 * on one GPU, from several streams or threads, race and must not be issued.
 * Otherwise as nnsort_sort_with_model (same checks, synchronises the stream). */
int nnsort_sort_with_model_noalloc(const nnsort_model* model, const void* d_in, void* d_out, int64_t n,
                                   nnsort_dtype dtype, const nnsort_sort_params* params, nnsort_stats* stats,
                                   void* stream);

/* Fit on d_in, then sort it: nnsort_fit followed by nnsort_sort_with_model.
 * The fitted model is copied to *model_out when it is not NULL; stats->
 * t_fit_ms is the fit and stats->t_total_ms the fit plus the sort. */
int nnsort_sort(const void* d_in, void* d_out, int64_t n, nnsort_dtype dtype,
                const nnsort_fit_params* fit_params, const nnsort_sort_params* sort_params,
                void* d_ws, size_t ws_bytes, nnsort_model* model_out, nnsort_stats* stats,
                void* stream);

/* The input and sorting phases' map only (the test hook that returns the
 * predicted slots; it also returns F, so it is named nnsort_predict): for each key, F(key) (the model's
 * normalised position, as a double; NaN for unmappable keys) and its slot
 * round(F m n) clamped to [0, m n] (0xFFFFFFFF for unmappable keys).  Either
 * output may be NULL.  d_ws must hold nnsort_model_device_bytes() bytes (the
 * device copy of the model, and the piecewise-linear form's table), aligned
 * to 256 bytes (EWORKSPACE otherwise).  Synchronises the stream. */
size_t nnsort_model_device_bytes(void);
int nnsort_predict(const nnsort_model* model, const void* d_in, int64_t n, nnsort_dtype dtype,
                   const nnsort_sort_params* params, uint32_t* d_slots, double* d_F, void* d_ws,
                   size_t ws_bytes, void* stream);

/* The sorting and polish phases driven by caller-given slots (one per key,
 * each < round(m n) + 1, or 0xFFFFFFFF for "no slot"), e.g. from a closed-form
 * model.  Otherwise as nnsort_sort_with_model.  EINVAL if a slot is out of
 * range (checked on the device). */
int nnsort_sort_with_slots(const uint32_t* d_slots, const void* d_in, void* d_out, int64_t n,
                           nnsort_dtype dtype, const nnsort_sort_params* params, void* d_ws,
                           size_t ws_bytes, nnsort_stats* stats, void* stream);

/* The conventional sort of the procedure's last conflict array: an LSD radix
 * sort over the 64-bit order keys, here applied to a whole array.  Needs
 * nnsort_radix_workspace_size(n) bytes of workspace. */
size_t nnsort_radix_workspace_size(int64_t n);
int nnsort_radix_sort(const void* d_in, void* d_out, int64_t n, nnsort_dtype dtype, void* d_ws,
                      size_t ws_bytes, void* stream);

/* Model pieces for training (Sec. 2, Training).  theta is the packed FP32
 * parameter vector w1[H] | b1[H] | W2[H*H] (row = hidden-2 unit) | b2[H] |
 * w3[H] | b3 on the device (H*H + 4H + 1 floats).  x holds B normalised
 * inputs in [0, 1] (FP64, split into two FP32 terms inside).
 *
 * nnsort_mlp_forward: d_F[b] = F(x[b]) in FP32 with the FP32 form's
 *   operation order; d_saved (nnsort_mlp_saved_floats(H, B) floats) receives
 *   what the backward pass needs (may be NULL when no backward follows).
 * nnsort_mlp_backward: given dL/dF in d_gF[0..B), writes dL/dtheta to
 *   d_gtheta (overwritten, not accumulated).  Needs the d_saved of the
 *   matching forward and nnsort_mlp_backward_ws_floats(H, B) floats of
 *   workspace.
 * nnsort_loss_grad: loss 0 MSE mean((F - y)^2), 1 Huber(delta) mean (the
 *   paper's Eq. (loss)); writes dL/dF to d_gF and the loss to d_loss[0]
 *   (FP32); d_ws holds nnsort_loss_ws_floats() floats of partial sums.
 * nnsort_adam_step: one bias-corrected Adam update of theta in place, t is
 *   the 1-based step. */
size_t nnsort_mlp_saved_floats(int hidden, int64_t batch);
size_t nnsort_mlp_backward_ws_floats(int hidden, int64_t batch);
int nnsort_mlp_forward(int hidden, const float* d_theta, const double* d_x, int64_t batch,
                       float* d_F, float* d_saved, void* stream);
int nnsort_mlp_backward(int hidden, const float* d_theta, const double* d_x, int64_t batch,
                        const float* d_saved, const float* d_gF, float* d_gtheta, float* d_ws,
                        void* stream);
size_t nnsort_loss_ws_floats(void);
int nnsort_loss_grad(const float* d_F, const float* d_y, int64_t batch, int loss, float delta,
                     float* d_gF, float* d_loss, float* d_ws, void* stream);
int nnsort_adam_step(float* d_theta, const float* d_g, float* d_m1, float* d_m2, int64_t count,
                     int64_t t, float lr, float beta1, float beta2, float eps, void* stream);

/* One training step of the fit as nnsort_fit runs it for hidden = 32 or 64
 * (one fused kernel on the FP32 matrix cores), without the Adam update: the
 * batch of `batch` entries drawn from the sample d_x[0..k) / d_y[0..k) with
 * replacement (entry b is index Philox4x32-10(seed, stream 3, counter (b,
 * step)) mod k), its loss (0 MSE, 1 Huber(delta), mean over the batch) into
 * d_loss[0] and dL/dtheta into d_gtheta (P floats, overwritten).  A test hook
 * for the gradient the fit applies.  d_ws holds
 * nnsort_fit_gradient_ws_floats(hidden, batch) floats.  EINVAL: hidden not 32
 * or 64, batch, k or step < 1, null pointers; EWORKSPACE: d_ws too small. */
size_t nnsort_fit_gradient_ws_floats(int hidden, int64_t batch);
int nnsort_fit_gradient(int hidden, const float* d_theta, const double* d_x, const float* d_y, int64_t k,
                        int64_t batch, uint64_t seed, int64_t step, int loss, float delta, float* d_gtheta,
                        float* d_loss, float* d_ws, size_t ws_floats, void* stream);

/* Save or load a model as a small binary file (magic "NNSM", version,
 * hidden, lo, inv_range, then the FP32 weights).  EIO on file errors,
 * EMODEL on a malformed file. */
int nnsort_model_save(const nnsort_model* model, const char* path);
int nnsort_model_load(nnsort_model* model, const char* path);

const char* nnsort_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* NNSORT_H */
