// C ABI of libnnsort: argument checks, workspace planning and the order of
// kernel launches for NN-sort (Sec. 2, Procedure NN-sort and polish; Sec. 2,
// Training).  No device memory is allocated here: every buffer is carved out
// of the caller's workspace.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "nnsort_internal.h"

namespace nns {
// launchers defined in the .hip translation units
hipError_t fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);
hipError_t fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t st);
hipError_t launch_classify(const int64_t* d_start, uint32_t* d_cnt, int64_t NB, int64_t big_max, int32_t* d_seglist,
                           int32_t* d_bigbucket, int32_t* d_halflist, uint64_t* d_bsum, uint64_t* d_counters,
                           hipStream_t st);
size_t classify_ws_words(int64_t NB);
hipError_t launch_big_counts(const uint32_t* d_hist, int64_t big_count, int eps, uint64_t* d_counters,
                             hipStream_t st);
size_t polish_part_words(int64_t NB);
hipError_t launch_polish_small(const int64_t* d_start, int64_t NB, const uint64_t* d_K, const uint32_t* d_S, int eps,
                               uint64_t* d_out, bool is_f64, uint32_t* d_part, uint64_t* d_counters, hipStream_t st);
hipError_t launch_polish_half(const int64_t* d_start, const int32_t* d_halflist, int64_t n_half, const uint64_t* d_K,
                              const uint32_t* d_S, int eps, uint64_t* d_out, bool is_f64, uint32_t* d_part,
                              uint64_t* d_counters, hipStream_t st);
hipError_t launch_sum_parts(const uint32_t* d_part, const uint32_t* d_cnt, int64_t NB, int eps, uint64_t* d_counters,
                            hipStream_t st);
hipError_t launch_boundary_plan(const uint64_t* d_out, bool is_f64, int64_t base, const int64_t* d_start,
                                const int32_t* d_seglist, int64_t K, void* d_zones, uint64_t* d_counters,
                                hipStream_t st);
hipError_t launch_boundary_merge(uint64_t* d_out, bool is_f64, const void* d_zones, int64_t K,
                                const uint64_t* d_counters, hipStream_t st);
hipError_t launch_junction_check(const uint64_t* d_out, bool is_f64, int64_t base, const int64_t* d_start,
                                 const int32_t* d_seglist, int64_t K, const void* d_zones, int64_t n, int64_t back,
                                 bool unmapped, uint64_t* d_counters, hipStream_t st);
size_t zone_bytes();
size_t partition_hist_words(int64_t n);
hipError_t partition_by_range(const uint64_t* in_keys, const uint32_t* in_slots, int64_t n, uint32_t NB, bool is_f64,
                              uint64_t* K0, uint32_t* S0, uint64_t* K1, uint32_t* S1, uint32_t* blockhist,
                              int* which, hipStream_t st, bool first_counted = false);
int range_passes(uint32_t NB, int* shifts, uint32_t* masks, int* widths);
hipError_t launch_range_bounds(const uint32_t* d_sorted_slots, int64_t n, uint32_t NB, int64_t* d_start,
                               hipStream_t st);
hipError_t launch_check_slots(const uint32_t* d_slots, int64_t n, int64_t S, uint64_t* d_bad, hipStream_t st);
hipError_t launch_big_chunks(const int32_t* d_bigbucket, int64_t big_count, const int64_t* d_start,
                             int64_t* d_chunk_pref, int64_t* d_gpref, hipStream_t st);
hipError_t launch_big_gather(const int32_t* d_bigbucket, int64_t big_count, int64_t nchunks,
                             const int64_t* d_chunk_pref, const int64_t* d_gpref, const int64_t* d_start,
                             const uint64_t* d_K, const uint32_t* d_S, uint32_t* d_hist, uint64_t* d_G,
                             hipStream_t st);
hipError_t launch_big_place(const int32_t* d_bigbucket, int64_t big_count, int64_t nchunks,
                            const int64_t* d_chunk_pref, const int64_t* d_gpref, const int64_t* d_start,
                            const uint64_t* d_Gs, int64_t u_neg, uint64_t* d_out, bool is_f64, hipStream_t st);
int seg_rounds(int64_t max_len, int64_t run0);
hipError_t seg_sort(const int64_t* d_chunk_pref, const int64_t* d_gpref, int64_t nseg, int64_t nchunks,
                    int rounds, int64_t run0, uint64_t* d_G, uint64_t* d_tmp, hipStream_t st,
                    const int32_t* d_seg_range = nullptr, const int64_t* d_range_start = nullptr,
                    SegOut fo = SegOut{nullptr, 0, 0});
hipError_t launch_count_neg(const uint64_t* d_K, const int64_t* d_start, uint32_t NB, int64_t n, uint64_t* d_count,
                            hipStream_t st);
hipError_t launch_copy_u64(const uint64_t* d_in, uint64_t* d_out, int64_t n, hipStream_t st);
hipError_t launch_pos_err_sum(const double* d_F, int64_t n, double* d_sum, hipStream_t st);
// fit
hipError_t launch_sample(const void* d_in, int64_t n, bool is_f64, uint64_t seed, int64_t k, uint64_t* d_out,
                         uint64_t* d_count, hipStream_t st);
hipError_t launch_one_segment(int64_t* d_seg, int64_t nchunks, int64_t k, hipStream_t st);
hipError_t launch_make_xy(const uint64_t* d_sorted, int64_t k, bool is_f64, double* d_x, float* d_y, double* d_lohi,
                          hipStream_t st);
hipError_t launch_init(float* d_theta, int H, int init, uint64_t seed, const double* d_x, int64_t k,
                       int64_t* d_knots, void* d_knotws, hipStream_t st);
size_t knot_ws_bytes();
size_t mlp_backward_ws_floats(int H, int64_t B);
size_t loss_ws_floats();
hipError_t launch_loss_grad(const float* d_F, const float* d_y, int64_t B, int loss, float delta, float* d_gF,
                            float* d_loss, float* d_partial, hipStream_t st);
size_t fit_loss_ws_floats(int64_t B);
hipError_t launch_fit_step_forward(int H, const float* d_theta, const double* d_x, const float* d_y, int64_t k,
                                   uint64_t seed, int64_t step, int64_t B, double* d_bx, float* d_saved, int loss,
                                   float delta, float* d_gF, float* d_loss, float* d_partial, float* d_best, int P,
                                   float* d_best_loss, hipStream_t st);
hipError_t launch_mlp_backward_adam(int H, float* d_theta, const double* d_x, int64_t B, const float* d_saved,
                                    const float* d_gF, float* d_ws, float* d_m1, float* d_m2, int64_t t, float lr,
                                    float b1, float b2, float eps, hipStream_t st);
size_t disorder_ws_doubles();
hipError_t launch_disorder(const double* d_F, int64_t k, double* d_ws, hipStream_t st);
bool fit_step_mfma(int H);
int fit_step_groups(int64_t B);
hipError_t launch_fit_gradient(int H, const float* d_theta, const double* d_x, const float* d_y, int64_t k,
                               int64_t B, uint64_t seed, int64_t t, int loss, float delta, float* d_part,
                               float* d_loss_part, float* d_gtheta, float* d_loss, hipStream_t st);
hipError_t launch_fit_step_mfma(int H, float* d_theta, const double* d_x, const float* d_y, int64_t k, int64_t B,
                                uint64_t seed, int64_t t, int loss, float delta, float lr, float b1, float b2,
                                float eps, float* d_part, float* d_loss_part, float* d_m1, float* d_m2, float* d_best,
                                float* d_best_loss, float* d_loss, hipStream_t st);
}  // namespace nns

using namespace nns;

namespace {

thread_local char g_last_error[256] = "";

int fail_hip(hipError_t e, const char* where) {
    std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s", where, hipGetErrorString(e));
    return NNSORT_EHIP;
}

#define NNS_HIP(call)                                   \
    do {                                                \
        hipError_t _e = (call);                         \
        if (_e != hipSuccess) return fail_hip(_e, #call); \
    } while (0)

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Device copy of the model, followed by the piecewise-linear form's table.
size_t model_region_bytes() { return align256(sizeof(DevModel)) + align256(sizeof(PwlTable)); }
PwlTable* pwl_table_of(void* model_region) { return (PwlTable*)((char*)model_region + align256(sizeof(DevModel))); }

int64_t num_slots(int64_t n, double m) {
    double M = m * (double)n;
    double t = std::trunc(M);
    if (M - t >= 0.5) t += 1.0;
    return (int64_t)t + 1;
}

bool valid_sort_params(const nnsort_sort_params* p, int64_t n) {
    if (!p) return false;
    if (!(p->m > 0.0) || !std::isfinite(p->m)) return false;
    if (p->eps < 1 || p->eps > NNSORT_MAX_EPS) return false;
    if (p->tau < 0) return false;
    if (p->form != NNSORT_FORM_FP32 && p->form != NNSORT_FORM_BF16 && p->form != NNSORT_FORM_PWL) return false;
    if (p->bf16_terms < 1 || p->bf16_terms > 3) return false;
    if (n >= (int64_t)0xFFFFFFFF) return false;
    if (p->m * (double)n >= 4294967294.0) return false;
    return true;
}

int model_width(int H) { return H <= 32 ? 32 : 64; }

int check_model(const nnsort_model* m) {
    if (!m) return NNSORT_EINVAL;
    if (m->version != NNSORT_ABI_VERSION || m->hidden < 1 || m->hidden > NNSORT_MAX_HIDDEN) return NNSORT_EMODEL;
    return NNSORT_OK;
}

// A model with a non-finite parameter maps no key: every key then stays in
// the conflict arrays and is sorted conventionally, whatever the form.
bool model_is_finite(const nnsort_model* m) {
    const int H = m->hidden;
    if (!std::isfinite(m->lo) || !std::isfinite(m->inv_range) || !std::isfinite(m->b3)) return false;
    for (int j = 0; j < H; ++j) {
        if (!std::isfinite(m->w1[j]) || !std::isfinite(m->b1[j]) || !std::isfinite(m->b2[j]) ||
            !std::isfinite(m->w3[j]))
            return false;
        for (int k = 0; k < H; ++k)
            if (!std::isfinite(m->w2[j * H + k])) return false;
    }
    return true;
}

float bf16_rne(float v) {
    uint32_t u;
    std::memcpy(&u, &v, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    u &= 0xFFFF0000u;
    float r;
    std::memcpy(&r, &u, 4);
    return r;
}

// Smallest k with 2^k >= U, for U > 0.
int ceil_log2(double U) {
    int e;
    double f = std::frexp(U, &e);  // U = f 2^e, f in [0.5, 1)
    return f == 0.5 ? e - 1 : e;
}

// v 2^k, and whether that value is exact.  A normal v whose scaled exponent
// stays in the normal range is scaled exactly by adding k to its exponent
// field (the common case, and the one the per-call host time depends on: the
// BF16 operands take 2H^2 + 3H such scalings); everything else goes through
// ldexp and a round trip.
bool scaled_exact(float v, int k, float* out) {
    uint32_t u;
    std::memcpy(&u, &v, 4);
    const int e = (int)((u >> 23) & 0xFFu);
    if (e != 0 && e != 255 && e + k >= 1 && e + k <= 254) {
        u += (uint32_t)k << 23;
        std::memcpy(out, &u, 4);
        return true;
    }
    float s = std::ldexp(v, k);
    *out = s;
    return std::isfinite(s) && std::ldexp(s, -k) == v;
}

// The BF16 form's scaled operands (see DevModel).  Bounds: for x in [0, 1] a
// hidden-1 pre-activation, rounded in FP32, stays below (|w1| + |b1|)(1 + 2^-22);
// a hidden-2 pre-activation below (|b2| + sum_j |bf16(W2)| U1_j) plus the FP32
// accumulation error of 3H + 1 terms (< 2^-16 relative).  A margin of 1/64
// covers both; a looser bound only makes a scaled value smaller.
void bf16_operands(DevModel* d) {
    const int H = d->H;
    const double margin = 1.0 + 1.0 / 64.0;
    double U1[64];
    int k1[64], k2[64];
    for (int j = 0; j < H; ++j) {
        U1[j] = ((double)std::fabs(d->w1[j]) + (double)std::fabs(d->b1[j])) * margin;
        k1[j] = U1[j] > 0.0 ? ceil_log2(U1[j]) : 0;
    }
    for (int i = 0; i < H; ++i) {
        double U = std::fabs((double)d->b2[i]);
        for (int j = 0; j < H; ++j) U += std::fabs((double)bf16_rne(d->w2[i * H + j])) * U1[j];
        U *= margin;
        k2[i] = U > 0.0 ? ceil_log2(U) : 0;
    }
    bool ok = true;
    for (int j = 0; j < H && ok; ++j)
        ok = k1[j] > -100 && k1[j] < 100 && scaled_exact(d->w1[j], -k1[j], &d->w1s[j]) &&
             scaled_exact(d->b1[j], -k1[j], &d->b1s[j]);
    for (int i = 0; i < H && ok; ++i) {
        ok = k2[i] > -100 && k2[i] < 100 && scaled_exact(d->b2[i], -k2[i], &d->b2s[i]);
        d->w3s[i] = std::ldexp((double)d->w3[i], k2[i]);
        for (int j = 0; j < H && ok; ++j) {
            float a = bf16_rne(d->w2[i * H + j]), as;
            uint32_t bitsv;
            ok = scaled_exact(a, k1[j] - k2[i], &as);
            std::memcpy(&bitsv, &as, 4);
            ok = ok && (bitsv & 0xFFFFu) == 0 && std::fpclassify(as) != FP_SUBNORMAL;
            d->w2s[i * H + j] = as;
        }
    }
    d->bf16_scaled = ok ? 1 : 0;
    if (ok) return;
    for (int j = 0; j < H; ++j) {
        d->w1s[j] = d->w1[j];
        d->b1s[j] = d->b1[j];
        d->b2s[j] = d->b2[j];
        d->w3s[j] = (double)d->w3[j];
        for (int k = 0; k < H; ++k) d->w2s[j * H + k] = bf16_rne(d->w2[j * H + k]);
    }
}

// Device layout of the model, zero-padded to a width of 32 or 64.
void to_dev_model(const nnsort_model* m, DevModel* d) {
    std::memset(d, 0, sizeof(*d));
    int H = m->hidden, HP = model_width(H);
    d->H = HP;
    d->H_true = H;
    d->lo = m->lo;
    d->inv_range = m->inv_range;
    for (int j = 0; j < H; ++j) {
        d->w1[j] = m->w1[j];
        d->b1[j] = m->b1[j];
        d->b2[j] = m->b2[j];
        d->w3[j] = m->w3[j];
        for (int k = 0; k < H; ++k) d->w2[j * HP + k] = m->w2[j * H + k];
    }
    d->b3 = m->b3;
    bf16_operands(d);
}

}  // namespace

namespace nns {

// Merge rounds of the range-by-range sort of dense ranges beyond which the
// radix sort of the whole residue is used instead (ranges of up to 1M keys).
constexpr int kSegMaxRounds = 8;
constexpr int64_t kWideRunKeys = (int64_t)1 << 22;  // dense keys above which runs start at kSortRun

SortPlan plan_sort(int64_t n, double m) {
    SortPlan p{};
    p.n = n;
    p.S = num_slots(n, m);
    p.NB = (p.S + kBucketSlots - 1) / kBucketSlots;
    p.big_max = n / (kBucketCap + 1) + 1;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += align256(bytes);
        return at;
    };
    size_t nn = (size_t)(n > 0 ? n : 1);
    p.off_counters = take(kNumCounters * 8);
    p.off_cnt = take((size_t)p.NB * 4);
    p.off_start = take((size_t)(p.NB + 2) * 8);
    p.off_slots0 = take(nn * 4);
    p.off_S0 = take(nn * 4);
    p.off_K0 = take(nn * 8);
    p.off_K1 = take(nn * 8);
    p.off_phist = take(partition_hist_words(n) * 4);
    p.off_clsum = take(classify_ws_words(p.NB) * 8);
    p.off_seglist = take((size_t)p.NB * 4);
    p.off_bigbucket = take((size_t)p.big_max * 4);
    p.off_halflist = take((size_t)p.NB * 4);
    p.off_bigpref = take((size_t)(p.big_max + 1) * 2 * 8);
    p.off_part = take(polish_part_words(p.NB) * 4);
    p.off_zones = take((size_t)p.NB * zone_bytes());
    p.off_G = take(nn * 8);
    p.off_big_hist = take((size_t)p.big_max * kBucketSlots * 4);
    p.off_model = take(model_region_bytes());
    p.radix_bytes = radix_ws_bytes(n);
    p.off_radix = take(p.radix_bytes);
    p.total = o;
    return p;
}

}  // namespace nns

namespace {

constexpr int kMaxDevices = 64;
constexpr int kNumEvents = 10;

// Timing events of a sort call, created once per host thread and device and
// kept until the process ends: a call records and reads them, and waits for
// the last one before it returns, so the next call on the thread may record
// them again.  Set 0 serves the sort, set 1 the fit-then-sort call around it.
struct EventPool {
    hipEvent_t e[2][kNumEvents] = {};
    bool ready = false;
};
static thread_local EventPool t_event_pool[kMaxDevices];

hipEvent_t* event_pool(int set) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    EventPool& p = t_event_pool[dev];
    if (!p.ready) {
        hipEvent_t* all = &p.e[0][0];
        // timing only: no system-scope cache writeback at each record, which
        // otherwise leaves the GPU idle for several microseconds between the
        // kernels around it (the host reads these events' times only after
        // the stream has been synchronised)
        for (int i = 0; i < 2 * kNumEvents; ++i)
            if (hipEventCreateWithFlags(&all[i], hipEventDisableSystemFence) != hipSuccess) {
                for (int j = 0; j < i; ++j) (void)hipEventDestroy(all[j]);
                return nullptr;
            }
        p.ready = true;
    }
    return p.e[set];
}

struct Events {
    hipEvent_t* e = nullptr;
    bool on = false;
    hipStream_t st = nullptr;
    Events(bool enable, hipStream_t s, int set = 0) : st(s) {
        if (enable) e = event_pool(set);
        on = e != nullptr;
    }
    void mark(int i) {
        if (on) (void)hipEventRecord(e[i], st);
    }
    double ms(int a, int b) {
        float t = 0.0f;
        if (!on) return 0.0;
        if (hipEventElapsedTime(&t, e[a], e[b]) != hipSuccess) return 0.0;
        return (double)t;
    }
};

// Per-thread, per-device pinned host buffer for the mid-sort read of the
// counters, with an event that marks the copy's arrival: the host then waits
// for that copy alone while the GPU already polishes the small ranges.  Kept
// until the process ends.  Null when it cannot be set up; the caller then
// copies to pageable memory and synchronises the stream.
struct CounterStage {
    uint64_t* host = nullptr;
    hipEvent_t copied = nullptr;
};
static thread_local CounterStage t_counter_stage[kMaxDevices];

CounterStage* counter_stage() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    CounterStage& s = t_counter_stage[dev];
    if (!s.host) {
        void* p = nullptr;
        if (hipHostMalloc(&p, kNumCounters * sizeof(uint64_t), hipHostMallocDefault) != hipSuccess) return nullptr;
        if (hipEventCreateWithFlags(&s.copied, hipEventDisableTiming) != hipSuccess) {
            (void)hipHostFree(p);
            return nullptr;
        }
        s.host = (uint64_t*)p;
    }
    return &s;
}

// The device form of the last model a host thread prepared, so that repeated
// sorts with one model skip the host-side preparation (the BF16 operand
// scaling takes tens of microseconds).  A cached entry is used only when the
// caller's model matches it byte for byte.  Null when it cannot be allocated.
struct PreparedModel {
    nnsort_model key;
    DevModel dev;
    bool valid = false;
};

const DevModel* prepared_model(const nnsort_model* m) {
    static thread_local std::unique_ptr<PreparedModel> t;
    if (!t) t.reset(new (std::nothrow) PreparedModel());
    if (!t) return nullptr;
    if (!t->valid || std::memcmp(&t->key, m, sizeof(nnsort_model)) != 0) {
        to_dev_model(m, &t->dev);
        std::memcpy(&t->key, m, sizeof(nnsort_model));
        t->valid = true;
    }
    return &t->dev;
}

// Per-thread, per-device pinned host copy of the device model, read into
// the workspace by a copy kernel on the call's stream (a copy engine's
// transfer would add tens of microseconds of latency before the map kernel);
// an event marks the copy's end, which the next call on the thread waits for
// before it writes the buffer again.
struct ModelStage {
    DevModel* host = nullptr;
    const uint64_t* dev_view = nullptr;  // the buffer's device address
    hipEvent_t done = nullptr;
    bool pending = false;
};
static thread_local ModelStage t_model_stage[kMaxDevices];

ModelStage* model_stage() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    ModelStage& s = t_model_stage[dev];
    if (!s.host) {
        void* p = nullptr;
        void* dp = nullptr;
        if (hipHostMalloc(&p, sizeof(DevModel), hipHostMallocDefault) != hipSuccess) return nullptr;
        if (hipHostGetDevicePointer(&dp, p, 0) != hipSuccess ||
            hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) {
            (void)hipHostFree(p);
            return nullptr;
        }
        s.host = (DevModel*)p;
        s.dev_view = (const uint64_t*)dp;
    }
    return &s;
}

// Device copy of a model for a sort, written to dmodel on stream st.
// allocating = false (the no-allocation entry point) prepares it in place
// and copies from pageable memory.
hipError_t upload_model(const nnsort_model* m, DevModel* dmodel, bool allocating, hipStream_t st,
                        int* width, int* scaled) {
    const DevModel* dev = allocating ? prepared_model(m) : nullptr;
    if (!dev) {
        DevModel hm;
        to_dev_model(m, &hm);
        *width = hm.H;
        *scaled = hm.bf16_scaled;
        return hipMemcpyAsync(dmodel, &hm, sizeof(hm), hipMemcpyHostToDevice, st);
    }
    *width = dev->H;
    *scaled = dev->bf16_scaled;
    ModelStage* ms = model_stage();
    if (!ms) return hipMemcpyAsync(dmodel, dev, sizeof(DevModel), hipMemcpyHostToDevice, st);
    if (ms->pending) {
        hipError_t e = hipEventSynchronize(ms->done);
        if (e != hipSuccess) return e;
        ms->pending = false;
    }
    std::memcpy(ms->host, dev, sizeof(DevModel));
    static_assert(sizeof(DevModel) % 8 == 0, "copied in 8-byte words");
    hipError_t e = launch_copy_u64(ms->dev_view, (uint64_t*)dmodel, (int64_t)(sizeof(DevModel) / 8), st);
    if (e != hipSuccess) return e;
    e = hipEventRecord(ms->done, st);
    ms->pending = e == hipSuccess;
    return e;
}

// Conventional sort of everything (no round runs when n <= tau).
int plain_sort(const void* d_in, void* d_out, int64_t n, bool is_f64, void* d_ws, size_t ws_bytes,
               hipStream_t st) {
    int mode = is_f64 ? 1 : 2;
    if (ws_bytes < radix_ws_bytes(n)) return NNSORT_EWORKSPACE;
    NNS_HIP(radix_sort((const uint64_t*)d_in, (uint64_t*)d_out, n, mode, mode, d_ws, ws_bytes, st));
    return NNSORT_OK;
}

// allocating = false: the no-allocation entry point (no timing events, and
// the mid-sort counter read goes to pageable memory).
int sort_impl(const nnsort_model* model, const uint32_t* given_slots, const void* d_in, void* d_out, int64_t n,
              nnsort_dtype dtype, const nnsort_sort_params* prm, void* d_ws, size_t ws_bytes, nnsort_stats* stats,
              hipStream_t st, bool allocating = true) {
    if (n < 0 || (n > 0 && (!d_in || !d_out))) return NNSORT_EINVAL;
    if (dtype != NNSORT_F64 && dtype != NNSORT_U64) return NNSORT_EINVAL;
    if (!valid_sort_params(prm, n)) return NNSORT_EINVAL;
    if (model) {
        int rc = check_model(model);
        if (rc) return rc;
    }
    if (n > 0) {
        const char* a = (const char*)d_in;
        const char* b = (const char*)d_out;
        if (a < b + n * 8 && b < a + n * 8) return NNSORT_EINVAL;  // overlapping buffers
    }
    const bool is_f64 = dtype == NNSORT_F64;
    const int eps = prm->eps;
    nnsort_stats S{};
    S.n = n;
    S.form = prm->form;
    Events ev(allocating && stats && prm->stats_level >= 1, st);
    ev.mark(0);
    if (n == 0) {
        if (stats) *stats = S;
        return NNSORT_OK;
    }
    if (n <= prm->tau) {  // count(w) > tau fails at once: conventional sort only
        int rc = plain_sort(d_in, d_out, n, is_f64, d_ws, ws_bytes, st);
        if (rc) return rc;
        ev.mark(6);
        NNS_HIP(hipStreamSynchronize(st));
        S.rounds = 0;
        S.residue = n;
        S.t_total_ms = ev.ms(0, 6);
        if (stats) *stats = S;
        return NNSORT_OK;
    }

    SortPlan P = plan_sort(n, prm->m);
    if (!d_ws || ws_bytes < P.total || ((uintptr_t)d_ws & 255u)) return NNSORT_EWORKSPACE;
    char* ws = (char*)d_ws;
    uint64_t* counters = (uint64_t*)(ws + P.off_counters);
    uint32_t* cnt = (uint32_t*)(ws + P.off_cnt);
    int64_t* start = (int64_t*)(ws + P.off_start);
    uint32_t* slots0 = (uint32_t*)(ws + P.off_slots0);
    uint32_t* S0 = (uint32_t*)(ws + P.off_S0);
    uint64_t* K0 = (uint64_t*)(ws + P.off_K0);
    uint64_t* K1 = (uint64_t*)(ws + P.off_K1);
    uint32_t* phist = (uint32_t*)(ws + P.off_phist);
    uint64_t* clsum = (uint64_t*)(ws + P.off_clsum);
    int32_t* seglist = (int32_t*)(ws + P.off_seglist);
    int32_t* bigbucket = (int32_t*)(ws + P.off_bigbucket);
    int32_t* halflist = (int32_t*)(ws + P.off_halflist);
    int64_t* chunk_pref = (int64_t*)(ws + P.off_bigpref);
    int64_t* gpref = chunk_pref + (P.big_max + 1);
    uint32_t* part = (uint32_t*)(ws + P.off_part);
    void* zones = ws + P.off_zones;
    uint64_t* G = (uint64_t*)(ws + P.off_G);
    uint32_t* big_hist = (uint32_t*)(ws + P.off_big_hist);
    DevModel* dmodel = (DevModel*)(ws + P.off_model);
    void* radix_ws = ws + P.off_radix;
    uint64_t* out = (uint64_t*)d_out;

    NNS_HIP(fill_u64(counters, kNumCounters, 0, st));
    int HP = 32, scaled = 0;
    if (model) NNS_HIP(upload_model(model, dmodel, allocating, st, &HP, &scaled));

    // ---- input phase + map: a slot per key ----
    InferArgs ia{};
    ia.model = dmodel;
    ia.pwl = pwl_table_of(dmodel);
    ia.in = (const uint64_t*)d_in;
    ia.n = n;
    ia.is_f64 = is_f64 ? 1 : 0;
    ia.M = prm->m * (double)n;
    ia.S = P.S;
    ia.slots_out = slots0;
    ia.bf16_scaled = scaled;
    ev.mark(7);
    const uint32_t* slots_src = slots0;
    if (given_slots) {
        NNS_HIP(launch_check_slots(given_slots, n, P.S, counters + kCntBadSlot, st));
        slots_src = given_slots;
    } else if (!model_is_finite(model)) {
        NNS_HIP(fill_u32(slots0, n, kUnmapped, st));
    } else {
        if (prm->form == NNSORT_FORM_BF16) {
            // the BF16 map kernel also counts the partition's first digits
            int shifts[4], widths[4];
            uint32_t masks[4];
            range_passes((uint32_t)P.NB, shifts, masks, widths);
            ia.tile_hist = phist;
            ia.NB = (uint32_t)P.NB;
            ia.dmask = masks[0];
        }
        NNS_HIP(launch_infer(ia, HP, prm->form, prm->bf16_terms, st));
    }
    ev.mark(1);

    // ---- hand-off: stable partition of (key, slot) by slot range ----
    const uint32_t NB = (uint32_t)P.NB;
    int which = 0;
    NNS_HIP(partition_by_range((const uint64_t*)d_in, slots_src, n, NB, is_f64, K0, S0, K1, slots0, phist, &which,
                               st, ia.tile_hist != nullptr));
    const uint64_t* Ks = which ? K1 : K0;
    const uint32_t* Ss = which ? slots0 : S0;
    NNS_HIP(launch_range_bounds(Ss, n, NB, start, st));
    NNS_HIP(launch_classify(start, cnt, P.NB, P.big_max, seglist, bigbucket, halflist, clsum, counters, st));
    NNS_HIP(launch_count_neg(Ks, start, NB, n, counters + kCntUnmappedNeg, st));
    uint64_t c[kNumCounters];
    // caller-given slots are checked (counters read back) before any range
    // is polished: an out-of-range slot leaves the range table inconsistent,
    // and a polish on it could write outside the output.  The map kernel's
    // own slots are in range by construction.
    const bool early_polish = given_slots == nullptr;
    CounterStage* cs = allocating && early_polish ? counter_stage() : nullptr;
    if (cs) {
        NNS_HIP(hipMemcpyAsync(cs->host, counters, sizeof(c), hipMemcpyDeviceToHost, st));
        NNS_HIP(hipEventRecord(cs->copied, st));
    } else {
        NNS_HIP(hipMemcpyAsync(c, counters, sizeof(c), hipMemcpyDeviceToHost, st));
        NNS_HIP(hipStreamSynchronize(st));
    }
    ev.mark(2);

    // ---- rounds + polish of each slot range in LDS, straight to out ----
    // The ranges of at most half the LDS capacity (nearly all keys) need no
    // value from the host: they are polished while the host reads the counters
    // and queues the rest.
    if (early_polish) NNS_HIP(launch_polish_small(start, P.NB, Ks, Ss, eps, out, is_f64, part, counters, st));
    ev.mark(8);
    if (cs) {
        NNS_HIP(hipEventSynchronize(cs->copied));
        std::memcpy(c, cs->host, sizeof(c));
    }
    const int64_t first_unmapped = (int64_t)c[kCntFirstUnmapped];
    if (c[kCntBadSlot] || (int64_t)c[kCntBigBuckets] > P.big_max) {
        NNS_HIP(hipStreamSynchronize(st));  // no kernel may still be writing to the caller's buffers
        return c[kCntBadSlot] ? NNSORT_EINVAL : NNSORT_EINTERNAL;
    }
    const int64_t big_count = (int64_t)c[kCntBigBuckets];
    const int64_t big_keys = (int64_t)c[kCntBigKeys];
    const int64_t nseg = (int64_t)c[kCntSegments];
    const int64_t unm = n - first_unmapped;
    const int64_t u_neg = (int64_t)c[kCntUnmappedNeg];
    // G: the keys of ranges too dense for LDS, then the keys without a slot
    const int64_t G_size = big_keys + unm;

    // chunks of kBucketCap keys over the dense ranges: at most one partial
    // chunk per range beyond the full ones; the kernels skip chunks past the
    // real count, so no host round trip is needed
    const int64_t nchunks = big_count > 0 ? big_keys / kBucketCap + big_count : 0;
    // Dense ranges up to run0 << kSegMaxRounds keys are sorted range by range
    // where the partition left them (chunks in LDS, then merge rounds through
    // the other partition buffer); larger ones send the whole residue through
    // one LSD radix sort in G, which then moves fewer bytes than the merge
    // rounds.  Runs start at two chunks once the dense keys fill the GPU with
    // such runs (the longer runs save a merge round), at one otherwise.
    const int64_t run0 = big_keys > kWideRunKeys ? (int64_t)kSortRun : (int64_t)kBigChunk;
    const int rounds = big_count > 0 ? seg_rounds((int64_t)c[kCntBigMax], run0) : 0;
    const bool seg_mode = rounds <= kSegMaxRounds;
    uint64_t* const Kw = which ? K1 : K0;   // Ks, written by the range-by-range sort
    uint64_t* const alt = which ? K0 : K1;  // the partition buffer that Ks is not in
    if (big_count > 0) {
        NNS_HIP(fill_u32(big_hist, big_count * (int64_t)kBucketSlots, 0u, st));
        NNS_HIP(launch_big_chunks(bigbucket, big_count, start, chunk_pref, gpref, st));
        NNS_HIP(launch_big_gather(bigbucket, big_count, nchunks, chunk_pref, gpref, start, Ks, Ss, big_hist,
                                  seg_mode ? nullptr : G, st));
        NNS_HIP(launch_big_counts(big_hist, big_count, eps, counters, st));
    }
    if (unm > 0) NNS_HIP(launch_copy_u64(Ks + first_unmapped, G + big_keys, unm, st));
    ev.mark(9);
    if (!early_polish) NNS_HIP(launch_polish_small(start, P.NB, Ks, Ss, eps, out, is_f64, part, counters, st));
    // the ranges above half the LDS capacity, then every range's round counts
    NNS_HIP(launch_polish_half(start, halflist, (int64_t)c[kCntHalfFull], Ks, Ss, eps, out, is_f64, part, counters,
                               st));
    NNS_HIP(launch_sum_parts(part, cnt, P.NB, eps, counters, st));
    ev.mark(3);

    // ---- dense ranges and keys without a slot: conventional sort, placed ----
    // (the keys without a slot by radix on their own in G, after the dense
    // keys' place there)
    if (G_size > 0) {
        if (seg_mode) {
            // each dense range's last sorting step writes it to its place in
            // the output
            NNS_HIP(seg_sort(chunk_pref, gpref, big_count, nchunks, rounds, run0, Kw, alt, st, bigbucket, start,
                             SegOut{out, u_neg, is_f64 ? 1 : 0}));
            if (unm > 0) NNS_HIP(radix_sort(G + big_keys, G + big_keys, unm, 0, 0, radix_ws, P.radix_bytes, st));
        } else {
            NNS_HIP(radix_sort(G, G, G_size, 0, 0, radix_ws, P.radix_bytes, st));
            NNS_HIP(launch_big_place(bigbucket, big_count, nchunks, chunk_pref, gpref, start, G, u_neg, out, is_f64,
                                     st));
        }
        // sorted keys without a slot: those with the order key's top bit clear
        // first (below every mapped key), the rest last
        const int64_t u_pos = unm - u_neg;
        if (u_neg > 0) NNS_HIP(launch_convert(seg_mode ? G + big_keys : G, out, u_neg, 0, is_f64 ? 1 : 2, st));
        if (u_pos > 0) NNS_HIP(launch_convert(G + G_size - u_pos, out + n - u_pos, u_pos, 0, is_f64 ? 1 : 2, st));
    }
    ev.mark(4);

    // ---- boundaries between neighbouring ranges ----
    // The plan, the in-place merges (skipped on the device when the plan
    // reports a fallback) and the junction check run back to back; the one
    // read of the counters that ends the call decides whether the output must
    // be sorted whole instead.
    NNS_HIP(launch_boundary_plan(out, is_f64, u_neg, start, seglist, nseg, zones, counters, st));
    NNS_HIP(launch_boundary_merge(out, is_f64, zones, nseg, counters, st));
    if (nseg > 0 || unm > 0)
        NNS_HIP(launch_junction_check(out, is_f64, u_neg, start, seglist, nseg, zones, n, u_neg + first_unmapped,
                                      unm > 0, counters, st));

    // ---- statistics (and the verdict of the boundary checks) ----
    NNS_HIP(hipMemcpyAsync(c, counters, sizeof(c), hipMemcpyDeviceToHost, st));
    NNS_HIP(hipStreamSynchronize(st));
    if (c[kCntFallback] || c[kCntJunction]) {
        const int mode = is_f64 ? 1 : 2;
        if (P.radix_bytes < radix_ws_bytes(n)) return NNSORT_EINTERNAL;
        NNS_HIP(radix_sort(out, out, n, mode, mode, radix_ws, P.radix_bytes, st));
        NNS_HIP(hipStreamSynchronize(st));
    }
    ev.mark(5);
    // while i < eps and count(w) > tau: the rounds were computed for all eps;
    // the procedure stops at the first round whose conflict array is <= tau.
    int t = 1;
    while (t < eps && (int64_t)c[kCntCollided + t - 1] + unm > prm->tau) ++t;
    S.rounds = t;
    for (int r = 0; r < t; ++r) {
        S.collided[r] = (int64_t)c[kCntCollided + r] + unm;
        S.placed[r] = (int64_t)c[kCntPlaced + r];
    }
    S.residue = S.collided[t - 1];
    S.unmapped = unm;
    S.big_buckets = big_count;
    S.big_bucket_keys = big_keys;
    S.boundary_keys = (int64_t)c[kCntBoundary];
    S.fallback = c[kCntFallback] ? 1 : c[kCntJunction] ? 2 : 0;
    S.range_resorts = (int32_t)c[kCntResorted];
    if (stats && prm->stats_level >= 2 && model && model_is_finite(model)) {
        double* Fbuf = (double*)K1;  // partition storage is free now
        InferArgs pa = ia;
        pa.in = (const uint64_t*)d_out;
        pa.F_out = Fbuf;
        pa.slots_out = nullptr;
        NNS_HIP(launch_infer(pa, HP, prm->form, prm->bf16_terms, st));
        double* dsum = (double*)counters + kCntPosErrSum;
        NNS_HIP(launch_pos_err_sum(Fbuf, n, dsum, st));
        NNS_HIP(hipMemcpyAsync(c, counters, sizeof(c), hipMemcpyDeviceToHost, st));
        NNS_HIP(hipStreamSynchronize(st));
        double sum;
        std::memcpy(&sum, &c[kCntPosErrSum], 8);
        int64_t cntm = (int64_t)c[kCntPosErrCnt];
        S.pos_err = cntm ? sum / (double)cntm / (double)n : 0.0;
    }
    ev.mark(6);
    if (ev.on) {
        NNS_HIP(hipEventSynchronize(ev.e[6]));
        S.t_infer_ms = ev.ms(7, 1);  // the map kernel alone
        // the dense-range gather (8 -> 9) runs between the two polish
        // launches; it counts with the partition, as the hand-off to the
        // residue path
        S.t_place_ms = ev.ms(1, 2) + ev.ms(8, 9);
        S.t_polish_ms = ev.ms(2, 8) + ev.ms(9, 3);
        S.t_residue_ms = ev.ms(3, 4);
        S.t_merge_ms = ev.ms(4, 5);  // the boundary check and repair
        S.t_total_ms = ev.ms(0, 5);
    }
    if (stats) *stats = S;
    return NNSORT_OK;
}

// ---- fit workspace ----
struct FitPlan {
    int64_t k, B;
    int H;
    size_t off_init, off_Fs, off_dis, off_best, off_knots, off_knotws, off_sample, off_count, off_seg, off_x, off_y, off_bx, off_gF, off_saved, off_bws, off_theta,
        off_m1, off_m2, off_loss, off_lpart, off_radix, off_model, total;
};

int64_t sample_count(int64_t n, double frac) {
    double v = std::floor(frac * (double)n + 0.5);
    return v < 1.0 ? 1 : (int64_t)v;
}

FitPlan plan_fit(int64_t n, const nnsort_fit_params* fp) {
    FitPlan p{};
    p.k = sample_count(n, fp->sample_frac);
    p.B = fp->batch;
    p.H = fp->hidden;
    int P = p.H * p.H + 4 * p.H + 1;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += align256(bytes);
        return at;
    };
    p.off_sample = take((size_t)p.k * 8);
    p.off_count = take(64);
    p.off_seg = take(64);  // the sample as one segment of the chunk sort: chunk and key prefixes
    p.off_x = take((size_t)p.k * 8);
    p.off_y = take((size_t)p.k * 4);
    p.off_bx = take((size_t)p.B * 8);
    p.off_gF = take((size_t)p.B * 4);
    p.off_saved = take((size_t)p.B * 2 * p.H * 4);
    p.off_bws = take(mlp_backward_ws_floats(p.H, p.B) * 4);
    p.off_theta = take((size_t)P * 4);
    p.off_m1 = take((size_t)P * 4);
    p.off_m2 = take((size_t)P * 4);
    p.off_loss = take(64);
    p.off_lpart = take(fit_loss_ws_floats(p.B) * 4);
    p.off_knots = take((NNSORT_MAX_HIDDEN + 1) * 8);
    p.off_knotws = take(knot_ws_bytes());
    p.off_best = take((size_t)(P + 64) * 4);
    p.off_init = take((size_t)P * 4);
    p.off_Fs = take((size_t)p.k * 8);
    p.off_model = take(model_region_bytes());
    p.off_dis = take(disorder_ws_doubles() * 2 * 8);
    p.off_radix = take(radix_ws_bytes(p.k));
    p.total = o;
    return p;
}

// The fit's sample holds fewer than 2^32 - 1 keys (the bound nnsort_fit
// documents).
bool valid_sample_count(int64_t n, const nnsort_fit_params* f) {
    return (double)f->sample_frac * (double)n < 4294967294.0;
}

bool valid_fit_params(const nnsort_fit_params* f) {
    if (!f) return false;
    if (f->hidden != 8 && f->hidden != 16 && f->hidden != 32 && f->hidden != 64) return false;
    if (!(f->sample_frac > 0.0) || f->sample_frac > 1.0e6) return false;
    if (f->batch < 1 || f->steps < 0) return false;
    if (f->loss != 0 && f->loss != 1) return false;
    if (f->init < 0 || f->init > 2) return false;
    if (!std::isfinite(f->lr)) return false;
    return true;
}

int fit_impl(const void* d_keys, int64_t n, nnsort_dtype dtype, const nnsort_fit_params* fp, nnsort_model* out,
             void* d_ws, size_t ws_bytes, hipStream_t st, float* loss_history, int history_len) {
    if (n < 1 || !d_keys || !out || !valid_fit_params(fp)) return NNSORT_EINVAL;
    if (dtype != NNSORT_F64 && dtype != NNSORT_U64) return NNSORT_EINVAL;
    if (n >= (int64_t)0xFFFFFFFF || !valid_sample_count(n, fp)) return NNSORT_EINVAL;
    FitPlan P = plan_fit(n, fp);
    if (!d_ws || ws_bytes < P.total || ((uintptr_t)d_ws & 255u)) return NNSORT_EWORKSPACE;
    const bool is_f64 = dtype == NNSORT_F64;
    char* ws = (char*)d_ws;
    uint64_t* sample = (uint64_t*)(ws + P.off_sample);
    uint64_t* count = (uint64_t*)(ws + P.off_count);
    double* x = (double*)(ws + P.off_x);
    float* y = (float*)(ws + P.off_y);
    double* bx = (double*)(ws + P.off_bx);
    float* gF = (float*)(ws + P.off_gF);
    float* saved = (float*)(ws + P.off_saved);
    float* bws = (float*)(ws + P.off_bws);
    float* theta = (float*)(ws + P.off_theta);
    float* m1 = (float*)(ws + P.off_m1);
    float* m2 = (float*)(ws + P.off_m2);
    float* dloss = (float*)(ws + P.off_loss);
    float* lpart = (float*)(ws + P.off_lpart);
    int64_t* knots = (int64_t*)(ws + P.off_knots);
    void* rws = ws + P.off_radix;
    const int H = fp->hidden;
    const int Pn = H * H + 4 * H + 1;
    float* best = (float*)(ws + P.off_best);
    float* best_loss = best + Pn;
    float* init_theta = (float*)(ws + P.off_init);
    double* Fs = (double*)(ws + P.off_Fs);
    DevModel* dmodel = (DevModel*)(ws + P.off_model);
    double* dis = (double*)(ws + P.off_dis);

    NNS_HIP(fill_u64(count, 1, 0, st));
    NNS_HIP(launch_sample(d_keys, n, is_f64, fp->seed, P.k, sample, count, st));
    uint64_t k2 = 0;
    NNS_HIP(hipMemcpyAsync(&k2, count, 8, hipMemcpyDeviceToHost, st));
    NNS_HIP(hipStreamSynchronize(st));
    nnsort_model M{};
    M.version = NNSORT_ABI_VERSION;
    M.hidden = H;
    if (k2 == 0) {  // no finite key: a constant model sends every key to slot 0
        *out = M;
        return NNSORT_OK;
    }
    // the sample sorted as one segment: 4096-key chunks sorted in LDS, then
    // merge rounds into the radix scratch and back (fewer launches than the
    // LSD radix sort's 8 passes, and no host read of a digit census)
    uint64_t* sorted = sample;
    int64_t* seg = (int64_t*)(ws + P.off_seg);  // chunk prefix {0, nchunks}, key prefix {0, k2}, then (lo, inv)
    double* lohi = (double*)(seg + 4);
    {
        const int64_t nchunks = ((int64_t)k2 + kBigChunk - 1) / kBigChunk;
        const int rounds = seg_rounds((int64_t)k2, kBigChunk);
        NNS_HIP(launch_one_segment(seg, nchunks, (int64_t)k2, st));
        uint64_t* tmp = (uint64_t*)rws;  // radix_ws_bytes(k) >= 8 k
        NNS_HIP(seg_sort(seg, seg + 2, 1, nchunks, rounds, kBigChunk, sample, tmp, st));
        if (rounds & 1) sorted = tmp;
    }
    // lo and inv_range from the sample's extremes, on the device (read back
    // with the parameters at the end)
    NNS_HIP(launch_make_xy(sorted, (int64_t)k2, is_f64, x, y, lohi, st));
    NNS_HIP(launch_init(theta, H, fp->init, fp->seed, x, (int64_t)k2, knots, ws + P.off_knotws, st));
    NNS_HIP(hipMemsetAsync(m1, 0, (size_t)Pn * 4, st));
    NNS_HIP(hipMemsetAsync(m2, 0, (size_t)Pn * 4, st));
    NNS_HIP(hipMemcpyAsync(best, theta, (size_t)Pn * 4, hipMemcpyDeviceToDevice, st));
    NNS_HIP(hipMemcpyAsync(init_theta, theta, (size_t)Pn * 4, hipMemcpyDeviceToDevice, st));
    NNS_HIP(fill_u32((uint32_t*)best_loss, 1, 0x7F800000u, st));  // +inf
    for (int t = 1; t <= fp->steps; ++t) {
        // the batch, its forward, loss and dL/dF, keeping the parameters if
        // this batch's loss is the lowest so far; then the gradients applied
        // by one Adam step.  Widths 32 and 64: one fused kernel on the FP32
        // matrix cores plus the update; 8 and 16: forward, then backward.
        if (fit_step_mfma(H)) {
            NNS_HIP(launch_fit_step_mfma(H, theta, x, y, (int64_t)k2, P.B, fp->seed, t, fp->loss, fp->huber_delta,
                                         fp->lr, 0.9f, 0.999f, 1e-8f, bws, lpart, m1, m2, best, best_loss, dloss,
                                         st));
        } else {
            NNS_HIP(launch_fit_step_forward(H, theta, x, y, (int64_t)k2, fp->seed, t, P.B, bx, saved, fp->loss,
                                            fp->huber_delta, gF, dloss, lpart, best, Pn, best_loss, st));
            NNS_HIP(launch_mlp_backward_adam(H, theta, bx, P.B, saved, gF, bws, m1, m2, t, fp->lr, 0.9f, 0.999f,
                                             1e-8f, st));
        }
        if (loss_history && t - 1 < history_len)
            NNS_HIP(hipMemcpyAsync(loss_history + (t - 1), dloss, 4, hipMemcpyDeviceToHost, st));
    }
    // Returned: the parameters with the lowest batch loss seen, unless they
    // move F backwards along the sorted sample more than the initial ones do
    // (a model that is less monotone only adds work to the polish).  F is the
    // FP64 model's, through its piecewise-linear form, on the sample's
    // translated keys (already in [0, 1], so lo = 0 and inv_range = 1).
    std::vector<float> cand((size_t)2 * Pn);
    NNS_HIP(hipMemcpyAsync(cand.data(), best, (size_t)Pn * 4, hipMemcpyDeviceToHost, st));
    NNS_HIP(hipMemcpyAsync(cand.data() + Pn, init_theta, (size_t)Pn * 4, hipMemcpyDeviceToHost, st));
    double lo_inv[2];
    NNS_HIP(hipMemcpyAsync(lo_inv, lohi, sizeof(lo_inv), hipMemcpyDeviceToHost, st));
    NNS_HIP(hipStreamSynchronize(st));
    const double lo = lo_inv[0], inv = lo_inv[1];
    auto model_of = [&](const float* th, double lo_, double inv_) {
        nnsort_model m = M;
        m.lo = lo_;
        m.inv_range = inv_;
        for (int j = 0; j < H; ++j) {
            m.w1[j] = th[j];
            m.b1[j] = th[H + j];
            m.b2[j] = th[2 * H + H * H + j];
            m.w3[j] = th[3 * H + H * H + j];
        }
        for (int e = 0; e < H * H; ++e) m.w2[e] = th[2 * H + e];
        m.b3 = th[4 * H + H * H];
        return m;
    };
    int pick = 0;  // the best-loss parameters
    if (fp->steps > 0 && k2 > 1) {
        const size_t dw = disorder_ws_doubles();
        DevModel hm[2];  // host sources stay alive until the stream is synchronised
        for (int c = 0; c < 2; ++c) {
            const nnsort_model mc = model_of(cand.data() + (size_t)c * Pn, 0.0, 1.0);
            to_dev_model(&mc, &hm[c]);
            NNS_HIP(hipMemcpyAsync(dmodel, &hm[c], sizeof(DevModel), hipMemcpyHostToDevice, st));
            InferArgs ia{};
            ia.model = dmodel;
            ia.pwl = pwl_table_of(dmodel);
            ia.in = (const uint64_t*)x;
            ia.n = (int64_t)k2;
            ia.is_f64 = 1;
            ia.M = 1.0;
            ia.S = 2;
            ia.F_out = Fs;
            NNS_HIP(launch_infer(ia, hm[c].H, NNSORT_FORM_PWL, 3, st));
            NNS_HIP(launch_disorder(Fs, (int64_t)k2, dis + c * dw, st));
        }
        double d[2];
        NNS_HIP(hipMemcpyAsync(&d[0], dis + dw - 1, 8, hipMemcpyDeviceToHost, st));
        NNS_HIP(hipMemcpyAsync(&d[1], dis + 2 * dw - 1, 8, hipMemcpyDeviceToHost, st));
        NNS_HIP(hipStreamSynchronize(st));
        if (d[0] > d[1]) pick = 1;
    }
    *out = model_of(cand.data() + (size_t)pick * Pn, lo, inv);
    return NNSORT_OK;
}

}  // namespace

// ---- the allocation-free sort: a static device scratch array ----
// nnsort_sort_with_model_noalloc sorts in this array instead of a caller
// workspace.  Each GPU the library runs on holds its own copy for the life of
// the process.  Host code never passes the array's name to a kernel (on the
// host it is only a stand-in); it uses the device address that
// hipGetSymbolAddress returns, taken once per device with that device current.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_of_current_device(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return NNSORT_EINTERNAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
        if (!p || ((uintptr_t)p & 255u)) return NNSORT_EINTERNAL;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return NNSORT_OK;
}

}  // namespace

extern "C" {

int nnsort_sort_with_model_noalloc(const nnsort_model* model, const void* d_in, void* d_out, int64_t n,
                                   nnsort_dtype dtype, const nnsort_sort_params* params, nnsort_stats* stats,
                                   void* stream) {
    if (!model || !params) return NNSORT_EINVAL;
    size_t need = 0;
    int rc = nnsort_workspace_size(n, dtype, params, nullptr, &need);
    if (rc) return rc;
    if (need > kScratchBytes) return NNSORT_ETOOBIG;
    if (n == 0) return sort_impl(model, nullptr, d_in, d_out, n, dtype, params, nullptr, 0, stats,
                                 (hipStream_t)stream, false);
    void* ws = nullptr;
    rc = scratch_of_current_device(&ws);
    if (rc) return rc;
    return sort_impl(model, nullptr, d_in, d_out, n, dtype, params, ws, kScratchBytes, stats, (hipStream_t)stream,
                     false);
}

void nnsort_default_params(nnsort_sort_params* sp, nnsort_fit_params* fp) {
    if (sp) {
        std::memset(sp, 0, sizeof(*sp));
        sp->m = 1.25;
        sp->eps = 3;
        sp->form = NNSORT_FORM_FP32;
        sp->tau = 1024;
        sp->bf16_terms = 3;
        sp->stats_level = 1;
    }
    if (fp) {
        std::memset(fp, 0, sizeof(*fp));
        fp->hidden = 32;
        fp->batch = 65536;
        fp->sample_frac = 0.01;
        fp->steps = 200;
        fp->lr = 1e-7f;
        fp->seed = 0;
        fp->loss = 0;
        fp->huber_delta = 1.0f;
        fp->init = 1;
    }
}

int nnsort_workspace_size(int64_t n, nnsort_dtype dtype, const nnsort_sort_params* sp,
                          const nnsort_fit_params* fp, size_t* bytes) {
    if (!bytes || n < 0 || !sp) return NNSORT_EINVAL;
    if (dtype != NNSORT_F64 && dtype != NNSORT_U64) return NNSORT_EINVAL;
    if (!valid_sort_params(sp, n)) return NNSORT_EINVAL;
    size_t need = align256(radix_ws_bytes(n));
    if (n > sp->tau) {
        SortPlan P = plan_sort(n, sp->m);
        need = P.total > need ? P.total : need;
    }
    need = need > model_region_bytes() ? need : model_region_bytes();
    if (fp) {
        if (!valid_fit_params(fp) || !valid_sample_count(n > 0 ? n : 1, fp)) return NNSORT_EINVAL;
        FitPlan F = plan_fit(n > 0 ? n : 1, fp);
        need = F.total > need ? F.total : need;
    }
    *bytes = need;
    return NNSORT_OK;
}

int nnsort_fit(const void* d_keys, int64_t n, nnsort_dtype dtype, const nnsort_fit_params* params,
               nnsort_model* out, void* d_ws, size_t ws_bytes, void* stream) {
    return fit_impl(d_keys, n, dtype, params, out, d_ws, ws_bytes, (hipStream_t)stream, nullptr, 0);
}

int nnsort_fit_history(const void* d_keys, int64_t n, nnsort_dtype dtype, const nnsort_fit_params* params,
                       nnsort_model* out, void* d_ws, size_t ws_bytes, float* loss_history, int history_len,
                       void* stream) {
    return fit_impl(d_keys, n, dtype, params, out, d_ws, ws_bytes, (hipStream_t)stream, loss_history,
                    history_len);
}

int nnsort_sort_with_model(const nnsort_model* model, const void* d_in, void* d_out, int64_t n,
                           nnsort_dtype dtype, const nnsort_sort_params* params, void* d_ws, size_t ws_bytes,
                           nnsort_stats* stats, void* stream) {
    if (!model) return NNSORT_EINVAL;
    return sort_impl(model, nullptr, d_in, d_out, n, dtype, params, d_ws, ws_bytes, stats, (hipStream_t)stream);
}

int nnsort_sort_with_slots(const uint32_t* d_slots, const void* d_in, void* d_out, int64_t n, nnsort_dtype dtype,
                           const nnsort_sort_params* params, void* d_ws, size_t ws_bytes, nnsort_stats* stats,
                           void* stream) {
    if (n > 0 && !d_slots) return NNSORT_EINVAL;
    return sort_impl(nullptr, d_slots, d_in, d_out, n, dtype, params, d_ws, ws_bytes, stats, (hipStream_t)stream);
}

int nnsort_sort(const void* d_in, void* d_out, int64_t n, nnsort_dtype dtype, const nnsort_fit_params* fp,
                const nnsort_sort_params* sp, void* d_ws, size_t ws_bytes, nnsort_model* model_out,
                nnsort_stats* stats, void* stream) {
    if (n < 0 || !fp || !sp) return NNSORT_EINVAL;
    if (n == 0) {
        if (stats) std::memset(stats, 0, sizeof(*stats));
        return NNSORT_OK;
    }
    hipStream_t st = (hipStream_t)stream;
    Events ev(stats != nullptr, st, 1);
    ev.mark(0);
    nnsort_model m;
    int rc = fit_impl(d_in, n, dtype, fp, &m, d_ws, ws_bytes, st, nullptr, 0);
    if (rc) return rc;
    ev.mark(1);
    rc = sort_impl(&m, nullptr, d_in, d_out, n, dtype, sp, d_ws, ws_bytes, stats, st);
    if (rc) return rc;
    ev.mark(2);
    if (model_out) *model_out = m;
    if (stats && ev.on) {
        NNS_HIP(hipEventSynchronize(ev.e[2]));
        stats->t_fit_ms = ev.ms(0, 1);
        stats->t_total_ms = ev.ms(0, 2);
    }
    return NNSORT_OK;
}

size_t nnsort_model_device_bytes(void) { return model_region_bytes(); }

int nnsort_predict(const nnsort_model* model, const void* d_in, int64_t n, nnsort_dtype dtype,
                   const nnsort_sort_params* params, uint32_t* d_slots, double* d_F, void* d_ws, size_t ws_bytes,
                   void* stream) {
    int rc = check_model(model);
    if (rc) return rc;
    if (n < 0 || (n > 0 && !d_in) || !valid_sort_params(params, n)) return NNSORT_EINVAL;
    if (dtype != NNSORT_F64 && dtype != NNSORT_U64) return NNSORT_EINVAL;
    if (!d_ws || ws_bytes < model_region_bytes() || ((uintptr_t)d_ws & 255u)) return NNSORT_EWORKSPACE;
    if (n == 0) return NNSORT_OK;
    hipStream_t st = (hipStream_t)stream;
    DevModel hm;
    to_dev_model(model, &hm);
    NNS_HIP(hipMemcpyAsync(d_ws, &hm, sizeof(hm), hipMemcpyHostToDevice, st));
    InferArgs ia{};
    ia.model = (const DevModel*)d_ws;
    ia.pwl = pwl_table_of(d_ws);
    ia.in = (const uint64_t*)d_in;
    ia.n = n;
    ia.is_f64 = dtype == NNSORT_F64;
    ia.M = params->m * (double)n;
    ia.S = num_slots(n, params->m);
    ia.slots_out = d_slots;
    ia.F_out = d_F;
    ia.bf16_scaled = hm.bf16_scaled;
    if (model_is_finite(model)) {
        NNS_HIP(launch_infer(ia, hm.H, params->form, params->bf16_terms, st));
    } else {
        if (d_slots) NNS_HIP(fill_u32(d_slots, n, kUnmapped, st));
        if (d_F) NNS_HIP(fill_u64((uint64_t*)d_F, n, 0x7FF8000000000000ull, st));
    }
    NNS_HIP(hipStreamSynchronize(st));
    return NNSORT_OK;
}

size_t nnsort_radix_workspace_size(int64_t n) { return radix_ws_bytes(n); }

int nnsort_radix_sort(const void* d_in, void* d_out, int64_t n, nnsort_dtype dtype, void* d_ws, size_t ws_bytes,
                      void* stream) {
    if (n < 0 || (n > 0 && (!d_in || !d_out))) return NNSORT_EINVAL;
    if (dtype != NNSORT_F64 && dtype != NNSORT_U64) return NNSORT_EINVAL;
    if (n >= (int64_t)0xFFFFFFFF) return NNSORT_EINVAL;
    if (n == 0) return NNSORT_OK;
    if (!d_ws || ws_bytes < radix_ws_bytes(n)) return NNSORT_EWORKSPACE;
    int mode = dtype == NNSORT_F64 ? 1 : 2;
    NNS_HIP(radix_sort((const uint64_t*)d_in, (uint64_t*)d_out, n, mode, mode, d_ws, ws_bytes, (hipStream_t)stream));
    return NNSORT_OK;
}

size_t nnsort_mlp_saved_floats(int hidden, int64_t batch) { return (size_t)batch * 2 * hidden; }
size_t nnsort_mlp_backward_ws_floats(int hidden, int64_t batch) { return mlp_backward_ws_floats(hidden, batch); }

static bool fit_width(int H) { return H == 8 || H == 16 || H == 32 || H == 64; }

int nnsort_mlp_forward(int hidden, const float* d_theta, const double* d_x, int64_t batch, float* d_F,
                       float* d_saved, void* stream) {
    if (!fit_width(hidden) || batch < 0 || (batch > 0 && (!d_theta || !d_x || !d_F))) return NNSORT_EINVAL;
    if (batch == 0) return NNSORT_OK;
    NNS_HIP(launch_mlp_forward(hidden, d_theta, d_x, batch, d_F, d_saved, (hipStream_t)stream));
    return NNSORT_OK;
}

int nnsort_mlp_backward(int hidden, const float* d_theta, const double* d_x, int64_t batch, const float* d_saved,
                        const float* d_gF, float* d_gtheta, float* d_ws, void* stream) {
    if (!fit_width(hidden) || batch < 1 || !d_theta || !d_x || !d_saved || !d_gF || !d_gtheta || !d_ws)
        return NNSORT_EINVAL;
    NNS_HIP(launch_mlp_backward(hidden, d_theta, d_x, batch, d_saved, d_gF, d_gtheta, d_ws, (hipStream_t)stream));
    return NNSORT_OK;
}

size_t nnsort_loss_ws_floats(void) { return loss_ws_floats(); }

size_t nnsort_fit_gradient_ws_floats(int hidden, int64_t batch) {
    const int64_t G = fit_step_groups(batch > 0 ? batch : 1);
    return (size_t)G * (hidden * hidden + 4 * hidden + 1) + 256;
}

int nnsort_fit_gradient(int hidden, const float* d_theta, const double* d_x, const float* d_y, int64_t k,
                        int64_t batch, uint64_t seed, int64_t step, int loss, float delta, float* d_gtheta,
                        float* d_loss, float* d_ws, size_t ws_floats, void* stream) {
    if (!fit_step_mfma(hidden) || batch < 1 || k < 1 || step < 1 || (loss != 0 && loss != 1)) return NNSORT_EINVAL;
    if (!d_theta || !d_x || !d_y || !d_gtheta || !d_loss || !d_ws) return NNSORT_EINVAL;
    if (ws_floats < nnsort_fit_gradient_ws_floats(hidden, batch)) return NNSORT_EWORKSPACE;
    const int64_t G = fit_step_groups(batch);
    float* part = d_ws;
    float* lpart = d_ws + (size_t)G * (hidden * hidden + 4 * hidden + 1);
    NNS_HIP(launch_fit_gradient(hidden, d_theta, d_x, d_y, k, batch, seed, step, loss, delta, part, lpart, d_gtheta,
                                d_loss, (hipStream_t)stream));
    return NNSORT_OK;
}

int nnsort_loss_grad(const float* d_F, const float* d_y, int64_t batch, int loss, float delta, float* d_gF,
                        float* d_loss, float* d_ws, void* stream) {
    if (batch < 1 || !d_F || !d_y || !d_gF || !d_loss || !d_ws || (loss != 0 && loss != 1)) return NNSORT_EINVAL;
    NNS_HIP(launch_loss_grad(d_F, d_y, batch, loss, delta, d_gF, d_loss, d_ws, (hipStream_t)stream));
    return NNSORT_OK;
}

int nnsort_adam_step(float* d_theta, const float* d_g, float* d_m1, float* d_m2, int64_t count, int64_t t,
                     float lr, float beta1, float beta2, float eps, void* stream) {
    if (count < 0 || t < 1 || (count > 0 && (!d_theta || !d_g || !d_m1 || !d_m2))) return NNSORT_EINVAL;
    if (count == 0) return NNSORT_OK;
    NNS_HIP(launch_adam(d_theta, d_g, d_m1, d_m2, count, t, lr, beta1, beta2, eps, (hipStream_t)stream));
    return NNSORT_OK;
}

int nnsort_model_save(const nnsort_model* m, const char* path) {
    int rc = check_model(m);
    if (rc) return rc;
    if (!path) return NNSORT_EINVAL;
    FILE* f = std::fopen(path, "wb");
    if (!f) return NNSORT_EIO;
    const char magic[4] = {'N', 'N', 'S', 'M'};
    int32_t hdr[2] = {m->version, m->hidden};
    double aff[2] = {m->lo, m->inv_range};
    int H = m->hidden;
    bool ok = std::fwrite(magic, 1, 4, f) == 4 && std::fwrite(hdr, 4, 2, f) == 2 && std::fwrite(aff, 8, 2, f) == 2 &&
              std::fwrite(m->w1, 4, H, f) == (size_t)H && std::fwrite(m->b1, 4, H, f) == (size_t)H &&
              std::fwrite(m->w2, 4, (size_t)H * H, f) == (size_t)H * H && std::fwrite(m->b2, 4, H, f) == (size_t)H &&
              std::fwrite(m->w3, 4, H, f) == (size_t)H && std::fwrite(&m->b3, 4, 1, f) == 1;
    ok = (std::fclose(f) == 0) && ok;
    return ok ? NNSORT_OK : NNSORT_EIO;
}

int nnsort_model_load(nnsort_model* m, const char* path) {
    if (!m || !path) return NNSORT_EINVAL;
    FILE* f = std::fopen(path, "rb");
    if (!f) return NNSORT_EIO;
    nnsort_model t{};
    char magic[4];
    int32_t hdr[2];
    double aff[2];
    int rc = NNSORT_OK;
    if (std::fread(magic, 1, 4, f) != 4 || std::memcmp(magic, "NNSM", 4) != 0 || std::fread(hdr, 4, 2, f) != 2 ||
        hdr[0] != NNSORT_ABI_VERSION || hdr[1] < 1 || hdr[1] > NNSORT_MAX_HIDDEN || std::fread(aff, 8, 2, f) != 2) {
        rc = NNSORT_EMODEL;
    } else {
        int H = hdr[1];
        t.version = hdr[0];
        t.hidden = H;
        t.lo = aff[0];
        t.inv_range = aff[1];
        bool ok = std::fread(t.w1, 4, H, f) == (size_t)H && std::fread(t.b1, 4, H, f) == (size_t)H &&
                  std::fread(t.w2, 4, (size_t)H * H, f) == (size_t)H * H && std::fread(t.b2, 4, H, f) == (size_t)H &&
                  std::fread(t.w3, 4, H, f) == (size_t)H && std::fread(&t.b3, 4, 1, f) == 1;
        if (!ok) rc = NNSORT_EMODEL;
    }
    std::fclose(f);
    if (rc == NNSORT_OK) *m = t;
    return rc;
}

const char* nnsort_strerror(int status) {
    switch (status) {
    case NNSORT_OK: return "ok";
    case NNSORT_EINVAL: return "invalid argument";
    case NNSORT_EWORKSPACE: return "workspace too small or not 256-byte aligned";
    case NNSORT_EHIP: return g_last_error[0] ? g_last_error : "HIP runtime error";
    case NNSORT_EMODEL: return "malformed model";
    case NNSORT_EIO: return "model file I/O error";
    case NNSORT_EINTERNAL: return "internal consistency check failed";
    case NNSORT_ETOOBIG: return "input needs more than the 64 MiB static scratch of nnsort_sort_with_model_noalloc";
    default: return "unknown status";
    }
}

}  // extern "C"
