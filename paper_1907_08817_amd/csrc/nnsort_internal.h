// Internal declarations shared by the HIP translation units of libnnsort.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/nnsort.h"

namespace nns {

constexpr uint32_t kUnmapped = 0xFFFFFFFFu;

// Slot ranges: the sorting phase's slot array o_i is cut into ranges of
// kBucketSlots consecutive slots; the keys predicted into one range are made
// contiguous by a partition on the range id, and a range of at most
// kBucketCap keys is handled by one workgroup that runs every round and the
// polish in LDS (a "dense" range, with more keys, takes the residue path).
constexpr int kLogBucketSlots = 11;
constexpr uint32_t kBucketSlots = 1u << kLogBucketSlots;
constexpr uint32_t kBucketCap = 4096;
// dense ranges are gathered, sorted and placed in chunks of this many keys
constexpr int kBigChunk = 4096;
// the chunk sort leaves sorted runs of this many keys (two chunks), which the
// merge rounds then double
constexpr int kSortRun = 2 * kBigChunk;
constexpr int kBucketThreads = 256;

// Partition of keys by slot range: tiles of kPartTile keys in input order,
// 256 digits per pass.
constexpr int kPartTile = 2048;

// Range id of a slot; keys without a slot sort after every range.
__device__ __forceinline__ uint32_t range_of(uint32_t slot, uint32_t NB) {
    return slot == kUnmapped ? NB : (slot >> kLogBucketSlots);
}

// Counters kept in the workspace (uint64 each).
enum Counter : int {
    kCntResorted = 0,     // ranges sorted whole in LDS (a large slot group, or tile merges that did not settle)
    kCntUnmapped = 1,     // keys with no slot
    kCntCollided = 2,     // [2, 2 + 8): |c_r| for r = 1..8 (all ranges)
    kCntPlaced = 10,      // [10, 18): keys stored in o_r
    kCntBigKeys = 18,     // keys of dense ranges
    kCntBigBuckets = 19,
    kCntBoundary = 21,    // keys inside boundary fix-up zones
    kCntFallback = 22,    // nonzero: the boundary repair needs the full-sort fallback
    kCntBadSlot = 23,     // caller-given slot out of range
    kCntSegments = 24,    // non-empty slot ranges
    kCntPosErrSum = 25,   // double bits: sum |F n - p|
    kCntPosErrCnt = 26,
    kCntUnmappedNeg = 27, // keys with no slot whose order key has the top bit clear
    kCntHalfFull = 28,    // ranges of more than half the LDS capacity (and at most all of it)
    kCntJunction = 29,    // nonzero: blocks out of order after the boundary fix-up
    kCntBigMax = 30,      // keys in the largest dense range
    kCntFirstUnmapped = 31,  // position of the first key without a slot after the partition
    kNumCounters = 32
};

// IEEE 754-2019 totalOrder as an unsigned 64-bit key (identity for uint64).
__device__ __forceinline__ uint64_t order_key(uint64_t bits, bool is_f64) {
    if (!is_f64) return bits;
    return (bits >> 63) ? ~bits : (bits | 0x8000000000000000ull);
}
__device__ __forceinline__ uint64_t order_key_inverse(uint64_t key, bool is_f64) {
    if (!is_f64) return key;
    return (key >> 63) ? (key & 0x7FFFFFFFFFFFFFFFull) : ~key;
}

// Device copy of the model in the FP32 layout the kernels read, padded to a
// multiple of 32 hidden units with zero weights.
struct DevModel {
    int H;       // padded width (32 or 64)
    int H_true;  // width of the caller's model
    double lo;
    double inv_range;
    float w1[64];
    float b1[64];
    alignas(16) float w2[64 * 64];  // [i * H + j]; rows are read as 16-byte vectors
    float b2[64];
    float w3[64];
    float b3;
    // Operands of the BF16 form, prepared on the host (bf16_operands()):
    // with power-of-two scales 2^k1[j] per hidden-1 unit and 2^k2[i] per
    // hidden-2 unit chosen so that every pre-activation of the scaled network
    // lies in (-inf, 1] for inputs in [0, 1], relu becomes a clamp to [0, 1],
    // which the FMA producing layer 1 and the conversion feeding layer 3
    // apply for free.  Scaling by powers of two commutes with rounding, so the
    // scaled network computes the same F bit for bit (barring subnormals):
    //   w1s = w1 2^-k1, b1s = b1 2^-k1, w2s[i][j] = bf16(W2[i][j]) 2^(k1[j] - k2[i]),
    //   b2s = b2 2^-k2, w3s = w3 2^k2 (FP64).
    // bf16_scaled = 0 when some scaled operand would not be exact (subnormal
    // or out of range): the fields then hold the unscaled values and the
    // kernel applies relu explicitly.
    int bf16_scaled;
    float w1s[64];
    float b1s[64];
    float b2s[64];
    alignas(8) double w3s[64];
    alignas(16) float w2s[64 * 64];  // bf16 values held as FP32
};
static_assert(offsetof(DevModel, w2) % 16 == 0, "W2 rows are read as 16-byte vectors");
static_assert(offsetof(DevModel, w2s) % 16 == 0, "W2 rows are read as 16-byte vectors");

// Workspace carve-up for a sort of n keys.
struct SortPlan {
    int64_t n;
    int64_t S;         // slots
    int64_t NB;        // slot ranges
    int64_t big_max;   // most dense ranges possible (n / (kBucketCap + 1) + 1)
    size_t off_counters, off_cnt, off_start, off_slots0, off_S0, off_K0, off_K1, off_phist, off_clsum, off_seglist,
        off_bigbucket, off_halflist, off_bigpref, off_part, off_zones, off_G, off_radix, off_big_hist, off_model, total;
    size_t radix_bytes;
};

SortPlan plan_sort(int64_t n, double m);
size_t radix_ws_bytes(int64_t n);

// ---- launchers (each returns hipError_t of its launch) ----
// The model compiled into its piecewise-linear form (a network with one
// input and ReLU units is affine between breakpoints): each layer-1 unit
// switches at one input, which cuts [0, 1] into at most H + 1 intervals; on
// each interval every layer-2 unit is affine, z2 = A x + B, and changes sign
// at most once inside it.  F is affine on each resulting piece:
// F(x) = Fq[q] + alpha[q] (x - xq[q]) for the last q with xq[q] <= x.
// Built on the device for every call that uses the form; the map kernel
// indexes the pieces by kPwlGrid cells of [0, 1] to bracket its search.
constexpr int kPwlMaxIntervals = NNSORT_MAX_HIDDEN + 1;
constexpr int kPwlMaxPieces = kPwlMaxIntervals * (NNSORT_MAX_HIDDEN + 1);
constexpr int kPwlGrid = 1024;
struct PwlTable {
    int32_t nint;     // layer-1 intervals
    int32_t npieces;  // pieces in all
    double edge[kPwlMaxIntervals + 1];
    int32_t nroots[kPwlMaxIntervals];  // layer-2 sign changes inside each interval
    double A[kPwlMaxIntervals][NNSORT_MAX_HIDDEN];
    double B[kPwlMaxIntervals][NNSORT_MAX_HIDDEN];
    double sub[kPwlMaxIntervals][NNSORT_MAX_HIDDEN + 2];  // sorted piece edges per interval
    double xq[kPwlMaxPieces];
    double alpha[kPwlMaxPieces];
    double Fq[kPwlMaxPieces];
};
static_assert(kPwlMaxPieces < 65536, "piece index is 16-bit");

struct InferArgs {
    const DevModel* model;
    PwlTable* pwl;  // the piecewise-linear form's table (that form only)
    const uint64_t* in;
    int64_t n;
    int is_f64;
    double M;
    int64_t S;
    uint32_t* slots_out;  // optional per-key slot
    double* F_out;        // optional per-key F
    int bf16_scaled;      // the host copy's DevModel::bf16_scaled (BF16 form)
    // BF16 form, optional: the first partition pass's digit histogram of
    // every kPartTile-key tile, hist[tile][256], counted as the slots are
    // written (digit = range_of(slot, NB) & dmask)
    uint32_t* tile_hist;
    uint32_t NB;
    uint32_t dmask;
};

// Where the range-by-range sort of dense ranges leaves each range's final
// sorted keys: out[base + range_start[range] + i] as the caller's bit
// patterns (is_f64: binary64, else uint64).  A null out keeps them in the
// sort's own buffers.
struct SegOut {
    uint64_t* out;
    int64_t base;
    int is_f64;
};

// H is the padded model width (32 or 64).
hipError_t launch_infer(const InferArgs& a, int H, int form, int bf16_terms, hipStream_t st);

// Radix sort of 64-bit keys: in_mode/out_mode 0 = order keys, 1 = f64 bits,
// 2 = u64 bits (converted on load / store).
hipError_t radix_sort(const uint64_t* d_in, uint64_t* d_out, int64_t n, int in_mode, int out_mode,
                      void* d_ws, size_t ws_bytes, hipStream_t st);

// Copy with conversion between order keys and bits.
hipError_t launch_convert(const uint64_t* d_in, uint64_t* d_out, int64_t n, int in_mode, int out_mode,
                          hipStream_t st);

// Fit.
hipError_t launch_mlp_forward(int H, const float* d_theta, const double* d_x, int64_t B, float* d_F,
                              float* d_saved, hipStream_t st);
hipError_t launch_mlp_backward(int H, const float* d_theta, const double* d_x, int64_t B,
                               const float* d_saved, const float* d_gF, float* d_gtheta, float* d_ws,
                               hipStream_t st);
hipError_t launch_adam(float* d_theta, const float* d_g, float* d_m1, float* d_m2, int64_t count,
                       int64_t t, float lr, float b1, float b2, float eps, hipStream_t st);

}  // namespace nns
