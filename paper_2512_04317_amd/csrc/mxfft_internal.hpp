// mxfft_internal.hpp -- host-side interface between the plan code and the
// kernel launchers (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "mxfft.h"

struct mxfft_plan_s;

namespace mxk {

constexpr int kMaxLog2N = 12;       // n <= 4096
constexpr int kStatsBins = 288;     // floor(log2 |x|) + 149, |x| from FP32 parts: 0..276
constexpr int kBinOffset = 149;

// Prescale statistics of one chunk of one slice (device workspace, written
// in full by every call; summed per slice by the finalize kernel).
struct alignas(16) StatPart {
    uint32_t hist[kStatsBins];      // nonzero finite |x| per binade floor(log2 |x|)
    unsigned long long max_m2;      // bits of max |x|^2 (FP64, non-negative)
    uint32_t count;                 // unused (the count is the histogram's sum)
    uint32_t max_comp;              // bits of max(|re|, |im|) (FP32)
    uint32_t nonfinite;             // any Inf/NaN part
    int32_t emin, emax;             // range of the MX block exponents the unscaled row pass used
    uint32_t pad;
};

// Window of block exponents inside which an unscaled row pass times 2^k is
// bit-identical to the row pass of the input scaled by 2^k (checked for the
// exponents both before and after adding k): no E8M0 clamp at +-127, and
// every FP32 value of the pass stays zero or normal and finite (element
// grids are at least 2^(E - 32) for every MX element format, values below
// 2^(E + 17); the 6-bit formats' scale operand 2^(E + 12) at most stays in
// range there too).
constexpr int kEquivLo = -90, kEquivHi = 90;

// Device workspace of one call: everything the kernels of a transform write
// besides its output (and read back later in the same call).  A plan owns one
// sized for its largest batch; the no-allocation forward carves one out of a
// static device array instead.
struct Workspace {
    StatPart* parts = nullptr;    // prescale statistics per chunk or row tile
    int32_t* kp = nullptr;        // prescale exponent per slice
    int32_t* status = nullptr;    // device status word per slice
    uint32_t* codes = nullptr;    // register-resident intermediate: MX codes or packed 16-bit values
    uint8_t* exps = nullptr;      // MX intermediate block exponents (E8M0)
    int32_t* kadd = nullptr;      // fused statistics: exponent offset per slice
    int32_t* fix_list = nullptr;  // fused statistics: slices whose row pass is redone
    int32_t* fix_count = nullptr; // length of fix_list (cleared by the row pass)
    // element offset of each slice in the caller's input pool, or nullptr for
    // [batch][n][n] (uneven batches: slices anywhere in the pool); and in the
    // output pool, or nullptr for the same offsets as the input (coalesced
    // serving requests: slices of unrelated buffers)
    const unsigned long long* slice_off = nullptr;
    const unsigned long long* slice_off_out = nullptr;
};

// Chunks per slice for a batch: enough work-groups to fill the chip, at
// least 8192 elements each.
int stats_chunks(int n, int batch);
// StatPart entries a plan must hold for batches up to max_batch.
size_t stats_parts(int n, int max_batch);

// Alg. 1 parameters as the device needs them.
struct PrescaleArgs {
    double target;      // T > 0
    double tau;         // percent
    double tau_min;     // > 0
    int32_t k_min, k_max;
};

// One launch of the line kernel: a 1D pass over lines (rows or columns) of
// every slice in the batch.
struct LineArgs {
    const float2* src;
    float2* dst;
    const int32_t* kp;       // per-slice prescale exponent, or nullptr (= 0)
    int32_t* k_out;          // per-slice copy of kp written by the row pass, or nullptr
    int32_t kin_mul;         // input is scaled by 2^(kin_mul * kp)
    int32_t kout_mul;        // output is scaled by 2^(kout_mul * kp + kout_add)
    int32_t kout_add;
    const float2* tw;        // stage s, index j at [2^(s-1) - 1 + j]: element values (MX) or FP32 twiddles
    const int32_t* tw_exp;   // MX: twiddle block exponents, stage s at tw_exp_off[s]
    int32_t tw_exp_off[kMaxLog2N + 2];
    int32_t n, logn;
    int32_t cb, logcb;       // complex values per MX block (B/2)
    int32_t lines;           // lines per work-group (power of two)
    int32_t axis;            // 0 rows (contiguous), 1 columns
    int32_t inverse;
    int32_t encode;          // MX-encode the pass input
    float2* cap_mant;        // column pass: its encoded input's element values, or nullptr
    int32_t* cap_exp;        // column pass: its input block exponents [slice][column][row block]
    const unsigned long long* slice_off;      // slice offsets in src, or nullptr (contiguous)
    const unsigned long long* slice_off_out;  // slice offsets in dst, or nullptr (contiguous)
    int32_t* cap_trace;      // row pass, debug capture: (E_v, k_r, E_out) per stage and block of line 0,
                             // [slice][log2 n][n / B][3], or nullptr
};

// MX formats, the 16-bit positive controls (per-operation rounding) and plain FP32
enum Mode { MODE_E4M3 = 0, MODE_E5M2 = 1, MODE_FP16 = 2, MODE_BF16 = 3, MODE_FP32 = 4, MODE_E2M3 = 5, MODE_E3M2 = 6 };
// MX element formats: MXFP8 (E4M3, E5M2) and MXFP6 (E2M3, E3M2)
inline bool is_mx_mode(int m) { return m == MODE_E4M3 || m == MODE_E5M2 || m == MODE_E2M3 || m == MODE_E3M2; }

// Register-resident passes for n = 512 (see mxfft_fast.hip).
struct FastPassArgs {
    const float2* src;
    float2* dst;
    uint32_t* codes;         // intermediate: MX codes (2 bytes per complex value) or packed FP16/BF16 (4)
    uint8_t* exps;           // MX intermediate block exponents (E8M0)
    const int32_t* kp;
    int32_t* k_out;
    int32_t kin_mul, kout_mul, kout_add;
    const float2* tw;        // stage s (h = 2^(s-1)) index j at [h + j]
    const int32_t* tw_exp;
    int32_t tw_off[16];
    StatPart* parts;         // row pass with statistics: one part per 16-row tile, [slice][tile]
    const int32_t* kadd;     // column pass: per-slice offset added to the stored block exponents, or nullptr
    const int32_t* fix_list; // list-driven row pass: slices to redo
    int32_t* fix_count;      // number of list entries (zeroed by the row pass with statistics)
    const uint32_t* tw16;    // FP16 form: twiddles as packed halves at [h + j]
    float* rss;              // COL_RSS: [reconstruction][n][n] root-sum-of-squares image
    int32_t coils;           // COL_RSS: coil slices per reconstruction
    const unsigned long long* slice_off;      // slice offsets in src, or nullptr (contiguous)
    const unsigned long long* slice_off_out;  // slice offsets in dst, or nullptr (contiguous)
};

// Row pass kinds of the register-resident passes.
// ROW_RAW: an MX row pass whose input enters the stages without the input
// encode (the inverse half of the fused round trip).
enum RowKind { ROW_PLAIN = 0, ROW_STATS = 1, ROW_FIX = 2, COL_RSS = 3, ROW_RAW = 4 };

bool fast_supported(int mode, int n, int cb);
// MXFP8 blocks of 64 values (cb = 32) on the register-resident passes: row
// tiles of 32 lines, so that a column block's 32 rows share a work-group
bool fast_wide(int mode, int n, int cb);
// whether the row pass can gather the Alg. 1 statistics (register-resident MX passes)
bool fast_fused_stats(int mode, int n);
// row: kind is one of RowKind; columns ignore it
hipError_t launch_fast(int mode, int n, int cb, bool row, bool inverse, int kind, const FastPassArgs& p,
                       int batch, hipStream_t s);
// Tiles (row chunks) per slice of the row pass with statistics.
int fast_row_tiles(int mode, int n, int cb);

// chunks: work-groups per slice (a power of two dividing n * n), 0 = by batch
hipError_t launch_stats(const float2* x, int n, int batch, StatPart* parts, int32_t* kp,
                        int32_t* slice_status, const PrescaleArgs& pa, const unsigned long long* slice_off,
                        int chunks, hipStream_t s);
// Alg. 1 from chunk statistics already in `parts` ([slice][chunks]) that the
// row pass wrote; also the equivariance check: kadd[slice] = kp when the
// unscaled row pass may stand, else 0 with the slice appended to fix_list.
// k_out (nullable) receives kp.
hipError_t launch_stats_final(const float2* x, int n, int batch, int chunks, const StatPart* parts, int32_t* kp,
                              int32_t* slice_status, const PrescaleArgs& pa, int32_t* kadd, int32_t* fix_list,
                              int32_t* fix_count, int32_t* k_out, const unsigned long long* slice_off,
                              hipStream_t s);
hipError_t launch_lines(int mode, const LineArgs& a, int batch, hipStream_t s);

// Single-launch transform of slices of n <= kSmallN (one work-group per
// slice: Alg. 1, all passes and the output in LDS); the default there
// wherever the plan has no register-resident passes, a tuning choice where it
// has them (128^2).
constexpr int kSmallN = 128;
struct SmallArgs {
    LineArgs a;                // tables, n, block, src, dst, k_out, capture pointers
    PrescaleArgs pa;
    int32_t op;                // 0 forward, 1 inverse, 2 round trip
    int32_t stats;             // Alg. 1 on the input; else k from k_in (or 0)
    int32_t kin_mul, kout_mul, kout_add;  // input x 2^(kin_mul k); output x 2^(kout_mul k + kout_add)
    int32_t raw_inverse_rows;  // round trip: the inverse row pass without the input MX encode
    const int32_t* k_in;
    int32_t* kp;               // per-slice k (stats), or nullptr
    int32_t* status;           // per-slice status (stats), or nullptr
};
// cus, lds_per_cu: the device's compute units and LDS bytes per CU (they
// set the work-group size; see small_block)
hipError_t launch_small(int mode, const SmallArgs& g, int batch, int cus, int lds_per_cu, hipStream_t s);
// The output of batch n x n slices (slice offsets off, or nullptr) MX-encoded
// in place in blocks of 2^logcb consecutive rows of one column.
hipError_t launch_quantize_out(int mode, float2* out, const unsigned long long* off, int n, int logcb, int batch,
                               hipStream_t s);
int small_block(int n, int batch, int cus, int lds_per_cu);
int line_lines_per_group(int n);
// Debug capture from the register-resident MX intermediate: element values
// [slice][row][col] and exponents [slice][col][row block] (plus kadd[slice]
// when given) of batch slices.
hipError_t launch_capture_mx(int mode, int n, int cb, const uint32_t* codes, const uint8_t* exps,
                             const int32_t* kadd, int batch, float2* mant, int32_t* cap_exp, hipStream_t s);
// Root-sum-of-squares coil combine of finished transforms (recon x coils slices).
hipError_t launch_rss(const float2* T, int coils, size_t nn, long recon, float* rss, hipStream_t s);

// Mean SSIM of count images x against references y (n x n FP32 each).
hipError_t launch_ssim(const float* x, const float* y, int n, int count, double* out, hipStream_t s);

// Synthetic finite data (tuning): count complex values, both parts in [-1, 1).
hipError_t launch_fill(float2* x, size_t count, uint32_t seed, hipStream_t s);

// Release a plan whose work has completed (the caller has seen its last
// event), without the device-wide synchronisation of mxfft_plan_destroy.
void plan_release_idle(mxfft_plan_s* pl);

// Forward transform of a checked call (1 <= batch) with the workspace w,
// which must be sized for batch slices (the plan's own, or a carve-out of the
// static array of mxfft_forward_static).
mxfft_status plan_forward_ws(mxfft_plan_s* pl, const Workspace& w, const void* in, void* out, int32_t batch,
                             int32_t* k_out, void* stream);

// Inverse and round trip of a checked call with the workspace w (as
// plan_forward_ws).
mxfft_status plan_inverse_ws(mxfft_plan_s* pl, const Workspace& w, const void* in, void* out, int32_t batch,
                             const int32_t* k_in, void* stream);
mxfft_status plan_roundtrip_ws(mxfft_plan_s* pl, const Workspace& w, const void* in, void* out, int32_t batch,
                               int32_t* k_out, void* stream);

// Workspace of a plan's forward call over `batch` slices laid out from
// `base` (each buffer 256-byte aligned): *bytes gets the extent; with base
// non-null, *w gets the buffer addresses.
void plan_workspace_layout(const mxfft_plan_s* pl, int batch, char* base, Workspace* w, size_t* bytes);

// Device the plan was created on.
int plan_device(const mxfft_plan_s* pl);

// The plan's own workspace (sized for its max_batch).
const Workspace& plan_workspace(const mxfft_plan_s* pl);

// dst[idx[i]] = src[i] for i < count (k of a merged batch branch back in the
// caller's slice order).
hipError_t launch_scatter_k(const int32_t* src, const int32_t* idx, int32_t* dst, int count, hipStream_t s);

// Device status words of a plan (one int32 per slice of its last call, written
// by the prescale statistics), and whether its calls write them.
const int32_t* plan_status_words(mxfft_plan_s* pl);
bool plan_has_status(mxfft_plan_s* pl);

}  // namespace mxk
