/*
 * mxfft.h -- C ABI of the MI355X (gfx950) MX-scaled mixed-precision 2D FFT.
 *
 * Method: Deveshwar, Rajagopal, Larson, "A mixed precision FFT with applications
 * in MRI".  A slice is one N x N complex k-space array of one coil.  Per slice the
 * library applies the single global power-of-two prescale of Alg. 1 (Sec. 2.1),
 * then an iterative radix-2 Cooley-Tukey FFT over every row and then every column,
 * whose butterflies multiply by pre-quantised FP8 twiddles in the MX-scaled form
 * of Alg. 2 (Sec. 2.2: MX-encoded operands, FP32 products and sums, stage-wise MX
 * re-encoding with one shared power-of-two scale per block of B real scalars).
 * The forward and round-trip transforms are those of Eq. 1 (Sec. 2.3).
 *
 * Conventions for every entry point:
 *  - Data pointers are DEVICE pointers owned by the caller (the library never
 *    frees or keeps them).  Complex data is interleaved FP32 (re, im), i.e.
 *    complex64; a batch is [batch][n][n], row-major, 8-byte aligned.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *    asynchronously on it; nothing here synchronises except where stated.
 *  - Errors are returned as mxfft_status.  Argument checks happen on the host
 *    before anything is enqueued, so on an argument error no buffer is touched.
 *    Data-dependent errors (non-finite input, prescale overflow) are found on
 *    the device: the slice's k becomes INT32_MIN, its output is undefined, and
 *    mxfft_plan_last_status() reports the error.
 *  - A plan is used by one stream at a time; calls that overlap on one plan race.
 */
#ifndef MXFFT_H
#define MXFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Element / arithmetic format (Sec. 2.2; Fig. 1C).  E4M3 and E5M2 are the OCP
 * 8-bit elements of MXFP8.  FP16 and BF16 are the 16-bit forms the paper
 * compares against (Sec. 2.3): every pass input, every twiddle (rounded once
 * from FP64), each stage's v operand and each product and sum of the complex
 * product are rounded to the format (IEEE round to nearest even, overflow to
 * infinity); u +/- p stays FP32 and the output is rounded to the format.  The
 * block size is ignored for them.  FP32 is the plain single-precision form of
 * the same radix-2 FFT (the comparison baseline, no quantisation).  E2M3 and
 * E3M2 are the OCP 6-bit elements of MXFP6 (no infinities or NaN), which the
 * paper evaluates beside MXFP8 (Sec. 3); blocks of 16 and 32 at n = 128..1024
 * run on the register-resident passes (the 6-bit codes held in 8-bit ones),
 * other blocks and sizes on the generic line kernels. */
typedef enum {
    MXFFT_E4M3 = 0,
    MXFFT_E5M2 = 1,
    MXFFT_FP16 = 2,
    MXFFT_BF16 = 3,
    MXFFT_FP32 = 4,
    MXFFT_E2M3 = 5,
    MXFFT_E3M2 = 6
} mxfft_format;

typedef enum {
    MXFFT_OK = 0,
    MXFFT_EINVAL = -1,        /* bad argument (size, block, parameter, pointer) */
    MXFFT_ENOMEM = -2,        /* device allocation failed while planning */
    MXFFT_EHIP = -3,          /* a HIP runtime call failed */
    MXFFT_ENONFINITE = -4,    /* a slice holds Inf or NaN (found on the device) */
    MXFFT_ERANGE = -5,        /* the prescale would overflow FP32 (found on the device) */
    MXFFT_EBUDGET = -6,       /* over a memory budget (a server's, or the static workspace) */
    MXFFT_EBUSY = -7,         /* reserved */
    MXFFT_EUNSUPPORTED = -8   /* valid for the method but not built in this library */
} mxfft_status;

/* Flags of mxfft_params.flags. */
#define MXFFT_NO_PRESCALE 0x1u  /* skip Alg. 1: k = 0 for every slice */
#define MXFFT_KEEP_SCALE  0x2u  /* forward: return 2^k * F{x} (do not de-scale) */
#define MXFFT_NORMALIZE   0x4u  /* inverse: multiply by 1/N^2 (Eq. 1 round trip) */
/* round trip, MX formats: the forward result enters the inverse transform's
 * row stages without being MX-encoded again (the encode -> F -> F^-1 -> decode
 * fusion the paper proposes in its discussion, Sec. 4; less round-trip loss).
 * No effect on the other operations and formats. */
#define MXFFT_FUSED_ROUNDTRIP 0x8u
/* MX formats: every forward call also records the column pass's MX input
 * (the row pass's result in blocks of B/2 rows of one column: Alg. 2's
 * EncodeBlockMX, element values and shared exponents), which
 * mxfft_plan_capture() returns.  The plan holds 8 + 8/B bytes more per
 * complex value of max_batch slices, and each forward call of up to
 * max_batch slices writes them. */
#define MXFFT_DEBUG_CAPTURE 0x10u
/* MX formats: the output is stored quantised, as the paper's 16-bit control
 * stores its output in its format (Sec. 2.2): after the last pass and the
 * de-scale, every column is MX-encoded in blocks of B/2 consecutive rows
 * (Alg. 2's EncodeBlockMX: shared exponent E from the block maximum, elements
 * rounded to nearest even and saturated) and each value becomes element *
 * 2^E, rounded once to FP32.  Forward, inverse and round trip; one more read
 * and write of the output.  The 16-bit forms always round their output to the
 * format; FP32 ignores the flag.  mxfft_rss refuses such plans
 * (MXFFT_EUNSUPPORTED): it never stores the per-coil results. */
#define MXFFT_QUANTIZE_OUTPUT 0x20u

typedef struct {
    uint32_t struct_size;  /* sizeof(mxfft_params); checked for ABI versioning */
    int32_t format;        /* mxfft_format */
    int32_t block;         /* B: real scalars per MX block, a power of two with
                              2 <= B <= n (B/2 complex values per block; Sec.
                              2.2 and Sec. 4.2); blocks above 128 run on the
                              line kernels.  Ignored for FP16, BF16, FP32. */
    int32_t k_min, k_max;  /* clip bounds of the prescale exponent (Alg. 1);
                              INT32_MIN / INT32_MAX mean no bound */
    uint32_t flags;        /* MXFFT_* flags above */
    double target;         /* Alg. 1 peak target T > 0 (e.g. 2^7) */
    double tau_pct;        /* Alg. 1 tail percentile tau, in percent, 0..100 */
    double tau_min;        /* Alg. 1 tail floor tau_min > 0 (any value; when it is
                              not a power of two the statistics read each
                              slice once more to place the percentile against
                              it exactly) */
} mxfft_params;

typedef struct mxfft_plan_s* mxfft_plan_t;

/* Fill p with the defaults: E4M3, B = 32, T = 2^7, tau = 5, tau_min = 2^-6,
 * no clipping, no flags. */
void mxfft_params_default(mxfft_params* p);

/* Create a plan for n x n slices (n a power of two, 2 <= n <= 4096) and batches
 * of up to max_batch slices.  The plan owns the pre-quantised twiddle tables
 * (FP64-generated, MX-encoded once per stage and block: Sec. 2.2, Alg. 2) and
 * its device workspace; it allocates device memory here and never again.
 * `stream` orders the plan's initial uploads.  *out receives the handle. */
mxfft_status mxfft_plan(mxfft_plan_t* out, int32_t n, int32_t max_batch,
                        const mxfft_params* p, void* stream);

/* Device bytes mxfft_plan would allocate for (n, max_batch, p), computed on
 * the host without any HIP call (for capacity planning and admission).  The
 * same argument checks as mxfft_plan. */
mxfft_status mxfft_plan_bytes(int32_t n, int32_t max_batch, const mxfft_params* p, uint64_t* bytes);

/* Release a plan (synchronises the device first).  NULL is accepted. */
mxfft_status mxfft_plan_destroy(mxfft_plan_t plan);

/* Forward transform (Eq. 1, forward): per slice k = Alg. 1 prescale of `in`,
 * y = F{2^k x} with rows then columns, out = 2^-k y (2^k y with KEEP_SCALE).
 * in, out: complex64 [batch][n][n] device buffers; in == out is allowed.
 * k_out: device int32[batch] receiving k per slice, or NULL.
 * 1 <= batch <= max_batch. */
mxfft_status mxfft_forward(mxfft_plan_t plan, const void* in, void* out, int32_t batch,
                           int32_t* k_out, void* stream);

/* Forward transform without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, results and status words as
 * mxfft_forward, bit for bit, but every buffer the kernels write besides `out`
 * and `k_out` (the MX or 16-bit intermediate of the register-resident passes,
 * the prescale statistics and exponents, the status words, the redo list) is
 * taken from one static device array of MXFFT_STATIC_SCRATCH_BYTES per GPU,
 * which the library holds from its first use on a device until the process
 * ends.  The plan supplies only its twiddle tables, so batch may exceed the
 * plan's max_batch (1 <= batch <= 65535) as long as that workspace fits:
 * MXFFT_EBUDGET otherwise (nothing is enqueued).  It is about 0.55 MiB per
 * slice at n = 512 and 2.2 MiB at n = 1024 for MXFP8 B = 32 (114 and 28 slices),
 * 1 MiB per slice at n = 512 for FP16/BF16, and under 5 MiB in all for plans on
 * the generic line kernels.  The plan must belong to the current device
 * (MXFFT_EINVAL otherwise).  Every call on a GPU shares that GPU's array:
 * calls that overlap on one GPU (other streams, other plans, other host
 * threads) race and give undefined results, so order them on one stream or
 * with events.  The array keeps the last call's contents; the kernels rewrite
 * every entry they read, and mxfft_plan_last_status() reads the status words
 * from it, so query it before the next call of this kind on the device.  The
 * first call on a device looks the array's address up (no allocation). */
#define MXFFT_STATIC_SCRATCH_BYTES (64u << 20)
mxfft_status mxfft_forward_static(mxfft_plan_t plan, const void* in, void* out, int32_t batch,
                                  int32_t* k_out, void* stream);

/* Inverse transform F^-1 (conjugate twiddles, same pipeline; Eq. 1).
 * k_in == NULL: the input is prescaled by its own Alg. 1 exponent k and the
 * output is 2^-k F^-1{2^k x}.  k_in != NULL (device int32[batch]): the input is
 * taken as already scaled by 2^k_in (e.g. a KEEP_SCALE forward output) and the
 * output is 2^-k_in F^-1{x}.  With NORMALIZE the output is also multiplied by
 * 1/N^2 (an exact power of two). */
mxfft_status mxfft_inverse(mxfft_plan_t plan, const void* in, void* out, int32_t batch,
                           const int32_t* k_in, void* stream);

/* Round trip (Eq. 1): T = (1/N^2) F^-1{F{x}} with one prescale k per slice,
 * kept through both transforms and removed once at the end.  in == out is
 * allowed.  k_out: device int32[batch] or NULL. */
mxfft_status mxfft_roundtrip(mxfft_plan_t plan, const void* in, void* out, int32_t batch,
                             int32_t* k_out, void* stream);

/* Eq. 1 with its root-sum-of-squares coil combine.  `in` holds `recon`
 * reconstructions of `coils` coil slices each, coil-minor: complex64
 * [recon][coils][n][n].  op 0: T_c = the forward transform of each coil (as
 * mxfft_forward, KEEP_SCALE honoured); op 2: T_c = the round trip (as
 * mxfft_roundtrip).  Output: rss[r][i] = (sum_c |T_{r,c}[i]|^2)^(1/2), FP32
 * [recon][n][n], with |T|^2 = re re + im im (each product and the sum rounded
 * to FP32, no fused multiply-add), the coils summed in order and a correctly
 * rounded square root.  The combine is fused into the last column pass:
 * the per-coil complex results are never written, only the images (1/(2 C)
 * of the plain call's output bytes).  work: complex64 [recon * coils][n][n]
 * scratch for the round trip's forward result, for the FP32 form's complex64
 * intermediate, and for the per-coil results of plans without the fused
 * epilogue (may be `in`, which is then overwritten); MXFFT_EINVAL when it is
 * needed and NULL; unused (may be NULL) otherwise.  k_out: int32[recon * coils] or NULL.  recon * coils <=
 * max_batch.  Plans on the register-resident passes (n = 128..1024 with MXFP8
 * B = 4..32, MXFP8 B = 64 at n = 256..1024, MXFP6 B = 16 or 32, or FP16/BF16,
 * and FP32 at n = 512) fuse the combine; the others (generic line kernels,
 * the single launch) write the per-coil results to work and combine them in
 * a separate kernel with the same arithmetic. */
mxfft_status mxfft_rss(mxfft_plan_t plan, int32_t op, const void* in, void* work, float* rss, int32_t recon,
                       int32_t coils, int32_t* k_out, void* stream);

/* Image quality: mean SSIM of each of `count` images x against its reference
 * ref (device FP32 [count][n][n] each, 11 <= n <= 4096) into ssim (device
 * double[count]), in the form of Wang, Bovik, Sheikh and Simoncelli (2004),
 * the metric the paper reports on RSS images (Sec. 3): local statistics under
 * an 11 x 11 Gaussian window of standard deviation 1.5 normalised to unit
 * sum, C1 = (0.01 L)^2, C2 = (0.03 L)^2 with L = max(ref), the index averaged
 * over the positions where the window lies inside the image.  FP64; one
 * work-group per image; no workspace. */
mxfft_status mxfft_ssim(const float* x, const float* ref, int32_t n, int32_t count, double* ssim, void* stream);

/* MXFFT_DEBUG_CAPTURE plans: copy (on `stream`, asynchronously) what the
 * last forward call recorded for its `batch` slices, the MX encode of the
 * column pass's input (Alg. 2, EncodeBlockMX over blocks of B/2 consecutive
 * rows of one column, after the row pass and the Alg. 1 prescale):
 *   mant: complex64 [batch][n][n] element values (the decoded codes without
 *         the block scale: E4M3/E5M2/E2M3/E3M2 values, signed zeros kept);
 *   exps: int32 [batch][n][n / (B/2)] shared exponent E of column c and row
 *         block r at [slice][c][r] (value = mant * 2^E);
 *   trace (nullable): int32 [batch][log2 n][n / B][3], for row 0 of each
 *         slice's row pass, every stage's butterfly blocks' (E_v, k_r,
 *         E_out) of Alg. 2 (v's shared exponent, the renormalisation, the
 *         product's scale exponent E_w + E_v + k_r).  Recorded by the line
 *         kernels and the single-launch kernel only: MXFFT_EUNSUPPORTED when
 *         the call ran on the register-resident passes.
 * 1 <= batch <= the batch of that call; MXFFT_EINVAL otherwise (also for a
 * plan without the flag or before any forward call). */
mxfft_status mxfft_plan_capture(mxfft_plan_t plan, void* mant, int32_t* exps, int32_t* trace, int32_t batch,
                                void* stream);

/* Synchronise `stream` and return the device status of the plan's last call
 * (MXFFT_OK, MXFFT_ENONFINITE or MXFFT_ERANGE). */
mxfft_status mxfft_plan_last_status(mxfft_plan_t plan, void* stream);

/* Per-kernel timing for benchmarks.  While enabled, every kernel the plan
 * launches is bracketed by a pair of HIP events recorded on the same stream.
 * Enabling resets the accumulated times; disabling keeps them. */
mxfft_status mxfft_plan_profile(mxfft_plan_t plan, int32_t enable);

/* As mxfft_plan_profile, timing only the launches whose role bit is set in
 * role_mask (0 disables): bit 0 prescale_stats, 1 row_pass, 2 column_pass,
 * 3 inverse_row_pass, 4 inverse_column_pass, 5 row_redo.  Fewer event pairs
 * disturb the timed launches less. */
mxfft_status mxfft_plan_profile_roles(mxfft_plan_t plan, uint32_t role_mask);

typedef struct {
    char name[32];       /* kernel role, e.g. "prescale_stats", "row_pass" */
    uint64_t launches;   /* launches timed since profiling was enabled */
    double total_ms;     /* summed event-to-event durations */
} mxfft_kernel_time;

/* Synchronise the device and report the accumulated per-role times: writes
 * up to cap entries to out and the number of roles seen to *count. */
mxfft_status mxfft_plan_kernel_times(mxfft_plan_t plan, mxfft_kernel_time* out, int32_t cap,
                                     int32_t* count);

/* Bytes of device memory the plan holds (tables and workspace). */
uint64_t mxfft_plan_device_bytes(mxfft_plan_t plan);

/* ---- Launch tuning ------------------------------------------------------
 * Sizes and formats without register-resident passes (n below 128 or above
 * 1024, MX blocks of 2 and 128, MXFP8 blocks of 64 at n = 128, MXFP6 blocks
 * other than 16 and 32, FP32 at every n but 512) run the generic line
 * kernels: one work-group
 * holds `lines` whole lines of a pass in LDS, one thread per butterfly.  Slices
 * of n <= 128 can instead run the whole 2D transform in one launch (one
 * work-group per slice holding it in LDS: Alg. 1, the row and column passes,
 * both halves of a round trip; its work-group size follows the batch), the
 * default for every n <= 128 without register-resident passes.  Which is
 * faster, and the best `lines`, depend on n, the format, the batch and the
 * GPU, so they are measured. */
typedef struct {
    int32_t lines;   /* lines per work-group: a power of two, 1 <= lines <= n,
                        lines * n * 8 <= 65536; 0 = the default (8192 / n, at most n) */
    int32_t fast;    /* out: 1 when the plan runs the register-resident passes,
                        which have no such parameter (lines is then ignored) */
    double ms;       /* out (tuner): time of one forward call over its sample */
    int32_t single;  /* n <= 128: 1 = the single-launch kernel (the default
                        without register-resident passes; lines ignored),
                        0 = the line kernels with `lines` or the
                        register-resident passes; must be 0 for n > 128 */
    int32_t stats;   /* Alg. 1 with the prescale: 0 = gathered by the row pass
                        where the plan can (register-resident MX passes,
                        n = 128 .. 1024), 1 = a separate statistics read of
                        the input before the row pass (the only way elsewhere) */
    int32_t chunks;  /* work-groups per slice of that separate read: 0 = by the
                        batch (enough to fill the GPU), else a power of two
                        with n * n / chunks >= 1024 (lowered when a batch's
                        statistics would not fit the plan's workspace) */
} mxfft_tuning;

/* Set / read a plan's launch tuning.  Set: MXFFT_EINVAL for an invalid
 * field; takes effect from the next call (no synchronisation).  Every choice
 * gives bit-identical results. */
mxfft_status mxfft_plan_set_tuning(mxfft_plan_t plan, const mxfft_tuning* t);
mxfft_status mxfft_plan_get_tuning(mxfft_plan_t plan, mxfft_tuning* t);

/* Autotuner.  Looks up (GPU architecture name, n, format, B) in the cache file
 * `cache_path` (NULL: no cache); on a miss, or with MXFFT_TUNE_FORCE, it times
 * one forward call of a plan of `sample` slices of synthetic data for every
 * candidate (the default `lines` and its halvings, at least 1, or the
 * register-resident passes' statistics choices; for n <= 128 also the
 * single-launch kernel), keeps the fastest and records it in the
 * cache (the file is rewritten whole through a temporary file and a rename;
 * entries of other keys are kept).  *out gets the choice; its `lines` is the
 * best line-kernel candidate even when `single` wins.  Allocates and frees
 * device memory and synchronises `stream`. */
#define MXFFT_TUNE_FORCE 0x1u
mxfft_status mxfft_tune(int32_t n, const mxfft_params* p, int32_t sample, const char* cache_path,
                        uint32_t tune_flags, mxfft_tuning* out, void* stream);

/* Host-only cache lookup (no GPU call): MXFFT_OK and *out filled when the file
 * holds an entry for (arch, n, p->format, p->block), MXFFT_EINVAL when it does
 * not or the file cannot be read.  The file is plain text, one entry per line:
 *   {"arch": "gfx950", "n": 64, "format": 0, "block": 32, "lines": 8, "ms": 0.1, "single": 1}
 * (format as mxfft_format; block 0 for FP16/BF16/FP32). */
mxfft_status mxfft_tune_cache_lookup(const char* cache_path, const char* arch, int32_t n,
                                     const mxfft_params* p, mxfft_tuning* out);

/* ---- Uneven batches -----------------------------------------------------
 * A work list of slice groups of different sizes, transformed by one call
 * that launches one HIP graph.  Group g holds `count` slices of n x n at
 * element offset `offset` (complex values from the pool base) of both the
 * input and the output pool; groups must not overlap, and may lie anywhere
 * (one group per reconstruction of several coils, in arrival order, for
 * example).  The groups of one size form one branch of the graph: one plan
 * and one launch sequence over all their slices, which the kernels address
 * through a per-slice offset table (at most 65535 slices per size); the
 * branches of different sizes run side by side.  The graph is captured on the
 * first call for a given (operation, input, output, k) and replayed while
 * those stay the same.  k per slice goes to k_out[kbase_g + i], kbase_g = the
 * slices of the groups before g.  Every slice's result is bit-identical to a
 * single-plan call. */
typedef struct {
    int32_t n;        /* slice size (power of two, 2..4096) */
    int32_t count;    /* slices in the group (>= 1) */
    uint64_t offset;  /* complex-value offset of the group's first slice */
} mxfft_group;

typedef struct mxfft_batch_s* mxfft_batch_t;

/* Plans one branch per distinct n (params p for all), autotunes each size on
 * the line kernels through mxfft_tune with `tune_cache` (may be NULL: tune
 * without a cache) on up to 1024 slices of that size, uploads the offset
 * tables and creates the branch streams.  Sizes on the register-resident
 * passes keep the plans' defaults (the branches share the GPU, and the
 * choices that win for one size alone were measured slower beside the other
 * sizes).  Allocates device memory; synchronises. */
mxfft_status mxfft_batch_create(mxfft_batch_t* out, const mxfft_group* groups, int32_t ngroups,
                                const mxfft_params* p, const char* tune_cache, void* stream);

/* op: 0 forward (k_out written), 1 inverse with its own prescale, 2 round trip
 * (k_out written).  in, out: the pools (in == out allowed); k_out: device
 * int32[total slices] or NULL.  One graph launch on `stream`. */
mxfft_status mxfft_batch_execute(mxfft_batch_t b, int32_t op, const void* in, void* out, int32_t* k_out,
                                 void* stream);

/* Synchronise `stream`; the first non-OK device status of the last call. */
mxfft_status mxfft_batch_last_status(mxfft_batch_t b, void* stream);

/* Tuning chosen for group g's size. */
mxfft_status mxfft_batch_group_tuning(mxfft_batch_t b, int32_t g, mxfft_tuning* out);

/* Release the batch, its plans, streams and graphs (synchronises the device). */
mxfft_status mxfft_batch_destroy(mxfft_batch_t b);

/* ---- Serving ------------------------------------------------------------
 * A server accepts transform requests from any host thread and runs them on
 * the device as capacity frees up.  One scheduler thread admits queued
 * requests in arrival order (no overtaking) while a stream slot is free and
 * the device memory of the plans it holds stays within the budget: plans
 * (tables and workspace) are pooled by (n, parameters, batch capacity: the
 * coil count rounded up to a power of two, at least 32) and reused; idle plans
 * are evicted, least recently used first, when a new one would exceed the
 * budget.  A planner thread creates and frees the plans, so admission of later
 * requests and completion of running ones never wait on an allocation or a
 * free.  When a slot frees, the request at the head of the queue takes it
 * together with the queued requests behind it (up to 64 looked at) that have
 * the same n, parameters and operation and fit its plan's capacity (at most
 * 1024 slices): one launch sequence over all their slices, each request's
 * buffers addressed through per-slice offset tables.  Up to `slots` launches
 * run at once, each on its own stream, so transfers of results and the
 * kernels of different requests overlap.  A request's input and output stay
 * caller-owned (pre-staged device buffers; complex64, so 8-byte aligned for
 * a shared launch); each request is computed exactly as a single
 * mxfft_forward / mxfft_inverse / mxfft_roundtrip call on its coils would be
 * (every slice is transformed independently), so its result does not depend
 * on what else runs or shares its launch. */
typedef struct mxfft_server_s* mxfft_server_t;

typedef struct {
    const void* in;       /* device complex64 [coils][n][n] */
    void* out;            /* device complex64 [coils][n][n] (may equal in) */
    int32_t* k_out;       /* device int32[coils] or NULL (forward and round trip) */
    int32_t n;            /* slice size (power of two, 2..4096) */
    int32_t coils;        /* slices in the request, 1..65535 */
    int32_t op;           /* 0 forward, 1 inverse (own prescale), 2 round trip */
    mxfft_params params;  /* format, block, prescale parameters, flags */
    void* ready;          /* hipEvent_t or NULL.  The request's stream waits on
                             it before its first kernel: record it on the
                             stream that produces `in` (and last used `out`),
                             after that work.  NULL: the caller guarantees the
                             input is complete on the device at submission.
                             The event must stay valid until the ticket is
                             answered. */
} mxfft_request;

typedef struct {
    int32_t status;       /* MXFFT_OK, or the request's device status (ENONFINITE, ERANGE) */
    int32_t slot;         /* stream slot it ran on */
    double t_submit_ms;   /* host steady clock, ms since the server was created */
    double t_start_ms;    /* launched */
    double t_done_ms;     /* completion seen by the scheduler */
} mxfft_result;

typedef struct {
    uint64_t submitted, admitted, completed, rejected;
    uint64_t queued, in_flight;           /* now */
    uint64_t plan_bytes, peak_plan_bytes; /* device bytes of the pooled plans: now, highest */
    uint64_t plans_created, plans_evicted;
    uint64_t budget;
    uint64_t coalesced_launches;          /* launches that served several requests */
    uint64_t coalesced_requests;          /* requests served by them */
} mxfft_serve_counters;

/* Create a server with `slots` concurrent requests (1..16; each its own
 * non-blocking stream of default priority) and a device-memory budget for its
 * plans.  Starts the scheduler thread. */
mxfft_status mxfft_serve_create(mxfft_server_t* out, uint64_t hbm_budget_bytes, int32_t slots);

/* Queue a request (non-blocking; any thread).  *ticket identifies it.
 * MXFFT_EINVAL for bad arguments and MXFFT_EBUDGET when its plan alone would
 * exceed the budget (counted as rejected; nothing is queued).  The request
 * runs on a stream of the server, not on the caller's: its input must be
 * complete when its `ready` event fires (or at submission without one), and
 * in, out and k_out must stay allocated and untouched by other work until the
 * ticket is answered by mxfft_serve_wait or mxfft_serve_poll. */
mxfft_status mxfft_serve_submit(mxfft_server_t srv, const mxfft_request* req, uint64_t* ticket);

/* Block until the request is done and fill *res; a ticket is answered once
 * (then MXFFT_EINVAL).  The returned status is that of the call (MXFFT_OK when
 * *res is filled); the request's own status is res->status. */
mxfft_status mxfft_serve_wait(mxfft_server_t srv, uint64_t ticket, mxfft_result* res);

/* As mxfft_serve_wait without blocking: MXFFT_EBUSY while it is not done. */
mxfft_status mxfft_serve_poll(mxfft_server_t srv, uint64_t ticket, mxfft_result* res);

/* Hold (hold = 1) or resume (0) admissions: while held, submitted requests
 * queue and running ones finish, but nothing new is admitted (maintenance,
 * or filling the queue to measure the sustainable rate).  Destroying a held
 * server still runs its queued requests.  MXFFT_EINVAL for another value. */
mxfft_status mxfft_serve_hold(mxfft_server_t srv, int32_t hold);

/* Counters (a consistent snapshot). */
mxfft_status mxfft_serve_stats(mxfft_server_t srv, mxfft_serve_counters* out);

/* Finish every queued and running request, stop the scheduler and release
 * the plans, streams and host buffers.  Unanswered tickets are dropped. */
mxfft_status mxfft_serve_destroy(mxfft_server_t srv);

/* Static text for a status code. */
const char* mxfft_status_string(mxfft_status st);

/* Library version as 10000*major + 100*minor + patch. */
int32_t mxfft_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MXFFT_H */
