// mxfft_host.cpp -- plans, argument checks, twiddle pre-quantisation and the
// launch sequences behind the C ABI of include/mxfft.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>

#include "mxfft.h"
#include "mxfft_internal.hpp"

namespace {

constexpr uint32_t kKnownFlags =
    MXFFT_NO_PRESCALE | MXFFT_KEEP_SCALE | MXFFT_NORMALIZE | MXFFT_FUSED_ROUNDTRIP | MXFFT_DEBUG_CAPTURE |
    MXFFT_QUANTIZE_OUTPUT;

// Element formats for twiddle pre-quantisation (OCP E4M3 / E5M2) and the
// 16-bit forms (IEEE half, bfloat16; twiddles never reach their overflow).
struct HostElem {
    int mbits, emin, emax;
    double maxv;
};
const HostElem kE4M3 = {3, -6, 8, 448.0};
const HostElem kE5M2 = {2, -14, 15, 57344.0};
const HostElem kE2M3 = {3, 0, 2, 7.5};       // OCP FP6 (no infinities or NaN)
const HostElem kE3M2 = {2, -2, 4, 28.0};
const HostElem kFP16 = {10, -14, 15, 65504.0};
const HostElem kBF16 = {7, -126, 127, 3.3895313892515355e38};

// Nearest element value (ties to the even multiple of the grid step),
// saturating at the largest finite element.
double round_to_elem(double x, const HostElem& f)
{
    if (x == 0.0) return x;
    const double a = std::fabs(x);
    int e2;
    std::frexp(a, &e2);          // a in [2^(e2-1), 2^e2)
    int e = e2 - 1;
    if (e < f.emin) e = f.emin;  // subnormal grid
    const double step = std::ldexp(1.0, e - f.mbits);
    const double units = a / step;          // exact: power-of-two division
    double whole = std::floor(units);
    const double frac = units - whole;
    if (frac > 0.5 || (frac == 0.5 && std::fmod(whole, 2.0) != 0.0)) whole += 1.0;
    double r = whole * step;
    if (r > f.maxv) r = f.maxv;
    return std::copysign(r, x);
}

// exp(-2 pi i j / m) for 0 <= j < m / 2, evaluated in extended precision on
// the reduced angle and rounded to FP64; the axes are exact.
void twiddle(long j, long m, double* re, double* im)
{
    const long double two_pi = 6.283185307179586476925286766559005768L;
    long double c, s;
    if (j == 0) { c = 1.0L; s = 0.0L; }
    else if (4 * j == m) { c = 0.0L; s = 1.0L; }
    else if (4 * j < m) {
        const long double t = two_pi * (long double)j / (long double)m;
        c = cosl(t); s = sinl(t);
    } else {
        // pi - t: cos changes sign, sin does not
        const long double t = two_pi * (long double)(m / 2 - j) / (long double)m;
        c = -cosl(t); s = sinl(t);
    }
    *re = (double)c;
    *im = -(double)s;
}

int ilog2(long n)
{
    int l = 0;
    while ((1L << l) < n) l++;
    return l;
}

bool is_pow2(long n) { return n > 0 && (n & (n - 1)) == 0; }

}  // namespace

struct mxfft_plan_s {
    int n = 0, logn = 0, max_batch = 0;
    mxfft_params p{};
    int mode = 0;           // mxk::Mode
    int cb = 1, logcb = 0;  // complex values per MX block
    int device = 0;
    float2* d_tw = nullptr;
    int32_t* d_tw_exp = nullptr;
    int32_t tw_exp_off[mxk::kMaxLog2N + 2] = {};
    // per-call workspace for batches up to max_batch (the MX or 16-bit
    // intermediate of the register-resident passes, statistics, exponents)
    mxk::Workspace ws;
    // status words written by the last call (the plan's own, or those of the
    // shared static workspace after mxfft_forward_static)
    const int32_t* last_status = nullptr;
    // generic line kernels: lines per work-group (0 = line_lines_per_group)
    int lines = 0;
    // n <= 128: the whole transform in one launch instead of the line kernels
    bool single = false;
    // the device's compute units and LDS bytes per CU (the single launch's
    // work-group size follows them and the batch)
    int cus = 256, lds_per_cu = 160 * 1024;
    // Alg. 1 as a separate read even where the row pass could gather it, and
    // work-groups per slice of that read (0 = by batch)
    bool literal_stats = false;
    int chunks = 0;
    // sizing only: nothing is allocated or uploaded
    bool dry = false;
    // register-resident passes: twiddles at [h + j]
    bool fast = false;
    float2* d_twf = nullptr;
    uint32_t* d_tw16 = nullptr;      // FP16 form: the same twiddles as packed halves
    // statistics gathered by the row pass (MX at 512^2 and 1024^2)
    bool fused = false;
    // MXFFT_DEBUG_CAPTURE: the column pass input of the last forward call
    float2* d_cap_mant = nullptr;
    int32_t* d_cap_exp = nullptr;
    int32_t* d_cap_trace = nullptr;  // row pass line 0: (E_v, k_r, E_out) per stage and block
    int cap_batch = 0;
    bool cap_trace_ok = false;       // the last capture ran on kernels that record the trace
    uint64_t bytes = 0;
    int last_batch = 0;
    bool last_has_stats = false;
    // event timing of launches (benchmark support)
    struct Timed {
        int role;
        hipEvent_t start, stop;
    };
    bool profiling = false;
    uint32_t profile_mask = 0;
    std::vector<Timed> pending;
    std::vector<hipEvent_t> spare;
    uint64_t launches[8] = {};
    double total_ms[8] = {};
};

namespace {

enum Role { ROLE_STATS = 0, ROLE_ROW, ROLE_COL, ROLE_INV_ROW, ROLE_INV_COL, ROLE_FIX, ROLE_SMALL, ROLE_COUNT };
const char* const kRoleNames[ROLE_COUNT] = {"prescale_stats", "row_pass", "column_pass", "inverse_row_pass",
                                            "inverse_column_pass", "row_redo", "single_launch"};

hipEvent_t take_event(mxfft_plan_s* pl)
{
    hipEvent_t e = nullptr;
    if (!pl->spare.empty()) {
        e = pl->spare.back();
        pl->spare.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
    }
    return e;
}

// Brackets one launch with events when profiling is on.
struct LaunchTimer {
    mxfft_plan_s* pl;
    int role;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    LaunchTimer(mxfft_plan_s* p, int r, hipStream_t st) : pl(p), role(r), s(st)
    {
        if (!pl->profiling || !((pl->profile_mask >> r) & 1u)) return;
        a = take_event(pl);
        b = take_event(pl);
        if (a && b) (void)hipEventRecord(a, s);
    }
    ~LaunchTimer()
    {
        if (!a || !b) return;
        (void)hipEventRecord(b, s);
        pl->pending.push_back({role, a, b});
    }
};

void collect_times(mxfft_plan_s* pl)
{
    for (auto& t : pl->pending) {
        float ms = 0.f;
        if (hipEventSynchronize(t.stop) == hipSuccess && hipEventElapsedTime(&ms, t.start, t.stop) == hipSuccess) {
            pl->launches[t.role]++;
            pl->total_ms[t.role] += ms;
        }
        pl->spare.push_back(t.start);
        pl->spare.push_back(t.stop);
    }
    pl->pending.clear();
}

mxfft_status check_params(const mxfft_params* p, int n)
{
    if (!p || p->struct_size != sizeof(mxfft_params)) return MXFFT_EINVAL;
    if (p->flags & ~kKnownFlags) return MXFFT_EINVAL;
    switch (p->format) {
    case MXFFT_E4M3:
    case MXFFT_E5M2:
    case MXFFT_E2M3:
    case MXFFT_E3M2:
        if (!is_pow2(p->block) || p->block < 2 || p->block > n) return MXFFT_EINVAL;
        break;
    case MXFFT_FP32:
    case MXFFT_FP16:
    case MXFFT_BF16:
        if (p->flags & MXFFT_DEBUG_CAPTURE) return MXFFT_EINVAL;   // MX formats only
        break;
    default: return MXFFT_EINVAL;
    }
    if (!(p->flags & MXFFT_NO_PRESCALE)) {
        if (!std::isfinite(p->target) || !(p->target > 0.0)) return MXFFT_EINVAL;
        if (!(p->tau_pct >= 0.0 && p->tau_pct <= 100.0)) return MXFFT_EINVAL;
        if (!std::isfinite(p->tau_min) || !(p->tau_min > 0.0)) return MXFFT_EINVAL;
        if (p->k_min > p->k_max) return MXFFT_EINVAL;
    }
    return MXFFT_OK;
}

// Device allocation of a plan's table or workspace; a dry plan only counts
// the bytes (mxfft_plan_bytes).
template <class T>
mxfft_status dev_alloc(mxfft_plan_s* pl, T** ptr, size_t count)
{
    *ptr = nullptr;
    if (!pl->dry && hipMalloc((void**)ptr, count * sizeof(T)) != hipSuccess) {
        *ptr = nullptr;
        return MXFFT_ENOMEM;
    }
    pl->bytes += count * sizeof(T);
    return MXFFT_OK;
}

void release(mxfft_plan_s* pl)
{
    if (!pl) return;
    collect_times(pl);
    for (hipEvent_t e : pl->spare) (void)hipEventDestroy(e);
    (void)hipFree(pl->d_tw);
    (void)hipFree(pl->d_tw_exp);
    (void)hipFree(pl->d_twf);
    (void)hipFree(pl->d_tw16);
    (void)hipFree(pl->d_cap_mant);
    (void)hipFree(pl->d_cap_exp);
    (void)hipFree(pl->d_cap_trace);
    (void)hipFree(pl->ws.parts);
    (void)hipFree(pl->ws.kp);
    (void)hipFree(pl->ws.status);
    (void)hipFree(pl->ws.codes);
    (void)hipFree(pl->ws.exps);
    (void)hipFree(pl->ws.kadd);
    (void)hipFree(pl->ws.fix_list);
    (void)hipFree(pl->ws.fix_count);
    delete pl;
}

// Twiddle tables, stage s at offset 2^(s-1) - 1: FP32 values for the plain
// form; for MX the element values of each pre-quantised block (blocks of
// min(cb, h) consecutive j, shared exponent floor(log2 amax) - emax).
void build_twiddles(const mxfft_plan_s* pl, std::vector<float2>& tw, std::vector<int32_t>& tw_exp,
                    int32_t* off)
{
    const int n = pl->n;
    tw.assign(n > 1 ? n - 1 : 1, make_float2(0.f, 0.f));
    tw_exp.clear();
    const HostElem& f = (pl->mode == mxk::MODE_E5M2)   ? kE5M2
                        : (pl->mode == mxk::MODE_E2M3) ? kE2M3
                        : (pl->mode == mxk::MODE_E3M2) ? kE3M2
                                                       : kE4M3;
    for (int s = 1; s <= pl->logn; s++) {
        const long m = 1L << s, h = m / 2;
        off[s] = (int32_t)tw_exp.size();
        std::vector<double> wr(h), wi(h);
        for (long j = 0; j < h; j++) twiddle(j, m, &wr[j], &wi[j]);
        if (pl->mode == mxk::MODE_FP32) {
            for (long j = 0; j < h; j++) tw[h - 1 + j] = make_float2((float)wr[j], (float)wi[j]);
            continue;
        }
        if (pl->mode == mxk::MODE_FP16 || pl->mode == mxk::MODE_BF16) {
            // FP64 rounded once to the 16-bit format
            const HostElem& h16 = (pl->mode == mxk::MODE_FP16) ? kFP16 : kBF16;
            for (long j = 0; j < h; j++)
                tw[h - 1 + j] = make_float2((float)round_to_elem(wr[j], h16), (float)round_to_elem(wi[j], h16));
            continue;
        }
        const long tb = (pl->cb < h) ? pl->cb : h;
        for (long j0 = 0; j0 < h; j0 += tb) {
            double amax = 0.0;
            for (long j = j0; j < j0 + tb; j++) amax = std::fmax(amax, std::fmax(std::fabs(wr[j]), std::fabs(wi[j])));
            int e2;
            std::frexp(amax, &e2);
            const int E = (e2 - 1) - f.emax;   // amax >= 1/sqrt(2): no clamp needed
            tw_exp.push_back(E);
            for (long j = j0; j < j0 + tb; j++)
                tw[h - 1 + j] = make_float2((float)round_to_elem(std::ldexp(wr[j], -E), f),
                                            (float)round_to_elem(std::ldexp(wi[j], -E), f));
        }
    }
    if (tw_exp.empty()) tw_exp.push_back(0);
}

// Element counts of the per-call workspace for batches of up to `batch`
// slices (after pl->fast and pl->fused are set).
struct WsCounts {
    size_t parts, kp, status, codes, exps, kadd, fix_list, fix_count;
};

WsCounts ws_counts(const mxfft_plan_s* pl, int batch)
{
    const size_t n = (size_t)pl->n, b = (size_t)batch;
    WsCounts c{};
    // chunk statistics: the literal statistics pass, or one part per row tile
    c.parts = mxk::stats_parts(pl->n, batch);
    if (pl->fused) c.parts = std::max(c.parts, b * mxk::fast_row_tiles(pl->mode, pl->n, pl->cb));
    c.kp = b;
    c.status = b;
    if (pl->fast && mxk::is_mx_mode(pl->mode)) {
        // MX intermediate: codes (2 bytes per complex value) and block exponents
        c.codes = b * n * n / 2;
        c.exps = b * n * (n / (size_t)pl->cb);
        c.kadd = b;
        c.fix_list = b;
        c.fix_count = 1;
    }
    if (pl->fast && (pl->mode == mxk::MODE_FP16 || pl->mode == mxk::MODE_BF16))
        c.codes = b * n * n;   // one packed 16-bit pair per value
    return c;
}

#define MX_TRY(expr)                          \
    do {                                      \
        mxfft_status st_ = (expr);            \
        if (st_ != MXFFT_OK) return st_;      \
    } while (0)

// One pass over rows (axis 0) or columns (axis 1).  kind (row pass of the
// register-resident path): ROW_PLAIN, ROW_STATS (unscaled, with the Alg. 1
// statistics) or ROW_FIX (the listed slices only).  kadd: column pass offsets
// of the stored exponents (after a ROW_STATS row pass), else nullptr.
mxfft_status pass(mxfft_plan_s* pl, const mxk::Workspace& w, const void* src, void* dst, const int32_t* kp,
                  int32_t* k_out,
                  int kin_mul, int kout_mul, int kout_add, int axis, int inverse, int batch, hipStream_t s,
                  int kind = mxk::ROW_PLAIN, const int32_t* kadd = nullptr, float* rss = nullptr,
                  int coils = 0, bool capture = false)
{
    const int role = (kind == mxk::ROW_FIX) ? ROLE_FIX
                     : inverse              ? (axis ? ROLE_INV_COL : ROLE_INV_ROW)
                                            : (axis ? ROLE_COL : ROLE_ROW);
    LaunchTimer timer(pl, role, s);
    if (pl->fast) {
        // rows: complex64 src -> MX intermediate (or FP32 dst); columns: intermediate -> dst
        if (mxk::is_mx_mode(pl->mode) && (!w.codes || !w.exps)) return MXFFT_EHIP;
        mxk::FastPassArgs f{};
        f.src = (const float2*)src;
        f.dst = (float2*)dst;
        f.codes = w.codes;
        f.exps = w.exps;
        f.kp = kp;
        f.k_out = k_out;
        f.kin_mul = kin_mul;
        f.kout_mul = kout_mul;
        f.kout_add = kout_add;
        f.tw = pl->d_twf;
        f.tw16 = pl->d_tw16;
        f.rss = rss;
        f.coils = coils;
        f.tw_exp = pl->d_tw_exp;
        for (int i = 0; i < 16; i++) f.tw_off[i] = i < mxk::kMaxLog2N + 2 ? pl->tw_exp_off[i] : 0;
        f.parts = w.parts;
        f.kadd = kadd;
        f.fix_list = w.fix_list;
        f.fix_count = w.fix_count;
        f.slice_off = w.slice_off;
        f.slice_off_out = w.slice_off_out ? w.slice_off_out : w.slice_off;
        return mxk::launch_fast(pl->mode, pl->n, pl->cb, axis == 0, inverse != 0, kind, f, batch, s) == hipSuccess
                   ? MXFFT_OK
                   : MXFFT_EHIP;
    }
    mxk::LineArgs a{};
    a.src = (const float2*)src;
    a.dst = (float2*)dst;
    a.kp = kp;
    a.k_out = k_out;
    a.kin_mul = kin_mul;
    a.kout_mul = kout_mul;
    a.kout_add = kout_add;
    a.tw = pl->d_tw;
    a.tw_exp = pl->d_tw_exp;
    std::memcpy(a.tw_exp_off, pl->tw_exp_off, sizeof(a.tw_exp_off));
    a.n = pl->n;
    a.logn = pl->logn;
    a.cb = pl->cb;
    a.logcb = pl->logcb;
    a.lines = pl->lines ? pl->lines : mxk::line_lines_per_group(pl->n);
    a.axis = axis;
    a.inverse = inverse;
    a.encode = mxk::is_mx_mode(pl->mode) && kind != mxk::ROW_RAW;
    a.cap_mant = capture ? pl->d_cap_mant : nullptr;
    a.cap_exp = capture ? pl->d_cap_exp : nullptr;
    a.cap_trace = capture ? pl->d_cap_trace : nullptr;
    a.slice_off = w.slice_off;
    a.slice_off_out = w.slice_off_out ? w.slice_off_out : w.slice_off;
    return mxk::launch_lines(pl->mode, a, batch, s) == hipSuccess ? MXFFT_OK : MXFFT_EHIP;
}

mxk::PrescaleArgs prescale_args(const mxfft_plan_s* pl)
{
    mxk::PrescaleArgs pa{};
    pa.target = pl->p.target;
    pa.tau = pl->p.tau_pct;
    pa.tau_min = pl->p.tau_min;
    pa.k_min = pl->p.k_min;
    pa.k_max = pl->p.k_max;
    return pa;
}

int inverse_row_kind(const mxfft_plan_s* pl);

// whether a call with the prescale gathers Alg. 1's statistics in the row pass
bool fused_stats(const mxfft_plan_s* pl) { return pl->fused && !pl->literal_stats; }

// The whole transform of slices of n <= 64 in one launch.  op 0 forward,
// 1 inverse, 2 round trip; stats: Alg. 1 on the input (else k from k_in or 0).
mxfft_status small(mxfft_plan_s* pl, const mxk::Workspace& w, const void* in, void* out, int op, bool stats,
                   const int32_t* k_in, int32_t* k_out, int kin_mul, int kout_mul, int kout_add, bool capture,
                   int batch, hipStream_t s)
{
    LaunchTimer timer(pl, ROLE_SMALL, s);
    mxk::SmallArgs g{};
    g.a.src = (const float2*)in;
    g.a.dst = (float2*)out;
    g.a.k_out = k_out;
    g.a.tw = pl->d_tw;
    g.a.tw_exp = pl->d_tw_exp;
    std::memcpy(g.a.tw_exp_off, pl->tw_exp_off, sizeof(g.a.tw_exp_off));
    g.a.n = pl->n;
    g.a.logn = pl->logn;
    g.a.cb = pl->cb;
    g.a.logcb = pl->logcb;
    g.a.cap_mant = capture ? pl->d_cap_mant : nullptr;
    g.a.cap_exp = capture ? pl->d_cap_exp : nullptr;
    g.a.cap_trace = capture ? pl->d_cap_trace : nullptr;
    g.a.slice_off = w.slice_off;
    g.a.slice_off_out = w.slice_off_out ? w.slice_off_out : w.slice_off;
    g.pa = prescale_args(pl);
    g.op = op;
    g.stats = stats ? 1 : 0;
    g.kin_mul = kin_mul;
    g.kout_mul = kout_mul;
    g.kout_add = kout_add;
    g.raw_inverse_rows = (op == 2 && inverse_row_kind(pl) == mxk::ROW_RAW) ? 1 : 0;
    g.k_in = k_in;
    g.kp = stats ? w.kp : nullptr;
    g.status = stats ? w.status : nullptr;
    return mxk::launch_small(pl->mode, g, batch, pl->cus, pl->lds_per_cu, s) == hipSuccess ? MXFFT_OK : MXFFT_EHIP;
}

// Literal Alg. 1: a statistics pass over the input, then kp per slice.
mxfft_status stats(mxfft_plan_s* pl, const mxk::Workspace& w, const void* in, int batch, hipStream_t s)
{
    const mxk::PrescaleArgs pa = prescale_args(pl);
    LaunchTimer timer(pl, ROLE_STATS, s);
    // a chunk count the workspace cannot hold for this batch falls back to the default
    int chunks = pl->chunks;
    if (chunks > 0 && (size_t)chunks * batch > mxk::stats_parts(pl->n, batch)) chunks = 0;
    if (mxk::launch_stats((const float2*)in, pl->n, batch, w.parts, w.kp, w.status, pa, w.slice_off, chunks, s) !=
        hipSuccess)
        return MXFFT_EHIP;
    return MXFFT_OK;
}

// Row pass with Alg. 1 folded in (register-resident MX path).  MX encoding
// and the radix-2 stages are exactly equivariant under power-of-two scaling
// while no block exponent reaches the E8M0 limits and no FP32 value leaves
// the normal range, so the row pass runs on the unscaled input and gathers
// the prescale statistics on the way.  kp then follows per slice; where the
// block exponents of that pass (and the same plus kp) stay inside
// [kEquivLo, kEquivHi], the stored intermediate is the scaled row pass with
// its exponents offset by -kp, which the column pass adds back (kadd = kp);
// any other slice gets the literal row pass of x * 2^kp (kadd = 0).
mxfft_status row_with_stats(mxfft_plan_s* pl, const mxk::Workspace& w, const void* in, int32_t* k_out, int inverse,
                            int batch, hipStream_t s)
{
    MX_TRY(pass(pl, w, in, nullptr, nullptr, nullptr, 0, 0, 0, 0, inverse, batch, s, mxk::ROW_STATS));
    {
        const mxk::PrescaleArgs pa = prescale_args(pl);
        LaunchTimer timer(pl, ROLE_STATS, s);
        const int tiles = mxk::fast_row_tiles(pl->mode, pl->n, pl->cb);
        if (mxk::launch_stats_final((const float2*)in, pl->n, batch, tiles, w.parts, w.kp, w.status, pa, w.kadd,
                                    w.fix_list, w.fix_count, k_out, w.slice_off, s) != hipSuccess)
            return MXFFT_EHIP;
    }
    return pass(pl, w, in, nullptr, w.kp, nullptr, 1, 0, 0, 0, inverse, batch, s, mxk::ROW_FIX);
}

// Row pass kind of the round trip's inverse half: without the input encode
// when the fused round trip is asked for (MX formats).
int inverse_row_kind(const mxfft_plan_s* pl)
{
    return (pl->p.flags & MXFFT_FUSED_ROUNDTRIP) && mxk::is_mx_mode(pl->mode) ? mxk::ROW_RAW : mxk::ROW_PLAIN;
}

mxfft_status check_call(const mxfft_plan_s* pl, const void* in, const void* out, int32_t batch)
{
    if (!pl || !in || !out) return MXFFT_EINVAL;
    if (batch < 0 || batch > pl->max_batch) return MXFFT_EINVAL;
    return MXFFT_OK;
}


}  // namespace

extern "C" {

void mxfft_params_default(mxfft_params* p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->struct_size = sizeof(mxfft_params);
    p->format = MXFFT_E4M3;
    p->block = 32;
    p->k_min = INT32_MIN;
    p->k_max = INT32_MAX;
    p->flags = 0;
    p->target = 128.0;
    p->tau_pct = 5.0;
    p->tau_min = 1.0 / 64.0;
}

}  // extern "C"

namespace {

// Plan creation; with dry set, only the device bytes the plan would hold are
// counted (no HIP call is made) and returned in *dry_bytes.
mxfft_status plan_create(mxfft_plan_t* out, int32_t n, int32_t max_batch, const mxfft_params* p, void* stream,
                         bool dry, uint64_t* dry_bytes)
{
    if (!out) return MXFFT_EINVAL;
    *out = nullptr;
    if (!is_pow2(n) || n < 2 || n > (1 << mxk::kMaxLog2N)) return MXFFT_EINVAL;
    if (max_batch < 1 || max_batch > 65535) return MXFFT_EINVAL;
    MX_TRY(check_params(p, n));

    mxfft_plan_s* pl = new mxfft_plan_s();
    pl->dry = dry;
    pl->n = n;
    pl->logn = ilog2(n);
    pl->max_batch = max_batch;
    pl->p = *p;
    pl->mode = (p->format == MXFFT_E4M3)   ? mxk::MODE_E4M3
               : (p->format == MXFFT_E5M2) ? mxk::MODE_E5M2
               : (p->format == MXFFT_E2M3) ? mxk::MODE_E2M3
               : (p->format == MXFFT_E3M2) ? mxk::MODE_E3M2
               : (p->format == MXFFT_FP16) ? mxk::MODE_FP16
               : (p->format == MXFFT_BF16) ? mxk::MODE_BF16
                                           : mxk::MODE_FP32;
    if (mxk::is_mx_mode(pl->mode)) {
        pl->cb = p->block / 2;
        pl->logcb = ilog2(pl->cb);
    }
    if (!dry) {
        (void)hipGetDevice(&pl->device);
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, pl->device) == hipSuccess && v > 0)
            pl->cus = v;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, pl->device) == hipSuccess &&
            v > 0)
            pl->lds_per_cu = v;
    }
    hipStream_t s = (hipStream_t)stream;

    std::vector<float2> tw;
    std::vector<int32_t> tw_exp;
    build_twiddles(pl, tw, tw_exp, pl->tw_exp_off);

    pl->fast = mxk::fast_supported(pl->mode, n, pl->cb);
    pl->fused = pl->fast && mxk::fast_fused_stats(pl->mode, n);
    pl->single = !pl->fast && n <= mxk::kSmallN;
    mxfft_status st = MXFFT_OK;
    if (st == MXFFT_OK) st = dev_alloc(pl, &pl->d_tw, tw.size());
    if (st == MXFFT_OK) st = dev_alloc(pl, &pl->d_tw_exp, tw_exp.size());
    {
        const WsCounts c = ws_counts(pl, max_batch);
        if (st == MXFFT_OK) st = dev_alloc(pl, &pl->ws.parts, c.parts);
        if (st == MXFFT_OK) st = dev_alloc(pl, &pl->ws.kp, c.kp);
        if (st == MXFFT_OK) st = dev_alloc(pl, &pl->ws.status, c.status);
        if (st == MXFFT_OK && c.codes) st = dev_alloc(pl, &pl->ws.codes, c.codes);
        if (st == MXFFT_OK && c.exps) st = dev_alloc(pl, &pl->ws.exps, c.exps);
        if (st == MXFFT_OK && c.kadd) st = dev_alloc(pl, &pl->ws.kadd, c.kadd);
        if (st == MXFFT_OK && c.fix_list) st = dev_alloc(pl, &pl->ws.fix_list, c.fix_list);
        if (st == MXFFT_OK && c.fix_count) st = dev_alloc(pl, &pl->ws.fix_count, c.fix_count);
    }
    if (st == MXFFT_OK && (p->flags & MXFFT_DEBUG_CAPTURE)) {
        st = dev_alloc(pl, &pl->d_cap_mant, (size_t)max_batch * n * n);
        if (st == MXFFT_OK) st = dev_alloc(pl, &pl->d_cap_exp, (size_t)max_batch * n * (n / pl->cb));
        if (st == MXFFT_OK)
            st = dev_alloc(pl, &pl->d_cap_trace, (size_t)max_batch * pl->logn * (n / (2 * pl->cb)) * 3);
    }
    std::vector<float2> twf;
    std::vector<uint32_t> tw16;
    if (st == MXFFT_OK && pl->fast) {
        twf.assign((size_t)n, make_float2(0.f, 0.f));
        for (long h = 1; h < n; h <<= 1)
            for (long j = 0; j < h; j++) twf[h + j] = tw[h - 1 + j];
        st = dev_alloc(pl, &pl->d_twf, twf.size());
        if (st == MXFFT_OK && pl->mode == mxk::MODE_FP16) {
            // the twiddles are halves already: packed exactly
            tw16.assign((size_t)n, 0u);
            for (size_t i = 0; i < twf.size(); i++) {
                const _Float16 re = (_Float16)twf[i].x, im = (_Float16)twf[i].y;
                uint16_t br, bi;
                std::memcpy(&br, &re, 2);
                std::memcpy(&bi, &im, 2);
                tw16[i] = (uint32_t)br | ((uint32_t)bi << 16);
            }
            st = dev_alloc(pl, &pl->d_tw16, tw16.size());
        }
    }
    if (dry) {
        *dry_bytes = pl->bytes;
        delete pl;
        return st;
    }
    if (st != MXFFT_OK) {
        release(pl);
        return st;
    }
    bool ok = hipMemcpyAsync(pl->d_tw, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice, s) == hipSuccess;
    ok = ok && hipMemcpyAsync(pl->d_tw_exp, tw_exp.data(), tw_exp.size() * sizeof(int32_t), hipMemcpyHostToDevice, s) == hipSuccess;
    if (pl->fast)
        ok = ok && hipMemcpyAsync(pl->d_twf, twf.data(), twf.size() * sizeof(float2), hipMemcpyHostToDevice, s) == hipSuccess;
    if (pl->d_tw16)
        ok = ok && hipMemcpyAsync(pl->d_tw16, tw16.data(), tw16.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s) == hipSuccess;
    ok = ok && hipMemsetAsync(pl->ws.status, 0, sizeof(int32_t) * (size_t)max_batch, s) == hipSuccess;
    ok = ok && hipStreamSynchronize(s) == hipSuccess;
    if (!ok) {
        release(pl);
        return MXFFT_EHIP;
    }
    *out = pl;
    return MXFFT_OK;
}

}  // namespace

namespace mxk {

const int32_t* plan_status_words(mxfft_plan_t pl) { return pl->ws.status; }

void plan_release_idle(mxfft_plan_t pl) { release(pl); }

bool plan_has_status(mxfft_plan_t pl) { return !(pl->p.flags & MXFFT_NO_PRESCALE); }

int plan_device(const mxfft_plan_s* pl) { return pl->device; }

const Workspace& plan_workspace(const mxfft_plan_s* pl) { return pl->ws; }

void plan_workspace_layout(const mxfft_plan_s* pl, int batch, char* base, Workspace* w, size_t* bytes)
{
    const WsCounts c = ws_counts(pl, batch);
    size_t off = 0;
    auto take = [&](auto** ptr, size_t count) {
        using T = std::remove_pointer_t<std::remove_reference_t<decltype(*ptr)>>;
        if (base) *ptr = count ? (T*)(base + off) : nullptr;
        off += (count * sizeof(T) + 255) & ~(size_t)255;
    };
    Workspace tmp;
    Workspace* o = w ? w : &tmp;
    take(&o->parts, c.parts);
    take(&o->kp, c.kp);
    take(&o->status, c.status);
    take(&o->codes, c.codes);
    take(&o->exps, c.exps);
    take(&o->kadd, c.kadd);
    take(&o->fix_list, c.fix_list);
    take(&o->fix_count, c.fix_count);
    *bytes = off;
}

}  // namespace mxk

extern "C" {

mxfft_status mxfft_plan(mxfft_plan_t* out, int32_t n, int32_t max_batch, const mxfft_params* p, void* stream)
{
    return plan_create(out, n, max_batch, p, stream, false, nullptr);
}

mxfft_status mxfft_plan_bytes(int32_t n, int32_t max_batch, const mxfft_params* p, uint64_t* bytes)
{
    if (!bytes) return MXFFT_EINVAL;
    mxfft_plan_t tmp = nullptr;
    *bytes = 0;
    return plan_create(&tmp, n, max_batch, p, nullptr, true, bytes);
}

mxfft_status mxfft_plan_destroy(mxfft_plan_t plan)
{
    if (!plan) return MXFFT_OK;
    (void)hipDeviceSynchronize();
    release(plan);
    return MXFFT_OK;
}

mxfft_status mxfft_forward(mxfft_plan_t pl, const void* in, void* out, int32_t batch, int32_t* k_out, void* stream)
{
    MX_TRY(check_call(pl, in, out, batch));
    if (batch == 0) return MXFFT_OK;
    return mxk::plan_forward_ws(pl, pl->ws, in, out, batch, k_out, stream);
}

}  // extern "C"

namespace mxk {

// The workspace as the passes after the first see it: they read the output
// buffer, so the output's offset table addresses their input too.
Workspace output_side(const Workspace& w)
{
    Workspace o = w;
    if (w.slice_off_out) o.slice_off = w.slice_off_out;
    return o;
}

// MXFFT_QUANTIZE_OUTPUT (MX formats): the finished output MX-encoded in place.
mxfft_status quantize_output(const mxfft_plan_s* pl, const Workspace& w, void* out, int batch, hipStream_t s)
{
    if (!(pl->p.flags & MXFFT_QUANTIZE_OUTPUT) || !is_mx_mode(pl->mode)) return MXFFT_OK;
    const unsigned long long* off = w.slice_off_out ? w.slice_off_out : w.slice_off;
    return launch_quantize_out(pl->mode, (float2*)out, off, pl->n, pl->logcb, batch, s) == hipSuccess ? MXFFT_OK
                                                                                                     : MXFFT_EHIP;
}

mxfft_status plan_forward_ws(mxfft_plan_s* pl, const Workspace& w, const void* in, void* out, int32_t batch,
                             int32_t* k_out, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    const bool pre = !(pl->p.flags & MXFFT_NO_PRESCALE);
    const int32_t* kp = pre ? w.kp : nullptr;
    const int kout_mul = (pl->p.flags & MXFFT_KEEP_SCALE) ? 0 : -1;
    const bool cap = pl->d_cap_mant != nullptr && batch <= pl->max_batch;   // capture buffers hold max_batch
    const Workspace wo = output_side(w);
    if (pl->single) {
        MX_TRY(small(pl, w, in, out, 0, pre, nullptr, k_out, 1, kout_mul, 0, cap, batch, s));
    } else if (pre && fused_stats(pl)) {
        MX_TRY(row_with_stats(pl, w, in, k_out, 0, batch, s));
        MX_TRY(pass(pl, wo, out, out, kp, nullptr, 0, kout_mul, 0, 1, 0, batch, s, mxk::ROW_PLAIN, w.kadd));
    } else {
        if (pre) MX_TRY(stats(pl, w, in, batch, s));
        MX_TRY(pass(pl, w, in, out, kp, k_out, 1, 0, 0, 0, 0, batch, s, mxk::ROW_PLAIN, nullptr, nullptr, 0, cap));
        MX_TRY(pass(pl, wo, out, out, kp, nullptr, 0, kout_mul, 0, 1, 0, batch, s, mxk::ROW_PLAIN, nullptr, nullptr,
                    0, cap));
    }
    MX_TRY(quantize_output(pl, w, out, batch, s));
    if (cap && pl->fast && !pl->single) {
        // the register-resident intermediate holds the column pass input
        if (mxk::launch_capture_mx(pl->mode, pl->n, pl->cb, w.codes, w.exps, (pre && fused_stats(pl)) ? w.kadd : nullptr,
                                   batch, pl->d_cap_mant, pl->d_cap_exp, s) != hipSuccess)
            return MXFFT_EHIP;
    }
    if (cap) {
        pl->cap_batch = batch;
        pl->cap_trace_ok = pl->single || !pl->fast;
    }
    pl->last_batch = batch;
    pl->last_has_stats = pre;
    pl->last_status = w.status;
    return MXFFT_OK;
}

}  // namespace mxk

extern "C" {

mxfft_status mxfft_inverse(mxfft_plan_t pl, const void* in, void* out, int32_t batch, const int32_t* k_in,
                           void* stream)
{
    MX_TRY(check_call(pl, in, out, batch));
    if (batch == 0) return MXFFT_OK;
    return mxk::plan_inverse_ws(pl, pl->ws, in, out, batch, k_in, stream);
}

mxfft_status mxfft_roundtrip(mxfft_plan_t pl, const void* in, void* out, int32_t batch, int32_t* k_out,
                             void* stream)
{
    MX_TRY(check_call(pl, in, out, batch));
    if (batch == 0) return MXFFT_OK;
    return mxk::plan_roundtrip_ws(pl, pl->ws, in, out, batch, k_out, stream);
}

}  // extern "C"

namespace mxk {

mxfft_status plan_inverse_ws(mxfft_plan_s* pl, const Workspace& w, const void* in, void* out, int32_t batch,
                             const int32_t* k_in, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    const int kout_add = (pl->p.flags & MXFFT_NORMALIZE) ? -2 * pl->logn : 0;
    bool pre = false;
    const int32_t* kp = k_in;
    int kin_mul = 0;
    if (!k_in && !(pl->p.flags & MXFFT_NO_PRESCALE)) {
        pre = true;
        kp = w.kp;
        kin_mul = 1;
    }
    const Workspace wo = output_side(w);
    if (pl->single) {
        MX_TRY(small(pl, w, in, out, 1, pre, pre ? nullptr : k_in, nullptr, kin_mul, -1, kout_add, false, batch, s));
    } else if (pre && fused_stats(pl)) {
        MX_TRY(row_with_stats(pl, w, in, nullptr, 1, batch, s));
        MX_TRY(pass(pl, wo, out, out, kp, nullptr, 0, -1, kout_add, 1, 1, batch, s, mxk::ROW_PLAIN, w.kadd));
    } else {
        if (pre) MX_TRY(stats(pl, w, in, batch, s));
        MX_TRY(pass(pl, w, in, out, kp, nullptr, kin_mul, 0, 0, 0, 1, batch, s));
        MX_TRY(pass(pl, wo, out, out, kp, nullptr, 0, -1, kout_add, 1, 1, batch, s));
    }
    MX_TRY(quantize_output(pl, w, out, batch, s));
    pl->last_batch = batch;
    pl->last_has_stats = pre;
    pl->last_status = w.status;
    return MXFFT_OK;
}

mxfft_status plan_roundtrip_ws(mxfft_plan_s* pl, const Workspace& w, const void* in, void* out, int32_t batch,
                               int32_t* k_out, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    const bool pre = !(pl->p.flags & MXFFT_NO_PRESCALE);
    const int32_t* kp = pre ? w.kp : nullptr;
    const Workspace wo = output_side(w);
    if (pl->single) {
        MX_TRY(small(pl, w, in, out, 2, pre, nullptr, k_out, 1, -1, -2 * pl->logn, false, batch, s));
    } else {
        if (pre && fused_stats(pl)) {
            MX_TRY(row_with_stats(pl, w, in, k_out, 0, batch, s));
            MX_TRY(pass(pl, wo, out, out, kp, nullptr, 0, 0, 0, 1, 0, batch, s, mxk::ROW_PLAIN, w.kadd));
        } else {
            if (pre) MX_TRY(stats(pl, w, in, batch, s));
            MX_TRY(pass(pl, w, in, out, kp, k_out, 1, 0, 0, 0, 0, batch, s));
            MX_TRY(pass(pl, wo, out, out, kp, nullptr, 0, 0, 0, 1, 0, batch, s));
        }
        MX_TRY(pass(pl, wo, out, out, kp, nullptr, 0, 0, 0, 0, 1, batch, s, inverse_row_kind(pl)));
        MX_TRY(pass(pl, wo, out, out, kp, nullptr, 0, -1, -2 * pl->logn, 1, 1, batch, s));
    }
    MX_TRY(quantize_output(pl, w, out, batch, s));
    pl->last_batch = batch;
    pl->last_has_stats = pre;
    pl->last_status = w.status;
    return MXFFT_OK;
}

}  // namespace mxk

extern "C" {

mxfft_status mxfft_rss(mxfft_plan_t pl, int32_t op, const void* in, void* work, float* rss, int32_t recon,
                       int32_t coils, int32_t* k_out, void* stream)
{
    if (!pl || !in || !rss || recon < 0 || coils < 1 || (op != 0 && op != 2)) return MXFFT_EINVAL;
    if ((pl->p.flags & MXFFT_QUANTIZE_OUTPUT) && mxk::is_mx_mode(pl->mode)) return MXFFT_EUNSUPPORTED;
    if ((long)recon * coils > pl->max_batch) return MXFFT_EINVAL;
    // the FP32 form keeps its intermediate in complex64 (the row pass writes
    // it where the column pass reads it): `work` is that buffer
    const bool plain = pl->mode == mxk::MODE_FP32;
    if ((op == 2 || plain || !pl->fast) && !work) return MXFFT_EINVAL;
    if (recon == 0) return MXFFT_OK;
    const mxk::Workspace& w = pl->ws;
    hipStream_t s = (hipStream_t)stream;
    const int batch = recon * coils;
    if (!pl->fast) {
        // no fused epilogue on the generic line kernels: the per-coil results
        // go to `work`, then the combine
        MX_TRY(op == 0 ? mxfft_forward(pl, in, work, batch, k_out, stream)
                       : mxfft_roundtrip(pl, in, work, batch, k_out, stream));
        return mxk::launch_rss((const float2*)work, coils, (size_t)pl->n * pl->n, recon, rss, s) == hipSuccess
                   ? MXFFT_OK
                   : MXFFT_EHIP;
    }
    const bool pre = !(pl->p.flags & MXFFT_NO_PRESCALE);
    const int32_t* kp = pre ? w.kp : nullptr;
    if (op == 0) {
        const int kout_mul = (pl->p.flags & MXFFT_KEEP_SCALE) ? 0 : -1;
        if (pre && fused_stats(pl)) {
            MX_TRY(row_with_stats(pl, w, in, k_out, 0, batch, s));
            MX_TRY(pass(pl, w, work, nullptr, kp, nullptr, 0, kout_mul, 0, 1, 0, recon, s, mxk::COL_RSS, w.kadd,
                        rss, coils));
        } else {
            if (pre) MX_TRY(stats(pl, w, in, batch, s));
            MX_TRY(pass(pl, w, in, work, kp, k_out, 1, 0, 0, 0, 0, batch, s));
            MX_TRY(pass(pl, w, work, nullptr, kp, nullptr, 0, kout_mul, 0, 1, 0, recon, s, mxk::COL_RSS, nullptr, rss,
                        coils));
        }
    } else {
        // round trip: the forward result (kept scaled) goes to `work`
        if (pre && fused_stats(pl)) {
            MX_TRY(row_with_stats(pl, w, in, k_out, 0, batch, s));
            MX_TRY(pass(pl, w, work, work, kp, nullptr, 0, 0, 0, 1, 0, batch, s, mxk::ROW_PLAIN, w.kadd));
        } else {
            if (pre) MX_TRY(stats(pl, w, in, batch, s));
            MX_TRY(pass(pl, w, in, work, kp, k_out, 1, 0, 0, 0, 0, batch, s));
            MX_TRY(pass(pl, w, work, work, kp, nullptr, 0, 0, 0, 1, 0, batch, s));
        }
        MX_TRY(pass(pl, w, work, work, kp, nullptr, 0, 0, 0, 0, 1, batch, s, inverse_row_kind(pl)));
        MX_TRY(pass(pl, w, work, nullptr, kp, nullptr, 0, -1, -2 * pl->logn, 1, 1, recon, s, mxk::COL_RSS, nullptr, rss,
                    coils));
    }
    pl->last_batch = batch;
    pl->last_has_stats = pre;
    pl->last_status = w.status;
    return MXFFT_OK;
}

mxfft_status mxfft_ssim(const float* x, const float* ref, int32_t n, int32_t count, double* ssim, void* stream)
{
    if (!x || !ref || !ssim || n < 11 || n > (1 << mxk::kMaxLog2N) || count < 0 || count > 65535)
        return MXFFT_EINVAL;
    if (count == 0) return MXFFT_OK;
    return mxk::launch_ssim(x, ref, n, count, ssim, (hipStream_t)stream) == hipSuccess ? MXFFT_OK : MXFFT_EHIP;
}

mxfft_status mxfft_plan_capture(mxfft_plan_t pl, void* mant, int32_t* exps, int32_t* trace, int32_t batch,
                                void* stream)
{
    if (!pl || !mant || !exps || !pl->d_cap_mant || batch < 1 || batch > pl->cap_batch) return MXFFT_EINVAL;
    if (trace && !pl->cap_trace_ok) return MXFFT_EUNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    const size_t nn = (size_t)pl->n * pl->n, b = (size_t)batch;
    if (hipMemcpyAsync(mant, pl->d_cap_mant, b * nn * sizeof(float2), hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(exps, pl->d_cap_exp, b * pl->n * (pl->n / pl->cb) * sizeof(int32_t), hipMemcpyDeviceToDevice,
                       s) != hipSuccess)
        return MXFFT_EHIP;
    if (trace && hipMemcpyAsync(trace, pl->d_cap_trace, b * pl->logn * (pl->n / (2 * pl->cb)) * 3 * sizeof(int32_t),
                                hipMemcpyDeviceToDevice, s) != hipSuccess)
        return MXFFT_EHIP;
    return MXFFT_OK;
}

mxfft_status mxfft_plan_last_status(mxfft_plan_t pl, void* stream)
{
    if (!pl) return MXFFT_EINVAL;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return MXFFT_EHIP;
    if (!pl->last_has_stats || pl->last_batch == 0) return MXFFT_OK;
    std::vector<int32_t> st(pl->last_batch);
    if (!pl->last_status ||
        hipMemcpy(st.data(), pl->last_status, st.size() * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
        return MXFFT_EHIP;
    for (int32_t v : st)
        if (v != 0) return (mxfft_status)v;
    return MXFFT_OK;
}

mxfft_status mxfft_plan_profile_roles(mxfft_plan_t pl, uint32_t role_mask)
{
    if (!pl) return MXFFT_EINVAL;
    if (hipDeviceSynchronize() != hipSuccess) return MXFFT_EHIP;
    collect_times(pl);
    role_mask &= (1u << ROLE_COUNT) - 1u;
    if (role_mask) {
        for (int r = 0; r < ROLE_COUNT; r++) {
            pl->launches[r] = 0;
            pl->total_ms[r] = 0.0;
        }
    }
    pl->profiling = role_mask != 0;
    pl->profile_mask = role_mask;
    return MXFFT_OK;
}

mxfft_status mxfft_plan_profile(mxfft_plan_t pl, int32_t enable)
{
    return mxfft_plan_profile_roles(pl, enable ? ~0u : 0u);
}

mxfft_status mxfft_plan_kernel_times(mxfft_plan_t pl, mxfft_kernel_time* out, int32_t cap, int32_t* count)
{
    if (!pl || !count || (cap > 0 && !out)) return MXFFT_EINVAL;
    if (hipDeviceSynchronize() != hipSuccess) return MXFFT_EHIP;
    collect_times(pl);
    int n = 0;
    for (int r = 0; r < ROLE_COUNT; r++) {
        if (!pl->launches[r]) continue;
        if (n < cap) {
            std::memset(out[n].name, 0, sizeof(out[n].name));
            std::strncpy(out[n].name, kRoleNames[r], sizeof(out[n].name) - 1);
            out[n].launches = pl->launches[r];
            out[n].total_ms = pl->total_ms[r];
        }
        n++;
    }
    *count = n;
    return MXFFT_OK;
}

uint64_t mxfft_plan_device_bytes(mxfft_plan_t pl) { return pl ? pl->bytes : 0; }

mxfft_status mxfft_plan_set_tuning(mxfft_plan_t pl, const mxfft_tuning* t)
{
    if (!pl || !t) return MXFFT_EINVAL;
    const int r = t->lines;
    if (r != 0 && (r < 1 || r > pl->n || (r & (r - 1)) != 0 || (long)r * pl->n * 8 > 65536)) return MXFFT_EINVAL;
    if (t->single != 0 && (t->single != 1 || pl->n > mxk::kSmallN)) return MXFFT_EINVAL;
    if (t->stats != 0 && t->stats != 1) return MXFFT_EINVAL;
    const long nn = (long)pl->n * pl->n;
    if (t->chunks != 0 && (t->chunks < 1 || (t->chunks & (t->chunks - 1)) != 0 || nn / t->chunks < 1024))
        return MXFFT_EINVAL;
    pl->lines = r;
    pl->single = t->single == 1;
    pl->literal_stats = t->stats == 1;
    pl->chunks = t->chunks;
    return MXFFT_OK;
}

mxfft_status mxfft_plan_get_tuning(mxfft_plan_t pl, mxfft_tuning* t)
{
    if (!pl || !t) return MXFFT_EINVAL;
    t->lines = pl->fast ? 0 : (pl->lines ? pl->lines : mxk::line_lines_per_group(pl->n));
    t->fast = pl->fast ? 1 : 0;
    t->ms = 0.0;
    t->single = pl->single ? 1 : 0;
    t->stats = (pl->fused && !pl->literal_stats) ? 0 : 1;
    t->chunks = pl->chunks;
    return MXFFT_OK;
}

const char* mxfft_status_string(mxfft_status st)
{
    switch (st) {
    case MXFFT_OK: return "ok";
    case MXFFT_EINVAL: return "invalid argument";
    case MXFFT_ENOMEM: return "device allocation failed";
    case MXFFT_EHIP: return "HIP runtime error";
    case MXFFT_ENONFINITE: return "non-finite input";
    case MXFFT_ERANGE: return "prescale overflows FP32";
    case MXFFT_EBUDGET: return "over memory budget";
    case MXFFT_EBUSY: return "busy";
    case MXFFT_EUNSUPPORTED: return "unsupported configuration";
    }
    return "unknown status";
}

int32_t mxfft_version(void) { return 100; }

}  // extern "C"
