// mxfft_fast.hpp -- register-resident row and column passes for 512 x 512 slices.
//
// Each lane holds 32 complex values of one 512-point line; 16 lanes (one DPP
// row) hold a line, a wave holds 4 lines and a work-group of 4 waves 16 lines.
// A "layout" names which 5 of the 9 position bits (bit-reversed order) sit in a
// lane.  Layout 0 holds bits 0..4 and runs stages 1..5 in registers; every later
// layout holds bits 0..C-1 (the low bits of an MX block of 2^C butterflies)
// plus the next 5-C unprocessed bits, so every MX block of every stage lies in
// one lane and its shared exponent is an in-register reduction.  Layouts change
// through a per-wave LDS exchange (re and im planes in turn, XOR-swizzled).
//
// MX arithmetic uses the gfx950 FP8/BF8 conversions with an E8M0-style scale:
// encode x / 2^E with round-to-nearest-even (saturation by a prior v_med3
// clamp, since the scaled conversion does not saturate) and decode codes
// times 2^E exactly.  These were checked bit for bit against integer rounding
// over all FP32 inputs of the relevant ranges.
//
// Row pass (MX):   load -> MX-encode blocks of 2^C consecutive values ->
//                  bit reversal -> 9 stages -> MX-encode each column over the
//                  work-group's 16 rows -> FP8 codes + E8M0 exponents.
// Column pass (MX): codes -> decode (this is the column input encode) -> bit
//                  reversal -> 9 stages -> 2^kout -> complex64.
// The FP32 plain form uses the same skeleton without quantisation and keeps
// an FP32 intermediate.  The FP16 and BF16 forms use it with every pass input,
// v operand, product and product sum rounded to the format (packed half
// arithmetic for FP16, FP32 products and packed conversions for BF16) and a
// 16-bit intermediate: the column pass input is the row pass output rounded
// to the format, so storing it rounded loses nothing.
//
// The header is included once per slice size: the including file defines
// MXF_LOGN (8, 9 or 10) and MXF_NS (the namespace of that size's kernels).
// The size-independent part (element arithmetic, kernel arguments) is
// compiled once per translation unit.

#ifndef MXFFT_FAST_COMMON_HPP
#define MXFFT_FAST_COMMON_HPP


#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "mx_device.hpp"
#include "mxfft_internal.hpp"
namespace mxf {

using mxd::short2v;
using mxd::float2v;
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf162v __attribute__((ext_vector_type(2)));

constexpr int FP16 = 2;          // format ids of the plain forms (mxk::MODE_FP16,
constexpr int BF16 = 3;          // mxk::MODE_BF16, mxk::MODE_FP32); 0 and 1 are
constexpr int FP32 = 4;          // the MXFP8 element formats E4M3 and E5M2, 5 and 6
constexpr int E2M3 = 5;          // the MXFP6 ones E2M3 and E3M2
constexpr int E3M2 = 6;
constexpr bool is_mx(int F) { return F < FP16 || F == E2M3 || F == E3M2; }
constexpr bool is_16(int F) { return F == FP16 || F == BF16; }

// ---------------------------------------------------------------------------
// compile-time helpers
// ---------------------------------------------------------------------------

template <int... Is, class Fn>
__device__ __forceinline__ void sfor_impl(std::integer_sequence<int, Is...>, Fn&& fn)
{
    (fn(std::integral_constant<int, Is>{}), ...);
}
// fn(integral_constant<int, i>) for i = 0 .. Nn-1, fully unrolled
template <int Nn, class Fn>
__device__ __forceinline__ void sfor(Fn&& fn)
{
    sfor_impl(std::make_integer_sequence<int, Nn>{}, fn);
}

constexpr int deposit(int v, int mask)
{
    int r = 0, k = 0;
    for (int b = 0; b < 31; b++)
        if ((mask >> b) & 1) {
            if ((v >> k) & 1) r |= 1 << b;
            k++;
        }
    return r;
}

constexpr int rev(int v, int bits)
{
    int r = 0;
    for (int b = 0; b < bits; b++) r |= ((v >> b) & 1) << (bits - 1 - b);
    return r;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// MX element conversions (gfx950)
// ---------------------------------------------------------------------------

// gfx950 element conversions and block scales: shared with the line kernels
// (mx_device.hpp)
using mxd::e8;
using mxd::Hw;
using mxd::maxv_frac;
using mxd::lim_of;
using mxd::Blk;
using mxd::blk;
using mxd::mulp;
using mxd::mulp1;
using mxd::unit_scale;
using mxd::enc2;
using mxd::dec2;
using mxd::clamp2;

// max(a, |v.x|, |v.y|) for a >= 0 in one v_max3_f32 (abs source modifiers)
__device__ __forceinline__ float amax2(float a, float2 v)
{
    float r;
    asm("v_max3_f32 %0, %1, |%2|, |%3|" : "=v"(r) : "v"(a), "v"(v.x), "v"(v.y));
    return r;
}

// largest |component| of CNT complex values: chains of v_max3_f32, four per
// asm statement (the compiler separates asm statements with wait states).
// SEED: the first three parts start the chain, one instruction fewer than
// from a zero register (which can cost registers where they are scarce)
template <int CNT, bool SEED = true>
__device__ __forceinline__ float amax_of(const float2* v)
{
    float a = 0.f;
    if constexpr (CNT % 4 == 0 && !SEED) {
#pragma unroll
        for (int g = 0; g < CNT / 4; g++) {
            const float2 p = v[4 * g], q = v[4 * g + 1], r = v[4 * g + 2], t = v[4 * g + 3];
            asm("v_max3_f32 %0, %0, |%1|, |%2|\n\t"
                "v_max3_f32 %0, %0, |%3|, |%4|\n\t"
                "v_max3_f32 %0, %0, |%5|, |%6|\n\t"
                "v_max3_f32 %0, %0, |%7|, |%8|"
                : "+v"(a)
                : "v"(p.x), "v"(p.y), "v"(q.x), "v"(q.y), "v"(r.x), "v"(r.y), "v"(t.x), "v"(t.y));
        }
    } else if constexpr (CNT % 4 == 0) {
        // the first three parts seed the chain (no zero register)
        asm("v_max3_f32 %0, |%1|, |%2|, |%3|" : "=v"(a) : "v"(v[0].x), "v"(v[0].y), "v"(v[1].x));
        asm("v_max3_f32 %0, %0, |%1|, |%2|\n\t"
            "v_max3_f32 %0, %0, |%3|, |%4|\n\t"
            "v_max_f32_e64 %0, %0, |%5|"
            : "+v"(a)
            : "v"(v[1].y), "v"(v[2].x), "v"(v[2].y), "v"(v[3].x), "v"(v[3].y));
#pragma unroll
        for (int g = 1; g < CNT / 4; g++) {
            const float2 p = v[4 * g], q = v[4 * g + 1], r = v[4 * g + 2], t = v[4 * g + 3];
            asm("v_max3_f32 %0, %0, |%1|, |%2|\n\t"
                "v_max3_f32 %0, %0, |%3|, |%4|\n\t"
                "v_max3_f32 %0, %0, |%5|, |%6|\n\t"
                "v_max3_f32 %0, %0, |%7|, |%8|"
                : "+v"(a)
                : "v"(p.x), "v"(p.y), "v"(q.x), "v"(q.y), "v"(r.x), "v"(r.y), "v"(t.x), "v"(t.y));
        }
    } else {
        sfor<CNT>([&](auto T) { a = amax2(a, v[T]); });
    }
    return a;
}

// Block exponent E, block scale and saturation bound MAXV * 2^E of a block
// whose largest magnitude has bits ab (mxd::block_exp, blk, lim_of).  For the
// 8-bit formats 2^E comes straight from the exponent field: E + 127 =
// max(field - EMAX, 0), which also gives E = -127 for a subnormal maximum; an
// all-zero block keeps E = 0.
struct BlkE {
    int E;
    Blk b;
    float lim;
};
template <int F>
__device__ __forceinline__ BlkE block_of(uint32_t ab)
{
    if constexpr (Hw<F>::OFF == 0) {
        constexpr uint32_t LIMADD = ((uint32_t)mxd::Elem<F>::EMAX << 23) | maxv_frac<F>();
        const uint32_t sb0 = __builtin_elementwise_sub_sat(ab & 0x7F800000u, (uint32_t)mxd::Elem<F>::EMAX << 23);
        const uint32_t sb = ab ? sb0 : 0x3F800000u;
        return BlkE{(int)(sb >> 23) - 127, Blk{__uint_as_float(sb), 1.0f, 1.0f}, __uint_as_float(sb + LIMADD)};
    } else {
        const int E = mxd::block_exp<F>(ab);
        const Blk b = blk<F>(E);
        return BlkE{E, b, mulp1<F>(lim_of<F>(E), b.pre)};
    }
}

// Codes of two complex values (each re, im) in the low and high halves of one
// register.  The first conversion's destination starts as the bits of its own
// first operand (dead afterwards), so no register needs clearing.
template <int F>
__device__ __forceinline__ uint32_t enc4(float2 v0, float2 v1, float scale)
{
    const uint32_t c = enc2<F, false>(__float_as_uint(v0.x), v0.x, v0.y, scale);
    return enc2<F, true>(c, v1.x, v1.y, scale);
}

// MX-encode a group of values sharing one block exponent, in place:
// v <- Q(v / 2^E) * 2^E with E from the group maximum am.  Returns E.
template <int F, int CNT>
__device__ __forceinline__ int mx_requant(float2* v, float& am)
{
    am = amax_of<CNT>(v);
    const int E = mxd::block_exp<F>(__float_as_uint(am));
    const Blk b = blk<F>(E);
    const float s = b.s, lim = mulp1<F>(lim_of<F>(E), b.pre);
    uint32_t c[CNT / 2];
    sfor<CNT / 2>([&](auto H) {
        c[H] = enc4<F>(clamp2(mulp<F>(v[2 * H], b.pre), lim), clamp2(mulp<F>(v[2 * H + 1], b.pre), lim), s);
    });
    sfor<CNT / 2>([&](auto H) {
        v[2 * H] = mulp<F>(dec2<F, false>(c[H], s), b.post);
        v[2 * H + 1] = mulp<F>(dec2<F, true>(c[H], s), b.post);
    });
    return E;
}

// Running range of the MX block exponents a pass uses (only tracked by the
// row pass that runs unscaled while it gathers the prescale statistics), and
// for BF16 whether some product fell below the FP32 normal range.
struct ERange {
    int lo = 0, hi = 0;
    bool sub = false;
    __device__ __forceinline__ void add(int e) { lo = min(lo, e); hi = max(hi, e); }
};

// max over the groups of G consecutive lanes (G = 1 .. 16, within a DPP row)
// of non-negative values given as bits, every lane receiving its group's
// value: quad_perm swaps of lanes 1 and 2 apart, then the half-row mirror
// (lane i <-> 7 - i), which after the first two steps meets the other quad of
// the 8, then the row mirror (lane i <-> 15 - i), which meets the other 8.
// Integer max: non-negative floats order like their bits.
template <int G>
__device__ __forceinline__ uint32_t group_max_bits(uint32_t v)
{
    static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16, "group of 1..16 lanes");
    if constexpr (G >= 2) v = max(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true));
    if constexpr (G >= 4) v = max(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true));
    if constexpr (G >= 8) v = max(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, true));
    if constexpr (G >= 16) v = max(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, true));
    return v;
}

// MX-encode a block of CB consecutive values held two per lane by CB / 2
// consecutive lanes (v0, v1 of this lane), in place.  Returns E; am is the
// block maximum.
template <int F, int CB>
__device__ __forceinline__ int mx_requant_pair(float2& v0, float2& v1, float& am)
{
    uint32_t a;
    asm("v_max3_f32 %0, |%1|, |%2|, |%3|\n\t"
        "v_max_f32_e64 %0, %0, |%4|"
        : "=&v"(a)
        : "v"(v0.x), "v"(v0.y), "v"(v1.x), "v"(v1.y));
    a = group_max_bits<CB / 2>(a);
    am = __uint_as_float(a);
    const BlkE q = block_of<F>(a);
    const int E = q.E;
    const Blk b = q.b;
    const float s = b.s, lim = q.lim;
    const uint32_t c = enc4<F>(clamp2(mulp<F>(v0, b.pre), lim), clamp2(mulp<F>(v1, b.pre), lim), s);
    v0 = mulp<F>(dec2<F, false>(c, s), b.post);
    v1 = mulp<F>(dec2<F, true>(c, s), b.post);
    return E;
}

// As mx_requant_pair for blocks of 4 G consecutive values held four per lane
// (v0..v3) by G consecutive lanes: lines of 4 lanes with blocks of 16.
template <int F, int G>
__device__ __forceinline__ int mx_requant_quad(float2& v0, float2& v1, float2& v2, float2& v3, float& am)
{
    uint32_t a;
    asm("v_max3_f32 %0, |%1|, |%2|, |%3|\n\t"
        "v_max3_f32 %0, %0, |%4|, |%5|\n\t"
        "v_max3_f32 %0, %0, |%6|, |%7|\n\t"
        "v_max_f32_e64 %0, %0, |%8|"
        : "=&v"(a)
        : "v"(v0.x), "v"(v0.y), "v"(v1.x), "v"(v1.y), "v"(v2.x), "v"(v2.y), "v"(v3.x), "v"(v3.y));
    a = group_max_bits<G>(a);
    am = __uint_as_float(a);
    const BlkE q = block_of<F>(a);
    const int E = q.E;
    const Blk b = q.b;
    const float s = b.s, lim = q.lim;
    const uint32_t c0 = enc4<F>(clamp2(mulp<F>(v0, b.pre), lim), clamp2(mulp<F>(v1, b.pre), lim), s);
    const uint32_t c1 = enc4<F>(clamp2(mulp<F>(v2, b.pre), lim), clamp2(mulp<F>(v3, b.pre), lim), s);
    v0 = mulp<F>(dec2<F, false>(c0, s), b.post);
    v1 = mulp<F>(dec2<F, true>(c0, s), b.post);
    v2 = mulp<F>(dec2<F, false>(c1, s), b.post);
    v3 = mulp<F>(dec2<F, true>(c1, s), b.post);
    return E;
}

struct Tw {
    const float2* tw;      // stage s = b+1, index j at [2^b + j]
    const int32_t* ex;     // twiddle block exponents
    const int32_t* off;    // per stage s: offset into ex
    const uint32_t* tw16;  // FP16 form: the same twiddles as packed halves
};

// ---------------------------------------------------------------------------
// FP16 / BF16 arithmetic
// ---------------------------------------------------------------------------

// (a, b) rounded to nearest even in the 16-bit format, packed (a low); one
// v_cvt_pk_f16_f32 / v_cvt_pk_bf16_f32 (overflow to infinity, NaN kept)
template <int F>
__device__ __forceinline__ uint32_t pack16(float a, float b)
{
    if constexpr (F == FP16) return __builtin_bit_cast(uint32_t, __builtin_convertvector((float2v){a, b}, half2v));
    else return __builtin_bit_cast(uint32_t, __builtin_convertvector((float2v){a, b}, bf162v));
}

// the two values of a packed pair as FP32 (exact)
template <int F>
__device__ __forceinline__ float2 unpack16(uint32_t w)
{
    if constexpr (F == FP16) {
        const half2v h = __builtin_bit_cast(half2v, w);
        return make_float2((float)h.x, (float)h.y);
    } else {
        return make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u));
    }
}

// FP16 complex product w v of packed halves: the four products and the two
// sums each round once to half (packed half multiplies and adds are correctly
// rounded; contraction into fused multiply-adds is off).  Three packed
// instructions; p = (wr vr - wi vi, wr vi + wi vr), wi negated for the inverse.
template <bool INV>
__device__ __forceinline__ float2 cmul_fp16(uint32_t wb, uint32_t vb)
{
#pragma clang fp contract(off)
    const half2v w = __builtin_bit_cast(half2v, wb), v = __builtin_bit_cast(half2v, vb);
    const half2v p1 = w.xx * v;                              // wr vr, wr vi
    const half2v p2 = (INV ? -w.yy : w.yy) * v.yx;           // wi vi, wi vr
    const half2v p = p1 + (half2v){-p2.x, p2.y};
    return make_float2((float)p.x, (float)p.y);
}

// BF16 product a b rounded to bfloat16 later by pack16: the FP32 product of
// two bfloat16 values (16 significant bits) is exact unless it is an FP32
// subnormal.  EX: such products are replaced by the exact value rounded to the
// bfloat16 subnormal grid 2^-133; else they are only flagged.  The exact
// rounding: both factors are then below 2^7 in magnitude (each is at least
// 2^-133), so q = (a 2^64) b is an exact normal FP32 value below 2^-62; adding
// and subtracting 1.5 * 2^-46 rounds it to the grid 2^-69 (nearest even), and
// 2^-64 scales back exactly.  The sign of a zero result is that of q.
template <bool EX>
__device__ __forceinline__ float mul_bf16(float a, float b, bool& sub)
{
#pragma clang fp contract(off)
    float p = a * b;
    const bool tiny = __builtin_isfpclass(p, 0x90);          // -subnormal | +subnormal
    if constexpr (EX) {
        const float q = (a * 0x1p64f) * b;
        const float r = __builtin_copysignf(((q + 0x1.8p-46f) - 0x1.8p-46f) * 0x1p-64f, q);
        if (tiny) p = r;
    } else {
        sub |= tiny;
    }
    return p;
}

// BF16 complex product w v (v packed bfloat16): products and sums each round
// once to bfloat16.  A sum of two bfloat16 values rounded to FP32 and then to
// bfloat16 equals its direct rounding (24 >= 2 * 8 + 2 bits).
template <bool INV, bool EX>
__device__ __forceinline__ float2 cmul_bf16(float2 w, uint32_t vb, bool& sub)
{
#pragma clang fp contract(off)
    const float2 v = unpack16<BF16>(vb);
    const float wi = INV ? -w.y : w.y;
    const uint32_t q1 = pack16<BF16>(mul_bf16<EX>(w.x, v.x, sub), mul_bf16<EX>(w.x, v.y, sub));   // wr vr, wr vi
    const uint32_t q2 = pack16<BF16>(mul_bf16<EX>(wi, v.y, sub), mul_bf16<EX>(wi, v.x, sub));     // wi vi, wi vr
    const float2 a = unpack16<BF16>(q1), b = unpack16<BF16>(q2);
    return unpack16<BF16>(pack16<BF16>(a.x - b.x, a.y + b.y));
}

// ---------------------------------------------------------------------------
// kernel arguments
// ---------------------------------------------------------------------------

struct FastArgs {
    const float2* src;       // complex64 [batch][N][N] (row pass input / column pass FP32 input)
    float2* dst;             // complex64 output (row pass FP32 form / column pass)
    uint32_t* codes;         // intermediate, [slice][16-column group][row][...]: MX, 8 words of 2 code
                             // pairs (swizzled); FP16/BF16, 16 words of one packed complex value
    uint8_t* exps;           // MX intermediate: [slice][row block][column] E8M0 bytes
    const int32_t* kp;       // per-slice prescale exponent or nullptr
    int32_t* k_out;          // per-slice copy of kp (row pass) or nullptr
    int32_t kin_mul, kout_mul, kout_add;
    const float2* tw;
    const int32_t* tw_exp;
    int32_t tw_off[16];
    mxk::StatPart* parts;    // row pass with statistics: [slice][tile]
    const int32_t* kadd;     // column pass: per-slice offset of the stored exponents, or nullptr
    const int32_t* fix_list; // list-driven row pass: slices to redo
    int32_t* fix_count;      // list length (zeroed by the row pass with statistics)
    const uint32_t* tw16;    // FP16 form: twiddles as packed halves, [2^b + j]
    float* rss;              // column pass with the coil combine: [reconstruction][N][N] FP32
    int32_t coils;           // coil slices per reconstruction (consecutive slices)
    const unsigned long long* slice_off;      // element offset of each slice in src, or nullptr
    const unsigned long long* slice_off_out;  // element offset of each slice in dst, or nullptr
};

using mxk::kStatsBins;
using mxk::StatPart;
using mxk::ROW_PLAIN;
using mxk::ROW_STATS;
using mxk::ROW_FIX;
using mxk::ROW_RAW;

__device__ __forceinline__ int slice_k(const FastArgs& g, int slice)
{
    int k = g.kp ? g.kp[slice] : 0;
    return k == INT32_MIN ? 0 : k;
}


template <class T>
__device__ __forceinline__ T wave_reduce_max(T v)
{
#pragma unroll
    for (int o = 32; o; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}
template <class T>
__device__ __forceinline__ T wave_reduce_min(T v)
{
#pragma unroll
    for (int o = 32; o; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

}  // namespace mxf

#endif  // MXFFT_FAST_COMMON_HPP

#if !defined(MXF_LOGN) || !defined(MXF_NS)
#error "define MXF_LOGN and MXF_NS before including mxfft_fast.hpp"
#endif

namespace MXF_NS {

using namespace mxf;

constexpr int LOGN = MXF_LOGN;
constexpr int N = 1 << LOGN;
constexpr int P = 32;               // complex values per lane
constexpr int LOG_LPL = LOGN - 5;
constexpr int LPL = N / P;          // lanes per line (16 at n = 512)
constexpr int LPW = 64 / LPL;       // lines per wave (4 at n = 512)
constexpr int LINES = 16;           // lines per work-group
constexpr int WAVES = LINES / LPW;  // waves per work-group (4 at n = 512)
constexpr int THREADS = 64 * WAVES;
// Waves per SIMD the register allocation of a kernel aims at (1: the
// compiler's own choice).  At 1024^2 the LDS of a 512-thread work-group lets
// two groups share a CU, four waves per SIMD; the kernels that take more
// than 128 VGPRs there would run two, and holding them to 128 (a few values
// go to scratch) measured 7 to 22 % faster.  At the smaller sizes the same
// limit takes three waves to four and measured slower.
constexpr int waves_target(bool over_128_vgprs) { return (LOGN == 10 && over_128_vgprs) ? 4 : 1; }
static_assert(LOGN >= 7 && LOGN <= 10, "register-resident passes for n = 128 .. 1024");

// Layouts for MX blocks of 2^C butterflies (1 <= C <= 4).
template <int C>
struct Lay {
    static constexpr int NEW = 5 - C;
    static constexpr int NL = 1 + (LOGN - 5 + NEW - 1) / NEW;
    // position bit held by in-lane offset bit i in layout k
    static constexpr int fbit(int k, int i)
    {
        if (k == 0 || i < C) return i;
        const int b = 5 + (k - 1) * NEW + (i - C);
        return b < LOGN ? b : C + (b - LOGN);
    }
    static constexpr int index_of(int k, int bit)
    {
        for (int i = 0; i < 5; i++)
            if (fbit(k, i) == bit) return i;
        return -1;
    }
    // q-th position bit fixed per lane (ascending), taken from lane bit q
    static constexpr int xbit(int k, int q)
    {
        int cnt = 0;
        for (int b = 0; b < LOGN; b++)
            if (index_of(k, b) < 0) {
                if (cnt == q) return b;
                cnt++;
            }
        return -1;
    }
    static constexpr int posF(int k, int o)
    {
        int p = 0;
        for (int i = 0; i < 5; i++)
            if ((o >> i) & 1) p |= 1 << fbit(k, i);
        return p;
    }
    static constexpr int bfirst(int k) { return k == 0 ? 0 : 5 + (k - 1) * NEW; }
    static constexpr int blast(int k)
    {
        const int e = (k == 0) ? 5 : 5 + k * NEW;
        return e < LOGN ? e : LOGN;
    }
};

template <int C, int K>
__device__ __forceinline__ int posM(int m)
{
    int p = 0;
    sfor<LOGN - 5>([&](auto Q) { p |= ((m >> Q) & 1) << Lay<C>::xbit(K, Q); });
    return p;
}

// LDS plane slot of position p of a line: 32-word rows (p >> 5) padded by a
// sum of per-bit amounts, slot(p) = p + 2 b5 + 4 b6 + 12 b7 + 18 b8 (b_j bit
// j of p).  The padding grows with the row index, so rows never overlap (548
// words per line), and it is additive: for p = c | m with disjoint in-lane
// bits c and lane bits m, slot(p) = slot(c) + slot(m), so every access is a
// per-lane base plus a compile-time offset, with no address arithmetic per
// access.  The amounts and the line bases (lines 584 words apart, odd pairs
// 16 words further) were chosen by enumeration against the LDS bank model of
// the target (64- and 128-bit accesses served by 32 banks of 8 bytes, 32-bit
// ones by 32 banks of 4 bytes): the layout exchanges of every block size reach
// 1.0-1.25 times the conflict-free cycle count (1.06 for blocks of 16
// butterflies).
__host__ __device__ constexpr int slot(int p)
{
    return p + 2 * ((p >> 5) & 1) + 4 * ((p >> 6) & 1) + 12 * ((p >> 7) & 1) + 18 * ((p >> 8) & 1) +
           36 * ((p >> 9) & 1);
}

constexpr int PLINE = slot(N - 1) + 1;    // words spanned by one line's slots (548 at n = 512)
// line stride: 8 words past a multiple of 32 (584 at n = 512)
constexpr int LSTRIDE = LOGN == 9 ? 584 : LOGN == 10 ? 1096 : LOGN == 8 ? 296 : 136;
static_assert(LSTRIDE >= PLINE && LSTRIDE % 32 == 8, "line stride");
// base of line l within its wave's planes
__host__ __device__ constexpr int line_base(int l) { return LSTRIDE * l + 16 * (l >> 1); }
constexpr int WPL = line_base(LPW - 1) + PLINE;   // words of one wave's planes (2316 at n = 512)

// pext: the bits of v at the set positions of MASK, packed from bit 0
template <int MASK>
__device__ __forceinline__ int pext(int v)
{
    int r = 0, q = 0;
    sfor<LOGN>([&](auto B) {
        if constexpr ((MASK >> B) & 1) { r |= ((v >> B) & 1) << q; q++; }
    });
    return r;
}

// position bits held by the lanes (not in-lane) in layout K
template <int C, int K>
constexpr int lane_mask()
{
    int mk = 0;
    for (int q = 0; q < LOGN - 5; q++) mk |= 1 << Lay<C>::xbit(K, q);
    return mk;
}

// Slot (in float2) of row r (0..N/2-1), column c (0..15) of an N/2 x 16 complex
// tile written by lanes whose rows differ in the bits LM (x are those
// bits of r): row bit 0 flips with x bit 0 (unless bit 0 is itself a lane
// bit) and column bits 2..3 XOR x bits 1..2, so one 64-bit store by a wave
// (4 columns x 16 rows) hits every 8-byte bank exactly twice, while a row of
// the tile stays one contiguous 128-byte run with column pairs kept adjacent.
template <int LM>
__device__ __forceinline__ int tslot(int r, int c)
{
    const int x = pext<LM>(r);
    const int R = (LM & 1) ? r : (r ^ (x & 1));
    return R * 16 + (c ^ (((x >> 1) & 3) << 2));
}

// Column slot in the [row][512] maximum and [block][512] scale arrays of the
// row pass: bits 2..5 XOR bits 4..7, so the 16 lanes of a line (16 different
// 4-column groups in every final layout) cover all banks.
__device__ __forceinline__ int csw(int c) { return c ^ (((c >> 4) & 15) << 2); }

// Word swizzle of the MX intermediate: in the 32-byte row segment of a
// 16-column group, the word of columns 2w, 2w+1 sits at w ^ cswz(row).  The
// column pass copies a group's 512 rows verbatim into LDS; its 32-bit reads
// (rows 16k + r for r = 0..15, two words per wave) then reach 32 distinct banks.
__device__ __forceinline__ int cswz(int row) { return ((row >> 2) & 3) << 1; }

// ---------------------------------------------------------------------------
// one radix-2 stage (butterfly position bit B) in layout K
// ---------------------------------------------------------------------------

// in-lane offsets of position bits 0..C-1 in layout K (offsets 0..C-1 except
// where a later layout wraps the low bits above the new stage bits)
template <int LC, int K, int C>
constexpr int block_offsets()
{
    int m = 0;
    for (int b = 0; b < C; b++) m |= 1 << Lay<LC>::index_of(K, b);
    return m;
}
// Block bits (of the BC bits enumerating a block's butterflies) held in-lane
// in layout K of family LC.  The first layout holds position bits 0..4: a
// block of 2^5 butterflies with its partner bit reaches position bit 5 there,
// so 4 of its bits are in-lane.  The later layouts hold a block's low position
// bits up to the first one that is a lane bit.
template <int LC, int K, int BC>
constexpr int block_bits_in_lane()
{
    if (K == 0) return BC < 4 ? BC : 4;
    int c = 0;
    while (c < BC && Lay<LC>::index_of(K, c) >= 0) c++;
    return c;
}

// LC: layout family (Lay<LC>); BC: log2 of butterflies per MX block.  A block
// whose bits are not all in-lane is split over 2 or 4 lanes: its remaining
// position bits are the lowest lane bits (lane bits 0 and 1, so DPP quad swaps
// reach the other lanes).  Each lane then works on its part of the block and
// the two block maxima (of v and of the products) are completed with one or
// two DPP exchanges (lanes m ^ 1, then m ^ 2): blocks of 16 butterflies in the
// later layouts of family 3 (a lane pair), blocks of 32 in its first layout
// (a lane pair) and in its later ones (four lanes, or a pair where the last
// layout wraps position bit 3 in-lane).
// EX (BF16): products below the FP32 normal range computed exactly.
template <int F, int LC, int BC, int K, int B, bool INV, bool TR, bool EX = false>
__device__ __forceinline__ void stage(float2 (&a)[P], int m, const Tw& t, ERange& er)
{
    using Ly = Lay<LC>;
    constexpr int C = block_bits_in_lane<LC, K, BC>();   // block bits held in-lane
    constexpr int NS = (K == 0) ? (BC > 4 ? 1 : 0) : BC - C;   // block bits held by lanes
    static_assert(NS <= 2, "a block spans at most four lanes");
    static_assert(NS < 1 || Ly::xbit(K, 0) == (K == 0 ? 5 : C), "next block bit in lane bit 0");
    static_assert(NS < 2 || Ly::xbit(K, 1) == C + 1, "last block bit in lane bit 1");
    static_assert(K > 0 || B < 5, "the first layout holds the stages of position bits 0..4");
    constexpr int ob = Ly::index_of(K, B);
    static_assert(ob >= 0, "butterfly bit must be in-lane");
    constexpr int h = 1 << B;
    constexpr int CB = 1 << C;                         // butterflies per (half-)block in a lane
    constexpr int fbb = (B > C) ? B : C;
    constexpr int obb = Ly::index_of(K, fbb);
    static_assert(obb >= 0, "block must be in-lane");
    constexpr int FREE = block_offsets<LC, K, C>() | (1 << obb);   // in-lane bits of one block
    constexpr int BFLY = FREE & ~(1 << ob);            // bits enumerating its butterflies
    constexpr int OTHER = (P - 1) & ~FREE;             // bits enumerating blocks
    constexpr int NBLK = P / (2 * CB);
    const int jm = posM<LC, K>(m) & (h - 1);          // lane part of j
    // block maximum (bits of a non-negative float): across the lanes of a split block
    auto bmax = [&](float v) -> uint32_t {
        uint32_t u = __float_as_uint(v);
        if constexpr (NS >= 1) u = max(u, (uint32_t)__builtin_amdgcn_mov_dpp((int)u, 0xB1, 0xF, 0xF, true));
        if constexpr (NS >= 2) u = max(u, (uint32_t)__builtin_amdgcn_mov_dpp((int)u, 0x4E, 0xF, 0xF, true));
        return u;
    };

    sfor<NBLK>([&](auto BLK) {
        constexpr int base = deposit(BLK, OTHER);
        float2 U[CB], V[CB];
        sfor<CB>([&](auto T) {
            constexpr int ou = base | deposit(T, BFLY);
            U[T] = a[ou];
            V[T] = a[ou | (1 << ob)];
        });
        if constexpr (F == FP32) {
            sfor<CB>([&](auto T) {
                constexpr int ou = base | deposit(T, BFLY);
                constexpr int jc = Ly::posF(K, ou) & (h - 1);
                const float2 w = t.tw[h + (jm | jc)];
                const float wi = INV ? -w.y : w.y;
                const float pr = w.x * V[T].x - wi * V[T].y;
                const float pi = w.x * V[T].y + wi * V[T].x;
                a[ou] = make_float2(U[T].x + pr, U[T].y + pi);
                a[ou | (1 << ob)] = make_float2(U[T].x - pr, U[T].y - pi);
            });
        } else if constexpr (is_16(F)) {
            // v rounded to the format, the product in the format, u +/- p in FP32
            sfor<CB>([&](auto T) {
                constexpr int ou = base | deposit(T, BFLY);
                constexpr int jc = Ly::posF(K, ou) & (h - 1);
                const uint32_t vb = pack16<F>(V[T].x, V[T].y);
                float2 p;
                if constexpr (F == FP16) p = cmul_fp16<INV>(t.tw16[h + (jm | jc)], vb);
                else p = cmul_bf16<INV, EX>(t.tw[h + (jm | jc)], vb, er.sub);
                a[ou] = make_float2(U[T].x + p.x, U[T].y + p.y);
                a[ou | (1 << ob)] = make_float2(U[T].x - p.x, U[T].y - p.y);
            });
        } else if constexpr (B <= 1) {
            // stages 1 and 2: twiddles 1 and -i with exponent -EMAX; the product
            // is the MX-encoded v itself (renormalisation by exactly 2^EMAX)
            const BlkE qv = block_of<F>(bmax(amax_of<CB, !TR>(V)));
            const int Ev = qv.E;
            if constexpr (TR) er.add(Ev);
            const Blk bv = qv.b;
            const float s = bv.s, lim = qv.lim;
            uint32_t c[CB / 2];
            sfor<CB / 2>([&](auto H) {
                c[H] = enc4<F>(clamp2(mulp<F>(V[2 * H], bv.pre), lim), clamp2(mulp<F>(V[2 * H + 1], bv.pre), lim), s);
            });
            sfor<CB>([&](auto T) {
                constexpr int ou = base | deposit(T, BFLY);
                constexpr int jc = Ly::posF(K, ou) & (h - 1);
                float2 w = mulp<F>(dec2<F, (T & 1) == 1>(c[T / 2], s), bv.post);
                if constexpr (jc == 1) w = INV ? make_float2(-w.y, w.x) : make_float2(w.y, -w.x);
                a[ou] = make_float2(U[T].x + w.x, U[T].y + w.y);
                a[ou | (1 << ob)] = make_float2(U[T].x - w.x, U[T].y - w.y);
            });
        } else {
            constexpr int jc0 = Ly::posF(K, base) & (h - 1);
            const int Ew = t.ex[t.off[B + 1] + (((1 << BC) <= h) ? ((jm | jc0) >> BC) : 0)];
            // operand v: EncodeBlockMX, element values as FP32 mantissas
            const BlkE qv = block_of<F>(bmax(amax_of<CB, !TR>(V)));
            const int Ev = qv.E;
            if constexpr (TR) er.add(Ev);
            const Blk bv = qv.b;
            const float s = bv.s, lim = qv.lim;
            float2 Pp[CB];
            uint32_t cv[CB / 2];
            sfor<CB / 2>([&](auto H) {
                cv[H] = enc4<F>(clamp2(mulp<F>(V[2 * H], bv.pre), lim), clamp2(mulp<F>(V[2 * H + 1], bv.pre), lim), s);
            });
            sfor<CB>([&](auto T) {
                constexpr int ou = base | deposit(T, BFLY);
                constexpr int jc = Ly::posF(K, ou) & (h - 1);
                const float2 x = t.tw[h + (jm | jc)];
                const float2 y = dec2<F, (T & 1) == 1>(cv[T / 2], unit_scale<F>());
                const float xi = INV ? -x.y : x.y;
                // products of 8-bit (and 6-bit) elements are exact: one rounding per component
                Pp[T].x = x.x * y.x - xi * y.y;
                Pp[T].y = x.x * y.y + xi * y.x;
            });
            const int kr = mxd::renorm_exp<F>(bmax(amax_of<CB, !TR>(Pp)));
            constexpr int OFF = Hw<F>::OFF;
            const float sp = e8(kr + OFF);
            const int Eo = Ew + Ev + kr;
            // the product block's scale operand 2^(Eo + OFF) must be in range
            const bool in_range = (OFF == 0) ? (Eo >= -127) : (Eo + OFF >= -127 && Eo + OFF <= 127);
            if (__builtin_expect(in_range, 1)) {
                const float so = e8(Eo + OFF);
                uint32_t cp[CB / 2];
                sfor<CB / 2>([&](auto H) { cp[H] = enc4<F>(Pp[2 * H], Pp[2 * H + 1], sp); });
                sfor<CB>([&](auto T) {
                    constexpr int ou = base | deposit(T, BFLY);
                    const float2 w = dec2<F, (T & 1) == 1>(cp[T / 2], so);
                    a[ou] = make_float2(U[T].x + w.x, U[T].y + w.y);
                    a[ou | (1 << ob)] = make_float2(U[T].x - w.x, U[T].y - w.y);
                });
            } else {
                // product scale outside the E8M0 range: decode the elements and
                // apply 2^Eo with ldexp (correctly rounded, subnormals kept)
                sfor<CB>([&](auto T) {
                    constexpr int ou = base | deposit(T, BFLY);
                    const uint32_t c = enc2<F, false>(__float_as_uint(Pp[T].x), Pp[T].x, Pp[T].y, sp);
                    const float2 q = dec2<F, false>(c, unit_scale<F>());
                    const float2 w = make_float2(ldexpf(q.x, Eo), ldexpf(q.y, Eo));
                    a[ou] = make_float2(U[T].x + w.x, U[T].y + w.y);
                    a[ou | (1 << ob)] = make_float2(U[T].x - w.x, U[T].y - w.y);
                });
            }
        }
    });
}

// all stages of layout K
template <int F, int LC, int BC, int K, bool INV, bool TR, bool EX>
__device__ __forceinline__ void stages(float2 (&a)[P], int m, const Tw& t, ERange& er)
{
    constexpr int b0 = Lay<LC>::bfirst(K), b1 = Lay<LC>::blast(K);
    sfor<b1 - b0>([&](auto I) { stage<F, LC, BC, K, b0 + I, INV, TR, EX>(a, m, t, er); });
}

// Layout K -> K+1 through this line's LDS plane (re, then im); addresses are
// a per-lane base (the lane bits' slot) plus the in-lane bits' slot.
template <int C, int K>
__device__ __forceinline__ void exchange(float2 (&a)[P], int m, float* plane)
{
    using Ly = Lay<C>;
    float* w = plane + slot(posM<C, K>(m));
    const float* r = plane + slot(posM<C, K + 1>(m));
    sfor<2>([&](auto R) {
        wave_sync();
        sfor<P / 2>([&](auto I) {
            constexpr int o = 2 * I;
            const float2 v = R ? make_float2(a[o].y, a[o + 1].y) : make_float2(a[o].x, a[o + 1].x);
            *(float2*)&w[slot(Ly::posF(K, o))] = v;
        });
        wave_sync();
        sfor<P / 2>([&](auto I) {
            constexpr int o = 2 * I;
            const float2 v = *(const float2*)&r[slot(Ly::posF(K + 1, o))];
            if (R) { a[o].y = v.x; a[o + 1].y = v.y; }
            else { a[o].x = v.x; a[o + 1].x = v.y; }
        });
    });
}

// plane: this line's exchange plane (line_base within the wave's planes)
template <int F, int LC, int BC, bool INV, bool TR = false, bool EX = false>
__device__ __forceinline__ void all_stages(float2 (&a)[P], int m, const Tw& t, float* plane, ERange& er)
{
    using Ly = Lay<LC>;
    sfor<Ly::NL>([&](auto K) {
        if constexpr (K > 0) exchange<LC, K - 1>(a, m, plane);
        stages<F, LC, BC, K, INV, TR, EX>(a, m, t, er);
    });
}

// Layout family of a pass with blocks of 2^C butterflies: blocks of 16 and 32
// use the layouts of blocks of 8 (two layout exchanges instead of four or
// more) with each block split over a lane pair or four lanes.
template <int F, int C>
constexpr int layout_family() { return !is_mx(F) ? 1 : (C >= 4 ? 3 : C); }

// Blocks of 32 butterflies (B = 64): a column block holds 32 rows, so the
// row pass takes tiles of 32 lines (twice the waves and LDS of a work-group)
// to encode the column pass's input inside one work-group.
template <int F, int C>
constexpr bool wide_blocks() { return is_mx(F) && C == 5; }
template <int F, int C>
constexpr int row_lines() { return wide_blocks<F, C>() ? 2 * LINES : LINES; }
template <int F, int C>
constexpr int row_threads() { return 64 * (row_lines<F, C>() / LPW); }

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Shared memory of the row pass.
template <int F, int C, int KIND>
struct alignas(16) RowLds {
    static constexpr int RL = row_lines<F, C>();      // lines of a row tile
    static constexpr int RW = RL / LPW;                // waves of its work-group
    static constexpr int NSB = !is_mx(F) ? 1 : RL / (1 << C);   // column blocks (of CB rows) per tile
    // copies of the statistics histogram: as many as the planes hold, up to 32
    static constexpr int HC_FIT = RW * WPL / kStatsBins;
    static constexpr int HC = HC_FIT >= 32 ? 32 : HC_FIT >= 16 ? 16 : HC_FIT >= 8 ? 8 : 4;
    // exchange planes; before them the statistics histogram (row pass with
    // statistics only: HC copies, bin * HC + lane % HC, so only lanes HC
    // apart can meet on an address; bin kStatsBins - 1 collects zeros and
    // non-finite values); after them the column maxima
    float plane[RW * WPL];
    float sc[NSB * N];                 // column block scales 2^E (MX)
    double m2[RW];
    uint32_t mc[RW];
    int nf[RW], elo[RW], ehi[RW];
};

// One 16-row tile of the row pass. F: 0 E4M3, 1 E5M2, 2 FP16, 3 BF16, 4 FP32.
// C: log2 of complex values per MX block (1 for the plain forms).  KIND:
//   ROW_PLAIN  input scaled by 2^(kin_mul * kp) (kp per slice, may be absent)
//   ROW_STATS  input unscaled; also the Alg. 1 statistics of the tile (with the
//              range of the block exponents used) into parts[slice][tile]
//   ROW_FIX    input scaled by 2^kp: the literal pass for a listed slice
//   ROW_RAW    as ROW_PLAIN without the input MX encode (fused round trip)
template <int F, int C, bool INV, int KIND>
__device__ __forceinline__ void row_tile(const FastArgs& g, int slice, int rb, RowLds<F, C, KIND>& L)
{
    constexpr int CB = 1 << C;
    constexpr int NSB = RowLds<F, C, KIND>::NSB;
    constexpr bool ST = (KIND == ROW_STATS);
    static_assert(!ST || is_mx(F), "statistics ride on the MX row pass only");
    static_assert(KIND != ROW_RAW || is_mx(F), "the raw row pass is an MX variant");
    constexpr int RL = RowLds<F, C, KIND>::RL, RW = RowLds<F, C, KIND>::RW, RT = 64 * RW;
    float* s_plane = L.plane;
    float* s_sc = L.sc;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int line = lane >> LOG_LPL, m = lane & (LPL - 1);
    const int rl = wave * LPW + line;                     // row within the tile
    const int row = rb * RL + rl;
    const int kp = slice_k(g, slice);
    const int kin = ST ? 0 : g.kin_mul * kp;
    if (KIND == ROW_PLAIN && g.k_out && rb == 0 && tid == 0) g.k_out[slice] = g.kp ? g.kp[slice] : 0;
    const float2* x = g.src + mxd::slice_base(g.slice_off, slice, (size_t)N * N) + (size_t)row * N;
    float* plane = s_plane + wave * WPL + line_base(line);
    uint32_t* hist = (uint32_t*)s_plane;                 // statistics only, before the planes are used
    const int rm = (int)(__brev((unsigned)m) >> (32 - LOG_LPL));   // m bit-reversed
    Tw t{g.tw, g.tw_exp, g.tw_off, g.tw16};
    float2 a[P];
    ERange er;
    // plain forms: layout 0 directly, natural LPL k + rm -> offset rev5(k);
    // the 16-bit forms round the pass input to the format
    auto load_plain = [&]() {
        sfor<P>([&](auto Kk) {
            const float2 v = x[LPL * Kk + rm];
            float2 s = make_float2(ldexpf(v.x, kin), ldexpf(v.y, kin));
            if constexpr (is_16(F)) s = unpack16<F>(pack16<F>(s.x, s.y));
            a[rev(Kk, 5)] = s;
        });
    };

    if constexpr (!is_mx(F)) {
        load_plain();
    } else {
        // IN4: loads of 32 consecutive bytes per lane, lane m of a line holding
        // naturals 4 LPL I + 4 m + e (e = 0 .. 3) as v[4 I + e] (two 16-byte
        // loads whose pair covers whole cache lines), so a block's part in a
        // lane is four values.  Otherwise coalesced 16-byte loads, lane m
        // holding naturals 2 LPL I + 2 m + e (e = 0, 1) as v[2 I + e].  IN4
        // takes fewer instructions; the statistics passes at 1024^2 and of
        // blocks of 32 at 512^2 keep the second form, which the register
        // allocation fits better there (no spills, four waves per SIMD)
        constexpr bool IN4 = !(ST && ((LOGN == 10 && C <= 4) || (LOGN == 9 && C == 5)));
        float2 v[P];
        const float4* x4 = (const float4*)x;
        sfor<P / 2>([&](auto I) {
            const float4 q = IN4 ? x4[2 * (LPL * (I / 2) + m) + (I % 2)] : x4[LPL * I + m];
            if constexpr (ST) {
                v[2 * I] = make_float2(q.x, q.y);
                v[2 * I + 1] = make_float2(q.z, q.w);
            } else {
                v[2 * I] = make_float2(ldexpf(q.x, kin), ldexpf(q.y, kin));
                v[2 * I + 1] = make_float2(ldexpf(q.z, kin), ldexpf(q.w, kin));
            }
        });
        // statistics: bits of the largest block maximum (= largest |part|), of
        // the smallest nonzero one (minus one, so that zero wraps to the top),
        // and whether a block was all zero.  block_exp is monotone in the
        // maximum of a nonzero block and 0 for a zero block, so these give the
        // exponent range of the input blocks (tracking each E instead holds
        // about 20 more VGPRs over the stages)
        uint32_t mcb = 0, mnz1 = 0xFFFFFFFFu;
        bool zblk = false;
        auto track = [&](uint32_t ab) {
            mcb = max(mcb, ab);
            mnz1 = min(mnz1, ab - 1u);
            zblk |= ab == 0u;
        };
        if constexpr (ST) {
            // Alg. 1 statistics of the unscaled input: |x|^2 in FP64 (both squares
            // exact, one rounding), its maximum, and the binade histogram
            // floor(log2 |x|) = floor(floor(log2 |x|^2) / 2) (the square root is
            // monotone and correctly rounded).  The local histogram's bins are
            // one above the part's: from the high word of |x|^2 (biased exponent
            // e), the saturating (hi - 723 * 2^20) / 2^21 is 0 for zero, (e - 723) / 2
            // = floor(log2 |x|) + 150 for finite nonzero |x| (1 .. 278), and 662 for
            // Inf/NaN (e = 2047), clamped to the last bin, which so counts the
            // non-finite elements
            constexpr int HC = RowLds<F, C, KIND>::HC;
            static_assert(kStatsBins * HC <= RW * WPL && HC >= 4, "histogram copies fit the planes");
            for (int i = tid; i < kStatsBins * HC / 4; i += RT) ((uint4*)hist)[i] = make_uint4(0, 0, 0, 0);
            if (blockIdx.x == 0 && tid == 0) *g.fix_count = 0;
            __syncthreads();
            double m2max = 0.0;
            sfor<P>([&](auto I) {
                const double m2 = (double)v[I].x * (double)v[I].x + (double)v[I].y * (double)v[I].y;
                m2max = fmax(m2max, m2);
                const uint32_t hi = (uint32_t)((unsigned long long)__double_as_longlong(m2) >> 32);
                const uint32_t bin = min(__builtin_elementwise_sub_sat(hi, 723u << 20) >> 21, (uint32_t)(kStatsBins - 1));
                atomicAdd(&hist[bin * HC + (lane & (HC - 1))], 1u);
            });
            m2max = wave_reduce_max(m2max);
            if (lane == 0) L.m2[wave] = m2max;
        }
        // MX encode: a block of CB consecutive naturals sits in CB / 4
        // consecutive lanes, four values each (blocks of 2: two blocks per
        // four values), or without IN4 in CB / 2 consecutive lanes, or (lines of
        // 4 lanes, blocks of 16) in two loads of every lane; ROW_RAW leaves the
        // input as it is
        if constexpr (KIND == ROW_RAW) {
        } else if constexpr ((IN4 && CB == 2) || (!IN4 && CB / 2 <= LPL)) {
            sfor<P / 2>([&](auto I) {
                float am;
                const int E = mx_requant_pair<F, CB>(v[2 * I], v[2 * I + 1], am);
                if constexpr (ST) { (void)E; track(__float_as_uint(am)); }
            });
        } else {
            constexpr int G = IN4 ? CB / 4 : LPL;
            static_assert(IN4 ? CB / 4 <= LPL : CB == 4 * LPL, "a block spans at most the lanes of its line");
            sfor<P / 4>([&](auto H) {
                float am;
                const int E = mx_requant_quad<F, G>(v[4 * H], v[4 * H + 1], v[4 * H + 2], v[4 * H + 3], am);
                if constexpr (ST) { (void)E; track(__float_as_uint(am)); }
            });
        }
        if constexpr (ST) {
            if (mnz1 != 0xFFFFFFFFu) {
                er.add(mxd::block_exp<F>(mnz1 + 1u));
                er.add(mxd::block_exp<F>(mcb));
            }
            if (zblk) er.add(0);
            mcb = wave_reduce_max(mcb);
            if (lane == 0) L.mc[wave] = mcb;
            // the tile's histogram to its part (the planes are needed next): part
            // bin i sums the HC copies of local bin i + 1, four at a time, the
            // quads in the order q ^ (i + 1) so a wave's reads fall in different
            // banks (one address operation per read); the last local bin gives
            // the non-finite flag
            __syncthreads();
            constexpr int HC = RowLds<F, C, KIND>::HC, NQ = HC / 4;
            StatPart* pt = g.parts + (size_t)slice * (N / RL) + rb;
            for (int i = tid; i < kStatsBins; i += RT) {
                const int j = i + 1;
                uint32_t h = 0;
                if (j < kStatsBins) {
                    const uint32_t a0 = (uint32_t)(j * HC * 4) | ((uint32_t)(j & (NQ - 1)) << 4);
#pragma unroll
                    for (int q = 0; q < NQ; q++) {
                        const uint4 u = *(const uint4*)((const char*)hist + (a0 ^ ((uint32_t)q << 4)));
                        h += u.x + u.y + u.z + u.w;
                    }
                }
                if (j == kStatsBins - 1) {
                    L.nf[0] = h != 0;
                    h = 0;
                }
                pt->hist[i] = h;
            }
            __syncthreads();
        }
        // bit reversal into layout 0 through the LDS plane
        float* wb = plane + slot(rm << (IN4 ? 3 : 4));
        const float* rbp = plane + slot(P * m);
        sfor<2>([&](auto R) {
            wave_sync();
            // IN4: natural 4 LPL I + 4 m + e sits at position rev2(e) N/4 + rm 8 +
            // rev3(I); otherwise natural 2 LPL I + 2 m + e at e N/2 + rm 16 + rev4(I)
            sfor<P>([&](auto J) {
                constexpr int off = IN4 ? ((rev(J % 4, 2) << (LOGN - 2)) | rev(J / 4, 3))
                                        : (((J % 2) << (LOGN - 1)) | rev(J / 2, 4));
                wb[slot(off)] = R ? v[J].y : v[J].x;
            });
            wave_sync();
            sfor<P / 2>([&](auto I) {
                const float2 q = *(const float2*)&rbp[slot(2 * I)];
                if (R) { a[2 * I].y = q.x; a[2 * I + 1].y = q.y; }
                else { a[2 * I].x = q.x; a[2 * I + 1].x = q.y; }
            });
        });
    }

    constexpr int CL = layout_family<F, C>();
    all_stages<F, CL, (is_mx(F) ? C : 1), INV, ST>(a, m, t, plane, er);
    if constexpr (F == BF16) {
        // some product of this wave's lines fell below the FP32 normal range:
        // the wave redoes its lines with such products computed exactly
        if (__builtin_amdgcn_ballot_w64(er.sub) != 0) {
            load_plain();
            all_stages<F, CL, 1, INV, false, true>(a, m, t, plane, er);
        }
    }

    constexpr int KL = Lay<CL>::NL - 1;
    const int pmL = posM<CL, KL>(m);
    if constexpr (F == FP32) {
        float2* y = g.dst + mxd::slice_base(g.slice_off_out, slice, (size_t)N * N) + (size_t)row * N;
        sfor<P>([&](auto O) { y[Lay<CL>::posF(KL, O) | pmL] = a[O]; });
    } else if constexpr (is_16(F)) {
        // 16-bit intermediate [slice][16-column group][row][16 words]: in-lane
        // offset bit 0 is position bit 0, so a lane holds pairs of adjacent
        // columns (one 8-byte store each; a line's 8 lanes of one group write
        // the row's 64 bytes).  Packing rounds to the format.
        uint32_t* cd = g.codes + (size_t)slice * N * N;
        sfor<P / 2>([&](auto I) {
            constexpr int o = 2 * I;
            const int c = Lay<CL>::posF(KL, o) | pmL;
            *(uint2*)&cd[((size_t)(c >> 4) * N + row) * 16 + (c & 15)] =
                make_uint2(pack16<F>(a[o].x, a[o].y), pack16<F>(a[o + 1].x, a[o + 1].y));
        });
    } else {
        // Column MX encode of the next pass's input: blocks of CB consecutive
        // rows of one column; this work-group holds NSB such blocks.
        // 1. per-element max(|re|, |im|) into a [16][N] array (column-swizzled);
        //    VW consecutive columns per lane are in-lane offset bits 0..log2(VW)-1
        constexpr int VW = (CL >= 2) ? 4 : 2;
        float* s_m = s_plane;
        static_assert(RL * N <= RW * WPL, "column maxima fit the planes");
        __syncthreads();                                   // every wave is done with its planes
        sfor<P / VW>([&](auto G) {
            constexpr int o0 = deposit(G, (P - 1) & ~(VW - 1));
            const int c0 = Lay<CL>::posF(KL, o0) | pmL;
            float mv[VW];
            sfor<VW>([&](auto J) { mv[J] = fmaxf(fabsf(a[o0 + J].x), fabsf(a[o0 + J].y)); });
            float* d = &s_m[rl * N + csw(c0)];
            if constexpr (VW == 4) *(float4*)d = make_float4(mv[0], mv[1], mv[2], mv[3]);
            else *(float2*)d = make_float2(mv[0], mv[1]);
        });
        __syncthreads();
        // 2. one thread per column pair: block exponents -> E8M0 bytes (global,
        //    [slice][row block][column]) and scales 2^E (LDS); tiles of 32
        //    lines have twice the threads
        static_assert(RT >= N / 2, "a thread per column pair");
        if (2 * tid < N) {
            const int c2 = 2 * tid;
            uint8_t* ex = g.exps + (size_t)slice * (N / CB) * N + (size_t)rb * NSB * N;
            sfor<NSB>([&](auto B) {
                float m0 = 0.f, m1 = 0.f;
                sfor<CB>([&](auto Rr) {
                    const float2 v = *(const float2*)&s_m[(B * CB + Rr) * N + csw(c2)];
                    m0 = fmaxf(m0, v.x);
                    m1 = fmaxf(m1, v.y);
                });
                const int E0 = mxd::block_exp<F>(__float_as_uint(m0)), E1 = mxd::block_exp<F>(__float_as_uint(m1));
                if constexpr (ST) { er.add(E0); er.add(E1); }
                *(uint16_t*)&ex[B * N + c2] = (uint16_t)((E0 + 127) | ((E1 + 127) << 8));
                *(float2*)&s_sc[B * N + csw(c2)] = make_float2(e8(E0), e8(E1));
            });
        }
        __syncthreads();
        // 3. encode: clamp to MAXV * 2^E (bits of 2^E plus those of MAXV), scaled conversion
        constexpr uint32_t LIMADD = ((uint32_t)mxd::Elem<F>::EMAX << 23) | maxv_frac<F>();
        const float* my_sc = s_sc + (rl / CB) * N;
        uint32_t* cd = g.codes + ((size_t)slice * N * N) / 2;
        // in-lane column groups: CG consecutive columns (in-lane offset bits 0..CL-1)
        constexpr int CG = 1 << CL;
        sfor<P / CG>([&](auto G) {
            constexpr int o0 = deposit(G, (P - 1) & ~(CG - 1));
            const int col0 = Lay<CL>::posF(KL, o0) | pmL;      // first column of the group
            float sc[CG];
            sfor<CG / VW>([&](auto J) {
                const float* src = &my_sc[csw(col0 + VW * J)];
                if constexpr (VW == 4) {
                    const float4 q = *(const float4*)src;
                    sc[4 * J] = q.x; sc[4 * J + 1] = q.y; sc[4 * J + 2] = q.z; sc[4 * J + 3] = q.w;
                } else {
                    const float2 q = *(const float2*)src;
                    sc[2 * J] = q.x; sc[2 * J + 1] = q.y;
                }
            });
            uint32_t w[CG / 2];
            sfor<CG / 2>([&](auto H) {
                constexpr int oa = o0 + 2 * H, obx = oa + 1;
                const float sa = sc[2 * H], sb = sc[2 * H + 1];
                if constexpr (Hw<F>::OFF == 0) {
                    const float la = __uint_as_float(__float_as_uint(sa) + LIMADD);
                    const float lb = __uint_as_float(__float_as_uint(sb) + LIMADD);
                    const float ra = __builtin_amdgcn_fmed3f(a[oa].x, -la, la);
                    uint32_t r = enc2<F, false>(__float_as_uint(ra), ra, __builtin_amdgcn_fmed3f(a[oa].y, -la, la), sa);
                    r = enc2<F, true>(r, __builtin_amdgcn_fmed3f(a[obx].x, -lb, lb),
                                      __builtin_amdgcn_fmed3f(a[obx].y, -lb, lb), sb);
                    w[H] = r;
                } else {
                    // MXFP6: scale operand 2^(E + OFF), or 2^E with the values
                    // times 2^-OFF when E + OFF is above the scale range
                    constexpr int OFF = Hw<F>::OFF;
                    auto prep = [&](float sc2, float& op, float& pre, float& lim) {
                        const uint32_t b = __float_as_uint(sc2);
                        const bool hi = b > ((uint32_t)(254 - OFF) << 23);
                        op = __uint_as_float(hi ? b : b + ((uint32_t)OFF << 23));
                        pre = hi ? e8(-OFF) : 1.0f;
                        lim = __uint_as_float(b + LIMADD) * pre;
                    };
                    float opa, pa, la, opb, pb, lb;
                    prep(sa, opa, pa, la);
                    prep(sb, opb, pb, lb);
                    const float ra = __builtin_amdgcn_fmed3f(a[oa].x * pa, -la, la);
                    uint32_t r = enc2<F, false>(__float_as_uint(ra), ra,
                                                __builtin_amdgcn_fmed3f(a[oa].y * pa, -la, la), opa);
                    r = enc2<F, true>(r, __builtin_amdgcn_fmed3f(a[obx].x * pb, -lb, lb),
                                      __builtin_amdgcn_fmed3f(a[obx].y * pb, -lb, lb), opb);
                    w[H] = r;
                }
            });
            // [16-column group][row][8 words], word of columns 2w, 2w+1 of the
            // group at position w ^ cswz(row)
            uint32_t* dstw = cd + ((size_t)(col0 / 16) * N + row) * 8;
            const int sw = cswz(row);
            if constexpr (CG >= 4) {
                sfor<CG / 4>([&](auto Q) {
                    const int q = ((col0 % 16) / 4 + Q) ^ (sw >> 1);
                    ((uint2*)dstw)[q] = make_uint2(w[2 * Q], w[2 * Q + 1]);
                });
            } else {
                dstw[((col0 % 16) / 2) ^ sw] = w[0];
            }
        });
        if constexpr (ST) {
            const int lo = wave_reduce_min(er.lo), hi = wave_reduce_max(er.hi);
            if (lane == 0) { L.elo[wave] = lo; L.ehi[wave] = hi; }
            __syncthreads();
            StatPart* pt = g.parts + (size_t)slice * (N / RL) + rb;
            if (tid == 0) {
                double m2 = L.m2[0];
                uint32_t mcw = L.mc[0];
                const int nf = L.nf[0];
                int elo = L.elo[0], ehi = L.ehi[0];
#pragma unroll
                for (int w = 1; w < RW; w++) {
                    m2 = fmax(m2, L.m2[w]);
                    mcw = max(mcw, L.mc[w]);
                    elo = min(elo, L.elo[w]);
                    ehi = max(ehi, L.ehi[w]);
                }
                pt->max_m2 = (unsigned long long)__double_as_longlong(m2);
                pt->count = 0;
                pt->max_comp = mcw;
                pt->nonfinite = (uint32_t)nf;
                pt->emin = elo;
                pt->emax = ehi;
            }
        }
    }
}

// Row pass over every tile of the batch (ROW_PLAIN, ROW_STATS).  Above 128
// VGPRs at 1024^2: the statistics form of blocks of 16 and 32, and BF16.
template <int F, int C, bool INV, int KIND>
__global__ __launch_bounds__((row_threads<F, C>()))
__attribute__((amdgpu_waves_per_eu(waves_target((KIND == ROW_STATS && C >= 3) || F == BF16), 8))) void k_row(FastArgs g)
{
    __shared__ RowLds<F, C, KIND> L;
    constexpr int TILES = N / row_lines<F, C>();
    row_tile<F, C, INV, KIND>(g, blockIdx.x / TILES, blockIdx.x % TILES, L);
}

// Row pass over the slices in fix_list only: the work-groups stride over the
// (list entry, tile) pairs, so a grid of a few slices' tiles serves any list
// length and an empty list costs one read per work-group.
template <int F, int C, bool INV>
__global__ __launch_bounds__((row_threads<F, C>())) void k_row_fix(FastArgs g)
{
    __shared__ RowLds<F, C, ROW_FIX> L;
    constexpr int TILES = N / row_lines<F, C>();
    const int total = *g.fix_count * TILES;            // the same for every thread
    for (int e = blockIdx.x; e < total; e += gridDim.x) {
        if (e != (int)blockIdx.x) __syncthreads();     // the previous tile is done with the LDS
        row_tile<F, C, INV, ROW_FIX>(g, g.fix_list[e / TILES], e % TILES, L);
    }
}

// Shared memory of the column pass: the exchange planes (which also hold the
// input and output tiles) and the exponent bytes of the MX input.
template <int F, int C>
struct alignas(16) ColLds {
    static constexpr int NRB = N / (1 << C);           // row blocks per column
    float plane[WAVES * WPL];
    uint8_t ex[!is_mx(F) ? 16 : LINES * NRB];          // [row block][16 columns]
};

// Column pass of the 16-column group cb16 of one slice up to its last stage:
// the input tile, its decode into the first layout, the stages (and, for
// BF16, the exact redo); a holds the unscaled results in the last layout.
// LOOP: called once per coil inside the combined pass's coil loop.
template <int F, int C, bool INV, bool LOOP = false>
__device__ __forceinline__ void col_lines(const FastArgs& g, int slice, int cb16, float2 (&a)[P], ColLds<F, C>& L)
{
    constexpr int CB = 1 << C;
    constexpr int NRB = ColLds<F, C>::NRB;
    float* s_plane = L.plane;
    uint8_t* s_ex = L.ex;
    // in the coil loop, an opaque copy of the thread index: the lane-dependent
    // addresses are then recomputed per coil instead of being hoisted out of
    // the loop (which would hold them all in registers)
    int tid = threadIdx.x;
    if constexpr (LOOP) asm volatile("" : "+v"(tid));
    const int wave = tid >> 6, lane = tid & 63;
    const int line = lane >> LOG_LPL, m = lane & (LPL - 1);
    const int cl = wave * LPW + line;                  // column within the work-group
    float* plane = s_plane + wave * WPL + line_base(line);
    const int rm = (int)(__brev((unsigned)m) >> (32 - LOG_LPL));   // m bit-reversed
    // in the coil loop, the table pointers plus an opaque zero: the twiddle
    // loads then stay inside the loop (all of them hoisted out of it would
    // need more registers than a lane has).  An offset rather than an opaque
    // pointer keeps the pointers' global address space known (global, not
    // flat, loads)
    size_t zo = 0;
    if constexpr (LOOP) asm volatile("" : "+s"(zo));
    const float2* twp = g.tw + zo;
    const int32_t* txp = g.tw_exp + zo;
    const uint32_t* t16p = g.tw16 + zo;
    Tw t{twp, txp, g.tw_off, t16p};
    float2* tile = (float2*)s_plane;                   // N/2 x 16 complex
    // 16-bit forms: this work-group's part of the intermediate, [row][16 words]
    const uint32_t* c16 = g.codes + (size_t)slice * N * N + (size_t)cb16 * LINES * N;

    if constexpr (F == FP32) {
        // rows are read whole (128 bytes = the work-group's 16 columns) into an
        // LDS tile, N/2 rows at a time; lanes then take rows (k << LOG_LPL) |
        // rev(m) (layout 0: offset rev5(k)), whose low bits are the lane bits
        static_assert(LOGN == 9, "the plain FP32 form is built for n = 512");
        static_assert(8 * THREADS == N / 2 * 8, "eight 16-byte pieces per thread and half");
        constexpr int LMR = (1 << LOG_LPL) - 1;
        const float2* xs = g.src + mxd::slice_base(g.slice_off, slice, (size_t)N * N) + cb16 * LINES;
        sfor<2>([&](auto H) {
            if constexpr (H == 1) __syncthreads();
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const int q = i * THREADS + tid, r = q >> 3, pr = q & 7;
                const float4 v = *(const float4*)&xs[(size_t)(H * (N / 2) + r) * N + 2 * pr];
                *(float4*)&tile[tslot<LMR>(r, 2 * pr)] = v;
            }
            __syncthreads();
            sfor<16>([&](auto Kl) {
                constexpr int Kk = H * 16 + Kl;
                a[rev(Kk, 5)] = tile[tslot<LMR>((Kl << LOG_LPL) | rm, cl)];
            });
        });
        __syncthreads();
    } else if constexpr (is_16(F)) {
        // the 512 rows of 64 bytes into LDS, the four 16-byte pieces of row n
        // rotated by XOR ((n >> 1) & 3): the 32-bit reads below (16 rows x 4
        // columns per wave) then reach every bank exactly twice
        uint32_t* ctile = (uint32_t*)s_plane;
        static_assert(LINES * N / 4 == 8 * THREADS, "eight 16-byte pieces per thread");
        const uint4* src = (const uint4*)c16;
        auto put = [&](int i, const uint4& v) {
            const int n = i >> 2;
            ((uint4*)ctile)[n * 4 + ((i & 3) ^ ((n >> 1) & 3))] = v;
        };
        sfor<2>([&](auto H) {   // four loads in flight, then their stores
            constexpr int J = 4 * H;
            const uint4 q0 = src[J * THREADS + tid], q1 = src[(J + 1) * THREADS + tid];
            const uint4 q2 = src[(J + 2) * THREADS + tid], q3 = src[(J + 3) * THREADS + tid];
            put(J * THREADS + tid, q0);
            put((J + 1) * THREADS + tid, q1);
            put((J + 2) * THREADS + tid, q2);
            put((J + 3) * THREADS + tid, q3);
        });
        __syncthreads();
        sfor<P>([&](auto O) {
            const int n = (rev(O, 5) << LOG_LPL) | rm;    // row of position 32m + O
            a[O] = unpack16<F>(ctile[n * 16 + (cl ^ (((n >> 1) & 3) << 2))]);
        });
        __syncthreads();
    } else {
        // code tile of the 16 columns ([row][8 words], swizzled by the row
        // pass): copied verbatim, 16 bytes per thread and step
        uint32_t* ctile = (uint32_t*)s_plane;
        const uint4* cd = (const uint4*)(g.codes + ((size_t)slice * N * N + (size_t)cb16 * LINES * N) / 2);
        static_assert(LINES * N / 8 == 4 * THREADS, "four 16-byte pieces per thread");
        const uint4 q0 = cd[tid], q1 = cd[THREADS + tid], q2 = cd[2 * THREADS + tid], q3 = cd[3 * THREADS + tid];
        // exponents [slice][row block][column]: 16 bytes per row block
        const uint8_t* ex = g.exps + (size_t)slice * NRB * N + cb16 * LINES;
        // stored exponents of a row pass that ran unscaled are offset by kadd
        const int eadd = g.kadd ? g.kadd[slice] : 0;
        // MXFP8: the tile's block scales 2^(E + kadd) as FP32 words [row block][16
        // columns], after the code tile in the planes, so a decode reads its
        // scale operand directly; MXFP6 keeps the bytes (its scale has two forms)
        float* s_scf = s_plane + LINES * N / 2;
        static_assert(LINES * N / 2 + NRB * 16 <= WAVES * WPL, "block scales fit after the code tile");
        if constexpr (Hw<F>::OFF == 0) {
            for (int i = tid; i < NRB * 4; i += THREADS) {
                const uint32_t w = *(const uint32_t*)&ex[(size_t)(i >> 2) * N + 4 * (i & 3)];
                *(float4*)&s_scf[4 * i] = make_float4(__uint_as_float((uint32_t)((int)(w & 0xffu) + eadd) << 23),
                                                      __uint_as_float((uint32_t)((int)((w >> 8) & 0xffu) + eadd) << 23),
                                                      __uint_as_float((uint32_t)((int)((w >> 16) & 0xffu) + eadd) << 23),
                                                      __uint_as_float((uint32_t)((int)(w >> 24) + eadd) << 23));
            }
        } else {
            for (int i = tid; i < NRB; i += THREADS) *(uint4*)&s_ex[i * 16] = *(const uint4*)&ex[(size_t)i * N];
        }
        ((uint4*)ctile)[tid] = q0;
        ((uint4*)ctile)[THREADS + tid] = q1;
        ((uint4*)ctile)[2 * THREADS + tid] = q2;
        ((uint4*)ctile)[3 * THREADS + tid] = q3;
        __syncthreads();
        // MXFP6: exponent bytes of this wave's 4 columns come as one dword per
        // row block (every lane of the wave reads the same dword: a broadcast;
        // byte reads of one dword by many lanes serialise)
        const uint32_t* s_ex4 = (const uint32_t*)s_ex + (cl >> 2);
        const int exsh = 8 * (cl & 3);
        const int cdsh = 16 * (cl & 1);                     // this column's code pair within the word
        const uint16_t* ctile16 = (const uint16_t*)ctile + (cl & 1);
        sfor<P>([&](auto O) {
            const int n = (rev(O, 5) << LOG_LPL) | rm;    // row of position 32m + O
            if constexpr (Hw<F>::OFF == 0) {
                // this column's code pair (a 16-bit read) and its block's scale
                // (one word, the same for the lanes of a line)
                const uint32_t cp = ctile16[2 * (n * 8 + ((cl >> 1) ^ cswz(n)))];
                a[O] = dec2<F, false>(cp, s_scf[(n / CB) * 16 + cl]);
            } else {
                // MXFP6: scale operand 2^(E + OFF), or 2^E and a factor 2^OFF
                // after decoding when E + OFF is above the scale range
                constexpr int OFF = Hw<F>::OFF;
                const uint32_t wd = ctile[n * 8 + ((cl >> 1) ^ cswz(n))];
                const int eb = (int)((s_ex4[(n / CB) * 4] >> exsh) & 0xffu);
                const int ebits = eb + eadd;
                const bool hi = ebits > 254 - OFF;
                const float s = __uint_as_float((uint32_t)(hi ? ebits : ebits + OFF) << 23);
                a[O] = mulp<F>(dec2<F, false>(wd >> cdsh, s), hi ? e8(OFF) : 1.0f);
            }
        });
        __syncthreads();
    }

    ERange er;
    constexpr int CL = layout_family<F, C>();
    all_stages<F, CL, (is_mx(F) ? C : 1), INV>(a, m, t, plane, er);
    if constexpr (F == BF16) {
        // a product below the FP32 normal range: the wave redoes its columns
        // (input read again from the intermediate) with such products exact
        if (__builtin_amdgcn_ballot_w64(er.sub) != 0) {
            sfor<P>([&](auto O) { a[O] = unpack16<F>(c16[(size_t)((rev(O, 5) << LOG_LPL) | rm) * 16 + cl]); });
            all_stages<F, CL, 1, INV, false, true>(a, m, t, plane, er);
        }
    }
}

// Column pass.
template <int F, int C, bool INV>
__global__ __launch_bounds__(THREADS)
__attribute__((amdgpu_waves_per_eu(waves_target(F == BF16), 8))) void k_col(FastArgs g)
{
    __shared__ ColLds<F, C> L;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int line = lane >> LOG_LPL, m = lane & (LPL - 1);
    const int slice = blockIdx.x / (N / LINES), cb16 = blockIdx.x % (N / LINES);
    const int cl = wave * LPW + line;                  // column within the work-group
    float2 a[P];
    col_lines<F, C, INV>(g, slice, cb16, a, L);
    const int kout = g.kout_mul * slice_k(g, slice) + g.kout_add;
    float2* tile = (float2*)L.plane;                   // N/2 x 16 complex
    static_assert(N / 2 * 16 * 2 <= WAVES * WPL, "output tile fits the planes");

    // output: scaled by 2^kout, staged through an LDS tile N/2 rows at a time
    // (the top row bit is an in-lane bit of the last layout) and written as
    // whole 128-byte row pieces
    constexpr int CL = layout_family<F, C>();
    constexpr int KL = Lay<CL>::NL - 1;
    constexpr int HB = Lay<CL>::index_of(KL, LOGN - 1);
    constexpr int LM = lane_mask<CL, KL>();
    static_assert(HB >= 0 && (LM & 1) == 0 && (LM >> (LOGN - 1)) == 0, "top row bit and bit 0 in-lane");
    const int pmL = posM<CL, KL>(m);
    float2* ys = g.dst + mxd::slice_base(g.slice_off_out, slice, (size_t)N * N) + cb16 * LINES;
    sfor<2>([&](auto H) {
        __syncthreads();
        sfor<P>([&](auto O) {
            if constexpr (((O >> HB) & 1) == H) {
                const int r = (Lay<CL>::posF(KL, O) | pmL) & (N / 2 - 1);
                float2 v = a[O];
                if constexpr (is_16(F)) v = unpack16<F>(pack16<F>(v.x, v.y));   // output in the format
                tile[tslot<LM>(r, cl)] = make_float2(ldexpf(v.x, kout), ldexpf(v.y, kout));
            }
        });
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const int q = i * THREADS + tid, R = q >> 3, pr = q & 7;
            const float4 v = *(const float4*)&tile[R * 16 + 2 * pr];
            const int xr = pext<LM>(R);
            const int r = R ^ (xr & 1);
            const int c = (2 * pr) ^ (((xr >> 1) & 3) << 2);
            *(float4*)&ys[(size_t)(H * (N / 2) + r) * N + c] = v;
        }
    });
}


// |v 2^kout|^2 added to a running FP32 sum: each square and their sum rounded
// to FP32 (no fused multiply-add); the 16-bit forms round v to the format first.
template <int F>
__device__ __forceinline__ float rss_add(float acc, float2 v, int kout)
{
#pragma clang fp contract(off)
    if constexpr (is_16(F)) v = unpack16<F>(pack16<F>(v.x, v.y));
    const float re = ldexpf(v.x, kout), im = ldexpf(v.y, kout);
    const float re2 = re * re;
    const float im2 = im * im;
    const float m2 = re2 + im2;
    return acc + m2;
}

// Column pass with the root-sum-of-squares coil combine (Eq. 1) as its
// epilogue: one work-group per (reconstruction, 16-column group) runs the
// column pass of every coil slice of the reconstruction in coil order and
// keeps the running sum of |T_c|^2 per value; only the FP32 image
// (sum)^(1/2), [reconstruction][n][n], is written.  Above 128 VGPRs in
// every form.
template <int F, int C, bool INV>
__global__ __launch_bounds__(THREADS)
__attribute__((amdgpu_waves_per_eu(waves_target(true), 8))) void k_col_rss(FastArgs g)
{
    __shared__ ColLds<F, C> L;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int line = lane >> LOG_LPL, m = lane & (LPL - 1);
    const int recon = blockIdx.x / (N / LINES), cb16 = blockIdx.x % (N / LINES);
    const int cl = wave * LPW + line;
    float acc[P];
    sfor<P>([&](auto O) { acc[O] = 0.0f; });
    for (int c = 0; c < g.coils; c++) {
        if (c > 0) __syncthreads();                    // the planes are free again
        const int slice = recon * g.coils + c;
        float2 a[P];
        col_lines<F, C, INV, true>(g, slice, cb16, a, L);
        const int kout = g.kout_mul * slice_k(g, slice) + g.kout_add;
        sfor<P>([&](auto O) { acc[O] = rss_add<F>(acc[O], a[O], kout); });
    }
    constexpr int CL = layout_family<F, C>();
    constexpr int KL = Lay<CL>::NL - 1;
    const int pmL = posM<CL, KL>(m);
    float* y = g.rss + (size_t)recon * N * N + cb16 * LINES + cl;
    sfor<P>([&](auto O) { y[(size_t)(Lay<CL>::posF(KL, O) | pmL) * N] = sqrtf(acc[O]); });
}

}  // namespace MXF_NS
