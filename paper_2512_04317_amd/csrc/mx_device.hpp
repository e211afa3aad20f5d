// mx_device.hpp -- gfx950 device helpers for the MX-scaled FFT: OCP FP8 element
// rounding, MX block exponents and the renormalisation exponent of Alg. 2.
//
// All element arithmetic is "fake quantisation" in FP32 registers: a value is
// kept as the FP32 number equal to its FP8 element (an FP8 value is exact in
// FP32), so codes need never be materialised except where they are stored.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mxd {

// OCP 8-bit elements of MXFP8 (Sec. 2.2; Fig. 1C).
//   EMAX : exponent of the largest normal (the OCP MX "emax_elem")
//   MBITS: explicit mantissa bits;  EMIN: exponent of the smallest normal
//   MAXV : largest finite magnitude (1.75 * 2^EMAX for both 8-bit formats)
template <int F> struct Elem;
template <> struct Elem<0> {  // E4M3 ("fn": no infinities)
    static constexpr int EMAX = 8, MBITS = 3, EMIN = -6;
    static constexpr float MAXV = 448.0f;
};
template <> struct Elem<1> {  // E5M2
    static constexpr int EMAX = 15, MBITS = 2, EMIN = -14;
    static constexpr float MAXV = 57344.0f;
};
// OCP 6-bit elements of MXFP6 (no infinities or NaN; MAXV = 1.875 * 2^2 and
// 1.75 * 2^4)
template <> struct Elem<5> {  // E2M3
    static constexpr int EMAX = 2, MBITS = 3, EMIN = 0;
    static constexpr float MAXV = 7.5f;
};
template <> struct Elem<6> {  // E3M2
    static constexpr int EMAX = 4, MBITS = 2, EMIN = -2;
    static constexpr float MAXV = 28.0f;
};

// Round y to the element grid of format F, ties to even, saturating at MAXV,
// keeping the sign (also of zero).  Requires |y| < 2^100 (block-scaled
// operands are below 2^(EMAX+1)).
// The grid step is 2^(max(e, EMIN) - MBITS) for |y| in [2^e, 2^(e+1)); adding
// and subtracting c = 1.5 * 2^(max(e,EMIN) - MBITS + 23) rounds |y| to it in one
// IEEE addition (round to nearest even), and the subtraction is exact.
template <int F>
__device__ __forceinline__ float quant(float y)
{
    using E = Elem<F>;
    const uint32_t b = __float_as_uint(y);
    const uint32_t e = max(b & 0x7f800000u, uint32_t(E::EMIN + 127) << 23);
    const float c = __uint_as_float(e + (uint32_t(23 - E::MBITS) << 23) + 0x00400000u);
    float r = (fabsf(y) + c) - c;
    r = fminf(r, E::MAXV);
    return __uint_as_float(__float_as_uint(r) | (b & 0x80000000u));
}

// |x| as an ordered integer key (non-negative floats order like their bits).
__device__ __forceinline__ uint32_t abs_key(float x) { return __float_as_uint(x) & 0x7fffffffu; }

// Shared block exponent from the block's largest magnitude (bits of a
// non-negative float): E = floor(log2 amax) - EMAX clamped to >= -127 (the
// upper clamp at 127 cannot bind for FP32 data); an all-zero block gets E = 0.
template <int F>
__device__ __forceinline__ int block_exp(uint32_t amax_key)
{
    const int e = __builtin_amdgcn_frexp_expf(__uint_as_float(amax_key)) - 1;  // exact, subnormals too
    const int E = max(e - Elem<F>::EMAX, -127);
    return amax_key ? E : 0;
}

// Alg. 2 renormalisation: the smallest k >= 1 with amax <= MAXV * 2^k when
// amax > MAXV, else 0.  MAXV = 1.m * 2^EMAX, so amax = 1.f * 2^e needs
// k = e - EMAX, plus one when f > m; adding 0x7FFFFF - m to the bits carries
// into the exponent field exactly when the fraction field exceeds m's (for
// the 8-bit formats m = 0.75: 0x600000, the addend 0x1FFFFF).
template <int F>
__device__ __forceinline__ int renorm_exp(uint32_t amax_key)
{
    constexpr uint32_t MF = __builtin_bit_cast(uint32_t, Elem<F>::MAXV) & 0x007FFFFFu;
    const int k = int((amax_key + (0x007FFFFFu - MF)) >> 23) - 127 - Elem<F>::EMAX;
    return max(k, 0);
}

// ---------------------------------------------------------------------------
// gfx950 element conversions (v_cvt_scalef32_pk_*): bit-identical to OCP
// rounding (round to nearest even, subnormals, signed zero) once the values
// are clamped to the largest element; they do not saturate by themselves
// ---------------------------------------------------------------------------

typedef short short2v __attribute__((ext_vector_type(2)));
typedef float float2v __attribute__((ext_vector_type(2)));

// 2^E as the E8M0-style scale operand, -127 <= E <= 127.
__device__ __forceinline__ float e8(int E) { return __uint_as_float((uint32_t)(E + 127) << 23); }

// Conversion hardware of element format F.  MXFP6 travels in the FP8
// conversions: an E2M3 value times 2^-6 is an E4M3 value and an E3M2 value
// times 2^-12 an E5M2 value (same mantissa width, subnormal spacing and
// smallest normal), so encoding x / 2^E to FP6 is encoding x / 2^(E + OFF)
// to FP8 and decoding multiplies by 2^(E + OFF).
template <int F> struct Hw { static constexpr int FMT = F, OFF = 0; };
template <> struct Hw<5> { static constexpr int FMT = 0, OFF = 6; };    // E2M3 via E4M3
template <> struct Hw<6> { static constexpr int FMT = 1, OFF = 12; };   // E3M2 via E5M2

// Mantissa field of MAXV (0x600000 for 1.75, 0x700000 for 1.875).
template <int F>
constexpr uint32_t maxv_frac() { return __builtin_bit_cast(uint32_t, Elem<F>::MAXV) & 0x007FFFFFu; }

// MAXV * 2^E, the saturation bound at block scale 2^E.
template <int F>
__device__ __forceinline__ float lim_of(int E)
{
    constexpr uint32_t MF = maxv_frac<F>();
    return __uint_as_float(((uint32_t)(E + Elem<F>::EMAX + 127) << 23) | MF);
}

// Block scale at exponent E for the conversions: the scale operand s, a
// factor pre applied to the values before encoding (and to the saturation
// bound) and post applied after decoding.  FP8: s = 2^E.  FP6: s = 2^(E+OFF),
// unless E + OFF is above the scale range; then s = 2^E with pre = 2^-OFF and
// post = 2^OFF (exact: such blocks hold values near 2^(127 - OFF)).
struct Blk {
    float s, pre, post;
};
template <int F>
__device__ __forceinline__ Blk blk(int E)
{
    constexpr int OFF = Hw<F>::OFF;
    if constexpr (OFF == 0) {
        return Blk{e8(E), 1.0f, 1.0f};
    } else {
        const bool hi = E > 127 - OFF;
        return Blk{e8(hi ? E : E + OFF), hi ? e8(-OFF) : 1.0f, hi ? e8(OFF) : 1.0f};
    }
}
// v * f, only for the formats with a scale offset
template <int F>
__device__ __forceinline__ float2 mulp(float2 v, float f)
{
    if constexpr (Hw<F>::OFF == 0) return v;
    else return make_float2(v.x * f, v.y * f);
}
template <int F>
__device__ __forceinline__ float mulp1(float v, float f)
{
    if constexpr (Hw<F>::OFF == 0) return v;
    else return v * f;
}
// scale operand that decodes codes to element values (2^OFF)
template <int F>
__device__ __forceinline__ float unit_scale() { return e8(Hw<F>::OFF); }

// codes of (a, b) / 2^E in the low (W = 0) or high (W = 1) half of `old`
template <int F, bool W>
__device__ __forceinline__ uint32_t enc2(uint32_t old, float a, float b, float scale)
{
    short2v o;
    __builtin_memcpy(&o, &old, 4);
    short2v r;
    if constexpr (Hw<F>::FMT == 0) r = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(o, a, b, scale, W);
    else r = __builtin_amdgcn_cvt_scalef32_pk_bf8_f32(o, a, b, scale, W);
    uint32_t u;
    __builtin_memcpy(&u, &r, 4);
    return u;
}

// element values of the two codes in half W, times 2^E
template <int F, bool W>
__device__ __forceinline__ float2 dec2(uint32_t codes, float scale)
{
    float2v d;
    if constexpr (Hw<F>::FMT == 0) d = __builtin_amdgcn_cvt_scalef32_pk_f32_fp8(codes, scale, W);
    else d = __builtin_amdgcn_cvt_scalef32_pk_f32_bf8(codes, scale, W);
    return make_float2(d.x, d.y);
}

// v clamped to +-lim (the saturation of the element format at scale lim / MAXV)
__device__ __forceinline__ float2 clamp2(float2 v, float lim)
{
    return make_float2(__builtin_amdgcn_fmed3f(v.x, -lim, lim), __builtin_amdgcn_fmed3f(v.y, -lim, lim));
}


// Element offset of slice `slice` in a pool: from the per-slice table when
// there is one (slices anywhere in the pool), else slice * nn (contiguous).
__device__ __forceinline__ size_t slice_base(const unsigned long long* off, int slice, size_t nn)
{
    return off ? (size_t)off[slice] : (size_t)slice * nn;
}

// Maximum over groups of `width` consecutive lanes (width a power of two,
// 1 <= width <= 64) of non-negative values given as bits, every lane
// receiving its group's value; every lane of a group must be active.  Inside
// a DPP row of 16 lanes: quad_perm swaps 1 and 2 lanes apart, then the
// half-row mirror (lane i <-> 7 - i) and the row mirror (i <-> 15 - i), each
// of which meets the other half of the group reduced so far; lane permutes
// beyond 16.
__device__ __forceinline__ uint32_t group_max(uint32_t v, int width)
{
    if (width >= 2) v = max(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true));
    if (width >= 4) v = max(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true));
    if (width >= 8) v = max(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, true));
    if (width >= 16) v = max(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, true));
    for (int o = 16; o < width; o <<= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}

// ---------------------------------------------------------------------------
// IEEE half and bfloat16 (the 16-bit forms of the comparison, Sec. 2.3):
// round to nearest even, overflow to infinity, subnormals kept.
// ---------------------------------------------------------------------------

// x rounded to IEEE half (hardware conversion, round to nearest even)
__device__ __forceinline__ float round_fp16(float x) { return __half2float(__float2half_rn(x)); }

// x rounded to bfloat16: round to nearest even on the FP32 bits (NaN kept)
__device__ __forceinline__ float round_bf16(float x)
{
    uint32_t b = __float_as_uint(x);
    if ((b & 0x7fffffffu) > 0x7f800000u) return x;
    b += 0x7fffu + ((b >> 16) & 1u);
    return __uint_as_float(b & 0xffff0000u);
}

// M: 2 half, 3 bfloat16
template <int M>
__device__ __forceinline__ float round16(float x)
{
    if constexpr (M == 2) return round_fp16(x);
    else return round_bf16(x);
}

// The format's rounding of the exact product of two of its values.  Half
// products are exact in FP32 (22 significant bits, at least 2^-48).  Bfloat16
// products are exact in FP32 while normal (16 bits); below 2^-126 the FP32
// product may already be rounded, so the exact FP64 product is rounded to the
// bfloat16 subnormal grid 2^-133 instead.
template <int M>
__device__ __forceinline__ float mul16(float a, float b)
{
    // the empty asm keeps the product an FP32 multiply: folded into the
    // conversion it becomes a mixed FMA with a +0 addend, which turns a -0
    // product into +0
    float p = a * b;
    asm volatile("" : "+v"(p));
    if constexpr (M == 3) {
        if (__builtin_expect(fabsf(p) < 0x1p-126f, 0) && a != 0.f && b != 0.f) {
            const double q = __builtin_rint((double)a * (double)b * 0x1p133) * 0x1p-133;
            return (float)q;
        }
    }
    return round16<M>(p);
}

// The format's rounding of the sum of two of its values: the FP32 sum is
// exact unless the exponents differ by more than the FP32 spare bits, and
// then the smaller operand is far below half a unit in the last place of the
// format, where FP32 rounding cannot move the result across a rounding
// boundary of the format.
template <int M>
__device__ __forceinline__ float add16(float a, float b) { return round16<M>(a + b); }

}  // namespace mxd
