/*
 * mxfft_oracle.c -- CPU oracle for the MX-scaled mixed-precision radix-2 FFT of
 * Deveshwar, Rajagopal and Larson, "A mixed precision FFT with applications in MRI".
 *
 * TEST INFRASTRUCTURE ONLY.  This file states, plainly and slowly, what the GPU
 * library must compute.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  The product library never calls it and shares no
 * code, header, table or helper with it.
 *
 * Arithmetic model.  Every value the method keeps is an FP32 number or an element
 * of a narrow format.  Each operation is evaluated exactly (in double precision
 * or integer arithmetic where that is exact, otherwise through round-to-odd) and
 * rounded ONCE to its target precision, so every stored result is the correctly
 * rounded value of its defining expression.
 *
 * Readings of the paper that this file fixes (the paper is silent or ambiguous):
 *   - an MX block holds B real scalars, i.e. B/2 complex values whose real and
 *     imaginary parts share one scale (Sec. 2.2 and Sec. 4.2);
 *   - block scale: E = floor(log2 amax) - emax_elem, clamped to [-127, 127] (OCP
 *     MX); elements rounded to nearest-even and saturated to the largest finite
 *     element; an all-zero block gets E = 0;
 *   - butterfly blocks are B/2 consecutive butterflies t = g*h + j of a stage;
 *     input-encode blocks are B/2 consecutive complex values along the pass axis;
 *   - EncodeFromMantBlock quantises the renormalised product directly with the
 *     carried scale (no fresh amax), Alg. 2;
 *   - u is never encoded; values between stages are FP32;
 *   - every 1D pass MX-encodes its input; MX outputs are FP32 decodes;
 *   - radix-2 decimation in time on bit-reversed input, forward kernel
 *     exp(-2*pi*i*j*k/N); 2D = every row (contiguous axis) then every column;
 *   - one prescale exponent per N x N slice (Alg. 1); the forward output is
 *     de-scaled by 2^-k; the round trip keeps k and applies 2^(-k - 2 log2 N);
 *   - percentile: linear interpolation between order statistics,
 *     pos = ((n-1)*tau)/100 in FP64, p = S[i] + f*(S[i+1]-S[i]) in FP64;
 *   - quantised output (flag, MX formats; the 16-bit control's "quantized
 *     outputs", Sec. 2.2, carried over to MX): EncodeBlockMX of the final
 *     de-scaled output in blocks of B/2 consecutive rows of one column (the
 *     last pass's axis), each value element * 2^E rounded once to FP32.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#include "mxfft_oracle.h"

/* ------------------------------------------------------------------------- */
/* 1. Number formats                                                          */
/* ------------------------------------------------------------------------- */

typedef struct {
    int ebits;       /* exponent field width                                   */
    int mbits;       /* explicit mantissa bits                                 */
    int bias;        /* exponent bias                                          */
    int emin;        /* exponent of the smallest normal                        */
    int emax;        /* exponent of the largest normal (OCP "emax_elem")       */
    double maxval;   /* largest finite magnitude                               */
    int saturate;    /* 1: overflow clamps to maxval; 0: overflow gives Inf    */
    int nan_all_ones;/* 1: only S.1111.111 is NaN and there is no Inf (E4M3);
                        2: every code is a finite number (OCP FP6)            */
} fmtdesc;

/* OCP 8-bit formats (E4M3 "fn" and E5M2), IEEE half, bfloat16, a wide
 * 6-bit-exponent / 23-bit-mantissa element used only to pin the data flow,
 * and the OCP 6-bit MX elements E2M3 and E3M2 (no infinities, no NaN). */
static const fmtdesc FMT[ORC_NFMT] = {
    /* E4M3  */ {4, 3, 7, -6, 8, 448.0, 1, 1},
    /* E5M2  */ {5, 2, 15, -14, 15, 57344.0, 1, 0},
    /* FP16  */ {5, 10, 15, -14, 15, 65504.0, 0, 0},
    /* BF16  */ {8, 7, 127, -126, 127, 0x1.fep127, 0, 0},
    /* E6M23 */ {6, 23, 31, -30, 31, 0x1.fffffep31, 1, 0},
    /* E2M3  */ {2, 3, 1, 0, 2, 7.5, 1, 2},
    /* E3M2  */ {3, 2, 3, -2, 4, 28.0, 1, 2},
};

int orc_fmt_info(int f, int* ebits, int* mbits, int* emin, int* emax, double* maxval)
{
    if (f < 0 || f >= ORC_NFMT) return ORC_EINVAL;
    *ebits = FMT[f].ebits; *mbits = FMT[f].mbits; *emin = FMT[f].emin;
    *emax = FMT[f].emax; *maxval = FMT[f].maxval;
    return ORC_OK;
}

/* Q_F(x): round x (any double) to the nearest value of format f, ties to even,
 * on the format's grid (normal binades and the subnormal grid 2^(emin-m)).
 * Magnitudes above the largest finite value saturate (MX elements) or become
 * infinite (IEEE half / bfloat16).  Signed zeros and NaN pass through. */
double orc_quantize(int f, double x)
{
    const fmtdesc* d = &FMT[f];
    if (x == 0.0 || isnan(x)) return x;
    if (isinf(x)) return d->saturate ? copysign(d->maxval, x) : x;
    double a = fabs(x);
    int e = ilogb(a);                 /* exact floor(log2 a) */
    if (e < d->emin) e = d->emin;     /* subnormal grid */
    /* a / ulp is exact (power-of-two scaling); nearbyint rounds to nearest even */
    double q = ldexp(nearbyint(ldexp(a, d->mbits - e)), e - d->mbits);
    if (q > d->maxval) q = d->saturate ? d->maxval : INFINITY;
    return copysign(q, x);
}

/* Bit code of a value that is exactly representable in format f. */
int orc_encode_code(int f, double q)
{
    const fmtdesc* d = &FMT[f];
    int sign = signbit(q) ? 1 : 0;
    int top = sign << (d->ebits + d->mbits);
    double a = fabs(q);
    if ((isnan(q) || isinf(q)) && d->nan_all_ones == 2) return ORC_EINVAL;   /* not representable */
    if (isnan(q)) return top | ((1 << (d->ebits + d->mbits)) - 1);
    if (isinf(q)) return top | (((1 << d->ebits) - 1) << d->mbits);
    if (a == 0.0) return top;
    int e = ilogb(a);
    if (e < d->emin) return top | (int)ldexp(a, d->mbits - d->emin);
    int mant = (int)ldexp(a, d->mbits - e) - (1 << d->mbits);
    return top | ((e + d->bias) << d->mbits) | mant;
}

/* Value of bit code c in format f (NaN for NaN codes). */
double orc_decode_code(int f, int c)
{
    const fmtdesc* d = &FMT[f];
    int sign = (c >> (d->ebits + d->mbits)) & 1;
    int ef = (c >> d->mbits) & ((1 << d->ebits) - 1);
    int mf = c & ((1 << d->mbits) - 1);
    double v;
    if (d->nan_all_ones == 1) {
        if (ef == (1 << d->ebits) - 1 && mf == (1 << d->mbits) - 1) return NAN;
    } else if (d->nan_all_ones == 0 && ef == (1 << d->ebits) - 1) {
        v = mf ? NAN : INFINITY;
        return sign ? -v : v;
    }
    if (ef == 0) v = ldexp((double)mf, d->emin - d->mbits);
    else v = ldexp((double)((1 << d->mbits) | mf), ef - d->bias - d->mbits);
    return sign ? -v : v;
}

/* ------------------------------------------------------------------------- */
/* 2. One rounding for sums                                                   */
/* ------------------------------------------------------------------------- */

/* Exact a + b rounded to odd at double precision.  Rounding the result again,
 * to any format with at least two fewer significand bits, gives the correctly
 * rounded sum (Boldo and Melquiond, "When double rounding is odd").  TwoSum
 * (Knuth) recovers the exact error of the double addition. */
static double sum_round_odd(double a, double b)
{
    double s = a + b;
    if (!isfinite(s)) return s;         /* IEEE: infinite and NaN sums need no rounding */
    double bb = s - a;
    double err = (a - (s - bb)) + (b - bb);
    if (err != 0.0) {
        uint64_t bits;
        memcpy(&bits, &s, sizeof bits);
        if ((bits & 1u) == 0) {
            if ((err > 0.0) == (s > 0.0)) bits += 1; else bits -= 1;
            memcpy(&s, &bits, sizeof bits);
        }
    }
    return s;
}

/* fl32(a + b) with a single rounding. */
static float f32_add(double a, double b) { return (float)sum_round_odd(a, b); }

/* fl_F(a + b): correctly rounded sum in format f (f has at most 24 bits). */
static double fmt_add(int f, double a, double b) { return orc_quantize(f, sum_round_odd(a, b)); }

/* ------------------------------------------------------------------------- */
/* 3. MX block codec (EncodeBlockMX, MantissasBlock, DecodeBlockMX; Sec. 2.2) */
/* ------------------------------------------------------------------------- */

/* EncodeBlockMX followed by MantissasBlock: given the n real scalars of one
 * block, return the shared exponent E (the block scale is 2^E) and write the
 * element values mant[i] = Q_F(vals[i] * 2^-E).  The element values are the
 * "de-scaled mantissas"; the block value is mant[i] * 2^E (DecodeBlockMX). */
int orc_mx_encode(int f, const double* vals, int n, double* mant)
{
    double amax = 0.0;
    for (int i = 0; i < n; i++)
        if (fabs(vals[i]) > amax) amax = fabs(vals[i]);
    int E = 0;
    if (amax > 0.0) {
        E = ilogb(amax) - FMT[f].emax;
        if (E < -127) E = -127;
        if (E > 127) E = 127;
    }
    for (int i = 0; i < n; i++) mant[i] = orc_quantize(f, ldexp(vals[i], -E));
    return E;
}

/* ------------------------------------------------------------------------- */
/* 4. Twiddles                                                                */
/* ------------------------------------------------------------------------- */

/* w = exp(-2*pi*i*j/m) in FP64 for 0 <= j < m/2 (conjugate for the inverse).
 * The angle is reduced to the first octant with exact symmetries, so w_0 = 1,
 * w_{m/4} = -i and w_{m/8} has equal parts sqrt(1/2). */
static void twiddle64(int j, int m, int inverse, double* wr, double* wi)
{
    const double two_pi = 6.283185307179586476925286766559;
    double c, s;                         /* cos and sin of 2*pi*j/m */
    long j8 = 8L * j;
    if (j == 0) { c = 1.0; s = 0.0; }
    else if (4L * j == m) { c = 0.0; s = 1.0; }
    else if (j8 == m || j8 == 3L * m) { c = sqrt(0.5); s = sqrt(0.5); if (j8 == 3L * m) c = -c; }
    else if (j8 < m) { double t = two_pi * j / m; c = cos(t); s = sin(t); }
    else if (j8 < 2L * m) { double t = two_pi * (m / 4 - j) / m; c = sin(t); s = cos(t); }
    else if (j8 < 3L * m) { double t = two_pi * (j - m / 4) / m; c = -sin(t); s = cos(t); }
    else { double t = two_pi * (m / 2 - j) / m; c = -cos(t); s = sin(t); }
    *wr = c;
    *wi = inverse ? s : -s;
}

void orc_twiddle64(int j, int m, int inverse, double* wr, double* wi) { twiddle64(j, m, inverse, wr, wi); }

/* ------------------------------------------------------------------------- */
/* 5. MX-scaled complex butterfly (Alg. 2)                                    */
/* ------------------------------------------------------------------------- */

/* One block of cb butterflies.  u, v: FP32 complex (interleaved re, im).
 * x: the twiddle block's element values (interleaved), Ew its exponent.
 * Writes y0 = u + w*v and y1 = u - w*v (FP32).  Optional trace of Ev, kr, Eout. */
static void mx_butterfly_block(int f, int cb, const float* u, const float* v,
                               const double* x, int Ew, float* y0, float* y1,
                               double* scratch, int* tr_ev, int* tr_kr, int* tr_eo)
{
    double* vin = scratch;            /* 2cb */
    double* y = scratch + 2 * cb;     /* 2cb */
    double* p = scratch + 4 * cb;     /* 2cb */
    const double M = FMT[f].maxval;

    /* operand v: EncodeBlockMX + MantissasBlock */
    for (int k = 0; k < 2 * cb; k++) vin[k] = v[k];
    int Ev = orc_mx_encode(f, vin, 2 * cb, y);

    /* complex product of mantissas: FP32 multiplies, one FP32 rounding of the
     * sum or difference (for 8-bit elements the products are exact) */
    for (int t = 0; t < cb; t++) {
        double xr = x[2 * t], xi = x[2 * t + 1], yr = y[2 * t], yi = y[2 * t + 1];
        float rr = (float)(xr * yr), ii = (float)(xi * yi);
        float ri = (float)(xr * yi), ir = (float)(xi * yr);
        p[2 * t] = f32_add(rr, -(double)ii);
        p[2 * t + 1] = f32_add(ri, ir);
    }

    /* scale of the product block, renormalised when a product exceeds M_max */
    int Eout = Ew + Ev;
    double a = 0.0;
    for (int k = 0; k < 2 * cb; k++)
        if (fabs(p[k]) > a) a = fabs(p[k]);
    int kr = 0;
    if (a > M) {
        kr = 1;
        while (a > ldexp(M, kr)) kr++;     /* smallest k >= 1 with a <= M * 2^k */
    }
    Eout += kr;

    /* EncodeFromMantBlock (carried scale) then DecodeBlockMX, then u +/- wv */
    for (int k = 0; k < 2 * cb; k++) {
        double q = orc_quantize(f, ldexp(p[k], -kr));
        float wv = (float)ldexp(q, Eout);
        y0[k] = f32_add(u[k], wv);
        y1[k] = f32_add(u[k], -(double)wv);
    }
    if (tr_ev) { *tr_ev = Ev; *tr_kr = kr; *tr_eo = Eout; }
}

/* ------------------------------------------------------------------------- */
/* 6. One-dimensional passes over a contiguous line of N complex FP32 values  */
/* ------------------------------------------------------------------------- */

static int ilog2i(long n) { int l = 0; while ((1L << l) < n) l++; return l; }

static void bit_reverse(float* a, int N)
{
    int L = ilog2i(N);
    for (int i = 0; i < N; i++) {
        int r = 0;
        for (int b = 0; b < L; b++) r |= ((i >> b) & 1) << (L - 1 - b);
        if (r > i) {
            float t0 = a[2 * i], t1 = a[2 * i + 1];
            a[2 * i] = a[2 * r]; a[2 * i + 1] = a[2 * r + 1];
            a[2 * r] = t0; a[2 * r + 1] = t1;
        }
    }
}

typedef struct {
    int mode, fmt, B;
    double* scratch;    /* sized by line_scratch_doubles() */
    int* trace;         /* optional: per stage, per block (Ev, kr, Eout) for the first line */
    int raw_input;      /* MX: the line enters the stages without the input encode */
} passcfg;

static long line_scratch_doubles(int N) { return 16L * N + 64; }

/* MX pass: input encode, bit reversal, log2 N stages of MX butterfly blocks. */
static void mx_line(const passcfg* c, int N, int inverse, float* a, int* trace)
{
    const int f = c->fmt, cb = c->B / 2, L = ilog2i(N);
    double* vals = c->scratch;                 /* 2cb */
    double* mant = c->scratch + 2L * N;        /* 2cb */
    double* w = c->scratch + 4L * N;           /* 2cb */
    double* x = c->scratch + 6L * N;           /* 2cb */
    double* bs = c->scratch + 8L * N;          /* 6cb */
    float* u = (float*)malloc(sizeof(float) * 8 * cb);
    float* v = u + 2 * cb;
    float* y0 = u + 4 * cb;
    float* y1 = u + 6 * cb;

    /* input encode: blocks of cb consecutive complex in natural order */
    for (int b = 0; b < N / cb && !c->raw_input; b++) {
        for (int k = 0; k < 2 * cb; k++) vals[k] = a[2 * b * cb + k];
        int E = orc_mx_encode(f, vals, 2 * cb, mant);
        for (int k = 0; k < 2 * cb; k++) a[2 * b * cb + k] = (float)ldexp(mant[k], E);
    }
    bit_reverse(a, N);

    int tix = 0;
    for (int s = 1; s <= L; s++) {
        const int m = 1 << s, h = m >> 1;
        for (int blk = 0; blk < (N / 2) / cb; blk++) {
            for (int k = 0; k < cb; k++) {
                int t = blk * cb + k, g = t / h, j = t % h;
                int iu = g * m + j, iv = iu + h;
                u[2 * k] = a[2 * iu]; u[2 * k + 1] = a[2 * iu + 1];
                v[2 * k] = a[2 * iv]; v[2 * k + 1] = a[2 * iv + 1];
                twiddle64(j, m, inverse, &w[2 * k], &w[2 * k + 1]);
            }
            /* pre-quantised twiddle block: EncodeBlockMX of the block's FP64 twiddles */
            int Ew = orc_mx_encode(f, w, 2 * cb, x);
            int* tr = trace ? trace + 3 * tix : NULL;
            mx_butterfly_block(f, cb, u, v, x, Ew, y0, y1, bs,
                               tr, tr ? tr + 1 : NULL, tr ? tr + 2 : NULL);
            tix++;
            for (int k = 0; k < cb; k++) {
                int t = blk * cb + k, g = t / h, j = t % h;
                int iu = g * m + j, iv = iu + h;
                a[2 * iu] = y0[2 * k]; a[2 * iu + 1] = y0[2 * k + 1];
                a[2 * iv] = y1[2 * k]; a[2 * iv + 1] = y1[2 * k + 1];
            }
        }
    }
    free(u);
}

/* FP32 plain pass: FP32 twiddles (FP64 rounded once), FP32 products and sums,
 * no fused multiply-add: p_r = fl(fl(wr vr) - fl(wi vi)), p_i = fl(fl(wr vi) + fl(wi vr)). */
static void f32_line(int N, int inverse, float* a)
{
    const int L = ilog2i(N);
    bit_reverse(a, N);
    for (int s = 1; s <= L; s++) {
        const int m = 1 << s, h = m >> 1;
        for (int g = 0; g < N / m; g++)
            for (int j = 0; j < h; j++) {
                double wr64, wi64;
                twiddle64(j, m, inverse, &wr64, &wi64);
                float wr = (float)wr64, wi = (float)wi64;
                int iu = g * m + j, iv = iu + h;
                float vr = a[2 * iv], vi = a[2 * iv + 1];
                float rr = (float)((double)wr * vr), ii = (float)((double)wi * vi);
                float ri = (float)((double)wr * vi), ir = (float)((double)wi * vr);
                float pr = f32_add(rr, -(double)ii), pi = f32_add(ri, ir);
                float ur = a[2 * iu], ui = a[2 * iu + 1];
                a[2 * iu] = f32_add(ur, pr); a[2 * iu + 1] = f32_add(ui, pi);
                a[2 * iv] = f32_add(ur, -(double)pr); a[2 * iv + 1] = f32_add(ui, -(double)pi);
            }
    }
}

/* FP16 / BF16 pass (the paper's 16-bit positive control): the pass input is
 * rounded to the format; twiddles are FP64 rounded once to the format; each
 * stage rounds v to the format and forms the complex product with one rounding
 * to the format per multiply and per add; u +/- p is FP32. */
static void half_line(int f, int N, int inverse, float* a)
{
    const int L = ilog2i(N);
    for (int k = 0; k < 2 * N; k++) a[k] = (float)orc_quantize(f, a[k]);
    bit_reverse(a, N);
    for (int s = 1; s <= L; s++) {
        const int m = 1 << s, h = m >> 1;
        for (int g = 0; g < N / m; g++)
            for (int j = 0; j < h; j++) {
                double wr, wi;
                twiddle64(j, m, inverse, &wr, &wi);
                wr = orc_quantize(f, wr); wi = orc_quantize(f, wi);
                int iu = g * m + j, iv = iu + h;
                double vr = orc_quantize(f, a[2 * iv]), vi = orc_quantize(f, a[2 * iv + 1]);
                double rr = orc_quantize(f, wr * vr), ii = orc_quantize(f, wi * vi);
                double ri = orc_quantize(f, wr * vi), ir = orc_quantize(f, wi * vr);
                double pr = fmt_add(f, rr, -ii), pi = fmt_add(f, ri, ir);
                float ur = a[2 * iu], ui = a[2 * iu + 1];
                a[2 * iu] = f32_add(ur, pr); a[2 * iu + 1] = f32_add(ui, pi);
                a[2 * iv] = f32_add(ur, -pr); a[2 * iv + 1] = f32_add(ui, -pi);
            }
    }
}

static void run_line(const passcfg* c, int N, int inverse, float* a, int* trace)
{
    switch (c->mode) {
    case ORC_MODE_MX: mx_line(c, N, inverse, a, trace); break;
    case ORC_MODE_FP32: f32_line(N, inverse, a); break;
    default: half_line(c->fmt, N, inverse, a); break;
    }
}

/* ------------------------------------------------------------------------- */
/* 7. Global power-of-two prescale (Alg. 1)                                   */
/* ------------------------------------------------------------------------- */

/* Normalised integer significand and exponent: x = M * 2^e, 2^52 <= M < 2^53. */
static void split53(double x, uint64_t* M, int* e)
{
    int ex;
    double fr = frexp(x, &ex);           /* x = fr * 2^ex, fr in [0.5, 1) */
    *M = (uint64_t)ldexp(fr, 53);
    *e = ex - 53;
}

/* k1 = round(log2(T / a)) exactly, for T, a > 0.  With R = (T/a)^2 and
 * l = floor(log2 R), round(log2(T/a)) = floor((l + 1) / 2); a tie would need
 * T/a to be an odd power of sqrt(2), which no ratio of doubles is. */
static int exact_round_log2_ratio(double T, double a)
{
    uint64_t MT, Ma; int eT, ea;
    split53(T, &MT, &eT);
    split53(a, &Ma, &ea);
    unsigned __int128 A = (unsigned __int128)MT * MT, C = (unsigned __int128)Ma * Ma;
    /* A / C lies in (1/4, 4): find j = floor(log2(A / C)) in {-2, -1, 0, 1} */
    int j;
    if (A >= (C << 1)) j = 1;
    else if (A >= C) j = 0;
    else if ((A << 1) >= C) j = -1;
    else j = -2;
    int l = 2 * (eT - ea) + j;
    return (int)floor((l + 1) / 2.0);
}

/* k2 = ceil(log2(tmin / p)) exactly, for tmin, p > 0. */
static int exact_ceil_log2_ratio(double tmin, double p)
{
    uint64_t Mt, Mp; int et, ep;
    split53(tmin, &Mt, &et);
    split53(p, &Mp, &ep);
    if (Mt == Mp) return et - ep;               /* exact power of two */
    if (Mt > Mp) return et - ep + 1;            /* ratio in (2^l, 2^(l+1)), l = et-ep */
    return et - ep;                             /* ratio in (2^(l-1), 2^l) */
}

static int cmp_double(const void* a, const void* b)
{
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

/* Prescale exponent of one slice of n complex values (interleaved FP32).
 * m_i = |x_i| = sqrt(re^2 + im^2) in FP64; amax = max m_i; p_tau = tau-th
 * percentile of the nonzero m_i; k1 places the peak at the target, k2 lifts
 * the tail to the floor; k = clip(max(k1, k2), kmin, kmax).  An all-zero slice
 * gets k = 0.  Non-finite input is an error; so is a k that overflows FP32. */
int orc_prescale(const float* x, long n, double target, double tau, double tau_min,
                 int kmin, int kmax, int32_t* k_out)
{
    double* S = (double*)malloc(sizeof(double) * (n > 0 ? n : 1));
    long nz = 0;
    double amax = 0.0, cmax = 0.0;
    for (long i = 0; i < n; i++) {
        double re = x[2 * i], im = x[2 * i + 1];
        if (!isfinite(re) || !isfinite(im)) { free(S); *k_out = INT32_MIN; return ORC_ENONFINITE; }
        if (fabs(re) > cmax) cmax = fabs(re);
        if (fabs(im) > cmax) cmax = fabs(im);
        double m = sqrt(re * re + im * im);   /* squares exact, one rounding each for sum and sqrt */
        if (m > amax) amax = m;
        if (m > 0.0) S[nz++] = m;
    }
    if (nz == 0) { free(S); *k_out = 0; return ORC_OK; }
    qsort(S, nz, sizeof(double), cmp_double);

    const double eps = 1e-30;
    int k1 = exact_round_log2_ratio(target, amax > eps ? amax : eps);

    double pos = ((double)(nz - 1) * tau) / 100.0;
    long i = (long)floor(pos);
    if (i > nz - 1) i = nz - 1;
    double fr = pos - (double)i;
    double lo = S[i], hi = (i + 1 < nz) ? S[i + 1] : S[nz - 1];
    double d = hi - lo;
    double fd = fr * d;
    double p = lo + fd;
    free(S);
    int k2 = exact_ceil_log2_ratio(tau_min, p > eps ? p : eps);

    int k = k1 > k2 ? k1 : k2;
    if (k < kmin) k = kmin;
    if (k > kmax) k = kmax;
    if (cmax > 0.0 && ilogb(cmax) + (long)k > 127) { *k_out = INT32_MIN; return ORC_ERANGE; }
    *k_out = k;
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* 8. Two-dimensional transforms of N x N slices                              */
/* ------------------------------------------------------------------------- */

/* x <- fl32(in * 2^k_in); every row then every column gets a 1D pass;
 * FP16/BF16 round the result to the format; out <- fl32(y * 2^k_out). */
static void transform2d(const passcfg* c, int N, int inverse, int k_in, int k_out,
                        const float* in, float* out, float* line, int* trace, int raw_rows)
{
    const long NN = (long)N * N;
    float* a = out;
    passcfg rc = *c;            /* the row passes' configuration */
    rc.raw_input = raw_rows;
    for (long i = 0; i < 2 * NN; i++) a[i] = (float)ldexp((double)in[i], k_in);
    for (int r = 0; r < N; r++) {
        memcpy(line, a + 2L * r * N, sizeof(float) * 2 * N);
        run_line(&rc, N, inverse, line, r == 0 ? trace : NULL);
        memcpy(a + 2L * r * N, line, sizeof(float) * 2 * N);
    }
    for (int col = 0; col < N; col++) {
        for (int r = 0; r < N; r++) {
            line[2 * r] = a[2L * (r * (long)N + col)];
            line[2 * r + 1] = a[2L * (r * (long)N + col) + 1];
        }
        run_line(c, N, inverse, line, NULL);
        for (int r = 0; r < N; r++) {
            a[2L * (r * (long)N + col)] = line[2 * r];
            a[2L * (r * (long)N + col) + 1] = line[2 * r + 1];
        }
    }
    if (c->mode == ORC_MODE_FP16 || c->mode == ORC_MODE_BF16)
        for (long i = 0; i < 2 * NN; i++) a[i] = (float)orc_quantize(c->fmt, a[i]);
    for (long i = 0; i < 2 * NN; i++) a[i] = (float)ldexp((double)a[i], k_out);
}

static int valid_cfg(int mode, int fmt, int B, int N)
{
    if (N < 2 || (N & (N - 1)) != 0 || N > (1 << 14)) return 0;
    if (mode == ORC_MODE_MX) {
        if (fmt != ORC_E4M3 && fmt != ORC_E5M2 && fmt != ORC_E6M23 && fmt != ORC_E2M3 && fmt != ORC_E3M2) return 0;
        if (B < 2 || (B & (B - 1)) != 0 || B > N) return 0;
        return 1;
    }
    return mode == ORC_MODE_FP32 || mode == ORC_MODE_FP16 || mode == ORC_MODE_BF16;
}

static int mode_fmt(int mode, int fmt)
{
    if (mode == ORC_MODE_FP16) return ORC_FP16;
    if (mode == ORC_MODE_BF16) return ORC_BF16;
    return fmt;
}

/* Work description shared by the per-slice driver and its worker threads. */
typedef struct {
    int op;              /* 0 forward, 1 inverse, 2 round trip */
    int mode, fmt, B, N;
    const float* in;
    float* out;
    int32_t* kp;         /* per slice: in (inverse with given k) or out */
    int kp_given;
    double target, tau, tau_min;
    int kmin, kmax;
    unsigned flags;
    long next;           /* next slice to take */
    long batch;
    int status;
    pthread_mutex_t mu;
} job;

/* The flag's output quantisation: every column of an N x N slice MX-encoded
 * in blocks of B/2 consecutive rows (EncodeBlockMX), each value replaced by
 * element * 2^E rounded once to FP32. */
static void quantize_columns(int fmt, int B, int N, float* a)
{
    const int cb = B / 2;
    double vals[2 * 4096], m[2 * 4096];
    for (int col = 0; col < N; col++)
        for (int rb = 0; rb < N / cb; rb++) {
            for (int k = 0; k < cb; k++) {
                const long idx = (long)(rb * cb + k) * N + col;
                vals[2 * k] = a[2 * idx];
                vals[2 * k + 1] = a[2 * idx + 1];
            }
            const int e = orc_mx_encode(fmt, vals, 2 * cb, m);
            for (int k = 0; k < cb; k++) {
                const long idx = (long)(rb * cb + k) * N + col;
                a[2 * idx] = (float)ldexp(m[2 * k], e);
                a[2 * idx + 1] = (float)ldexp(m[2 * k + 1], e);
            }
        }
}

static int run_slice_body(job* jb, long s, double* scratch, float* line);

static int run_slice(job* jb, long s, double* scratch, float* line)
{
    const int st = run_slice_body(jb, s, scratch, line);
    if (st == ORC_OK && (jb->flags & ORC_QUANTIZE_OUT) && jb->mode == ORC_MODE_MX)
        quantize_columns(jb->fmt, jb->B, jb->N, jb->out + 2 * (long)jb->N * jb->N * s);
    return st;
}

static int run_slice_body(job* jb, long s, double* scratch, float* line)
{
    const int N = jb->N, L = ilog2i(N);
    const long NN = (long)N * N;
    const float* in = jb->in + 2 * NN * s;
    float* out = jb->out + 2 * NN * s;
    passcfg c = { jb->mode, mode_fmt(jb->mode, jb->fmt), jb->B, scratch, NULL };
    int32_t k = 0;
    int st = ORC_OK;

    if (jb->op == 1 && jb->kp_given) {
        k = jb->kp[s];
        int ko = -k - ((jb->flags & ORC_NORMALIZE) ? 2 * L : 0);
        transform2d(&c, N, 1, 0, ko, in, out, line, NULL, 0);
        return ORC_OK;
    }
    if (!(jb->flags & ORC_NO_PRESCALE))
        st = orc_prescale(in, NN, jb->target, jb->tau, jb->tau_min, jb->kmin, jb->kmax, &k);
    if (jb->kp && !(jb->op == 1 && jb->kp_given)) jb->kp[s] = (st == ORC_OK) ? k : INT32_MIN;
    if (st != ORC_OK) { memset(out, 0, sizeof(float) * 2 * NN); return st; }

    if (jb->op == 0) {
        transform2d(&c, N, 0, k, (jb->flags & ORC_KEEP_SCALE) ? 0 : -k, in, out, line, NULL, 0);
    } else if (jb->op == 1) {
        int ko = -k - ((jb->flags & ORC_NORMALIZE) ? 2 * L : 0);
        transform2d(&c, N, 1, k, ko, in, out, line, NULL, 0);
    } else {
        /* round trip (Eq. 1): forward keeping the scale, then the inverse with
         * the same k, then 2^(-k - 2 log2 N).  Fused (the encode -> F -> F^-1
         * -> decode of the discussion, Sec. 4): the forward result enters the
         * inverse's row stages without being MX-encoded again. */
        float* mid = (float*)malloc(sizeof(float) * 2 * NN);
        transform2d(&c, N, 0, k, 0, in, mid, line, NULL, 0);
        transform2d(&c, N, 1, 0, -k - 2 * L, mid, out, line, NULL, (jb->flags & ORC_FUSED_RT) ? 1 : 0);
        free(mid);
    }
    return ORC_OK;
}

static void* worker(void* arg)
{
    job* jb = (job*)arg;
    double* scratch = (double*)malloc(sizeof(double) * line_scratch_doubles(jb->N));
    float* line = (float*)malloc(sizeof(float) * 2 * jb->N);
    for (;;) {
        pthread_mutex_lock(&jb->mu);
        long s = jb->next++;
        pthread_mutex_unlock(&jb->mu);
        if (s >= jb->batch) break;
        int st = run_slice(jb, s, scratch, line);
        if (st != ORC_OK) {
            pthread_mutex_lock(&jb->mu);
            if (jb->status == ORC_OK) jb->status = st;
            pthread_mutex_unlock(&jb->mu);
        }
    }
    free(scratch);
    free(line);
    return NULL;
}

static int run_job(job* jb, int nthreads)
{
    if (!valid_cfg(jb->mode, jb->fmt, jb->B, jb->N) || jb->batch < 0) return ORC_EINVAL;
    if (!(jb->tau >= 0.0 && jb->tau <= 100.0) || !(jb->target > 0.0) || !(jb->tau_min > 0.0)
        || !isfinite(jb->target) || !isfinite(jb->tau_min))
        if (!(jb->flags & ORC_NO_PRESCALE)) return ORC_EINVAL;
    jb->next = 0;
    jb->status = ORC_OK;
    pthread_mutex_init(&jb->mu, NULL);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > jb->batch) nthreads = (int)(jb->batch > 0 ? jb->batch : 1);
    pthread_t th[256];
    if (nthreads > 256) nthreads = 256;
    for (int t = 1; t < nthreads; t++) pthread_create(&th[t], NULL, worker, jb);
    worker(jb);
    for (int t = 1; t < nthreads; t++) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&jb->mu);
    return jb->status;
}

int orc_transform(int op, int mode, int fmt, int B, int N, long batch,
                  const float* in, float* out, int32_t* kp, int kp_given,
                  double target, double tau, double tau_min, int kmin, int kmax,
                  unsigned flags, int nthreads)
{
    job jb;
    memset(&jb, 0, sizeof jb);
    jb.op = op; jb.mode = mode; jb.fmt = fmt; jb.B = B; jb.N = N;
    jb.in = in; jb.out = out; jb.kp = kp; jb.kp_given = kp_given;
    jb.target = target; jb.tau = tau; jb.tau_min = tau_min;
    jb.kmin = kmin; jb.kmax = kmax; jb.flags = flags; jb.batch = batch;
    return run_job(&jb, nthreads);
}

/* Rows only (one 1D pass over each of `lines` contiguous lines of N complex
 * values), with an optional trace (Ev, kr, Eout per stage and block) of line 0. */
int orc_pass_lines(int mode, int fmt, int B, int N, int inverse, long lines, float* a, int* trace)
{
    if (!valid_cfg(mode, fmt, B, N)) return ORC_EINVAL;
    double* scratch = (double*)malloc(sizeof(double) * line_scratch_doubles(N));
    passcfg c = { mode, mode_fmt(mode, fmt), B, scratch, NULL };
    for (long r = 0; r < lines; r++) run_line(&c, N, inverse, a + 2L * N * r, r == 0 ? trace : NULL);
    free(scratch);
    return ORC_OK;
}

/* MX-encode the pass input of every column of an N x N slice (the values the
 * column pass starts from): blocks of B/2 consecutive rows within one column.
 * Writes the element values and one exponent per (column, row block). */
int orc_column_encode(int fmt, int B, int N, const float* a, double* mant, int32_t* E)
{
    if (!valid_cfg(ORC_MODE_MX, fmt, B, N)) return ORC_EINVAL;
    const int cb = B / 2;
    double vals[2 * 4096];
    double m[2 * 4096];
    if (cb > 4096) return ORC_EINVAL;
    for (int col = 0; col < N; col++)
        for (int rb = 0; rb < N / cb; rb++) {
            for (int k = 0; k < cb; k++) {
                long idx = (long)(rb * cb + k) * N + col;
                vals[2 * k] = a[2 * idx]; vals[2 * k + 1] = a[2 * idx + 1];
            }
            int e = orc_mx_encode(fmt, vals, 2 * cb, m);
            E[(long)col * (N / cb) + rb] = e;
            for (int k = 0; k < cb; k++) {
                long idx = (long)(rb * cb + k) * N + col;
                mant[2 * idx] = m[2 * k]; mant[2 * idx + 1] = m[2 * k + 1];
            }
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* 9. FP64 reference transforms                                               */
/* ------------------------------------------------------------------------- */

/* Radix-2 FFT of one line in FP64 (the algebraic reference). */
static void f64_line(int N, int inverse, double* a)
{
    const int L = ilog2i(N);
    for (int i = 0; i < N; i++) {
        int r = 0;
        for (int b = 0; b < L; b++) r |= ((i >> b) & 1) << (L - 1 - b);
        if (r > i) {
            double t0 = a[2 * i], t1 = a[2 * i + 1];
            a[2 * i] = a[2 * r]; a[2 * i + 1] = a[2 * r + 1];
            a[2 * r] = t0; a[2 * r + 1] = t1;
        }
    }
    for (int s = 1; s <= L; s++) {
        const int m = 1 << s, h = m >> 1;
        for (int g = 0; g < N / m; g++)
            for (int j = 0; j < h; j++) {
                double wr, wi;
                twiddle64(j, m, inverse, &wr, &wi);
                int iu = g * m + j, iv = iu + h;
                double vr = a[2 * iv], vi = a[2 * iv + 1];
                double pr = wr * vr - wi * vi, pi = wr * vi + wi * vr;
                double ur = a[2 * iu], ui = a[2 * iu + 1];
                a[2 * iu] = ur + pr; a[2 * iu + 1] = ui + pi;
                a[2 * iv] = ur - pr; a[2 * iv + 1] = ui - pi;
            }
    }
}

/* Unnormalised 2D FFT in FP64, rows then columns, of `batch` N x N slices. */
int orc_fft2_f64(int N, long batch, int inverse, double* a)
{
    if (N < 2 || (N & (N - 1)) != 0) return ORC_EINVAL;
    double* line = (double*)malloc(sizeof(double) * 2 * N);
    for (long s = 0; s < batch; s++) {
        double* x = a + 2L * N * N * s;
        for (int r = 0; r < N; r++) f64_line(N, inverse, x + 2L * r * N);
        for (int col = 0; col < N; col++) {
            for (int r = 0; r < N; r++) {
                line[2 * r] = x[2L * (r * (long)N + col)];
                line[2 * r + 1] = x[2L * (r * (long)N + col) + 1];
            }
            f64_line(N, inverse, line);
            for (int r = 0; r < N; r++) {
                x[2L * (r * (long)N + col)] = line[2 * r];
                x[2L * (r * (long)N + col) + 1] = line[2 * r + 1];
            }
        }
    }
    free(line);
    return ORC_OK;
}

int orc_fft1_f64(int N, long lines, int inverse, double* a)
{
    if (N < 2 || (N & (N - 1)) != 0) return ORC_EINVAL;
    for (long r = 0; r < lines; r++) f64_line(N, inverse, a + 2L * N * r);
    return ORC_OK;
}

/* Vector helpers for the tests. */
void orc_quantize_array(int f, const double* x, double* q, long n)
{
    for (long i = 0; i < n; i++) q[i] = orc_quantize(f, x[i]);
}

void orc_mx_butterfly(int f, int cb, const float* u, const float* v, const double* x, int Ew,
                      float* y0, float* y1, int* ev_kr_eo)
{
    double* scratch = (double*)malloc(sizeof(double) * 6 * cb);
    mx_butterfly_block(f, cb, u, v, x, Ew, y0, y1, scratch,
                       ev_kr_eo, ev_kr_eo ? ev_kr_eo + 1 : NULL, ev_kr_eo ? ev_kr_eo + 2 : NULL);
    free(scratch);
}

/* ------------------------------------------------------------------------- */
/* 10. Root-sum-of-squares coil combine (Eq. 1)                               */
/* ------------------------------------------------------------------------- */

/* x_RSS = (sum_c |T_c|^2)^(1/2) for every pixel of `recon` images of `coils`
 * coil slices each (T: [recon][coils][nn] interleaved complex, out:
 * [recon][nn]).  FP32 throughout: |T|^2 = re*re + im*im with each product and
 * the sum rounded to FP32 (no fused multiply-add), the coils added in order
 * c = 0 .. C-1 to a running FP32 sum, then the correctly rounded square root. */
int orc_rss(const float* T, long recon, int coils, long nn, float* out)
{
    if (coils < 1 || recon < 0 || nn < 0) return ORC_EINVAL;
    for (long r = 0; r < recon; r++)
        for (long i = 0; i < nn; i++) {
            float acc = 0.0f;
            for (int c = 0; c < coils; c++) {
                const float* t = T + 2 * ((r * coils + c) * nn + i);
                const float re2 = t[0] * t[0];
                const float im2 = t[1] * t[1];
                const float m = re2 + im2;
                acc = acc + m;
            }
            out[r * nn + i] = sqrtf(acc);
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* 11. Structural similarity (SSIM) of two images                             */
/* ------------------------------------------------------------------------- */

/* Mean SSIM of image x against reference y (both N x N, FP32 values) in the
 * form of Wang, Bovik, Sheikh and Simoncelli (2004): local statistics under
 * an 11 x 11 Gaussian window of standard deviation 1.5 normalised to unit
 * sum, C1 = (0.01 L)^2, C2 = (0.03 L)^2 with L the dynamic range, the index
 *   ((2 mx my + C1)(2 sxy + C2)) / ((mx^2 + my^2 + C1)(sx^2 + sy^2 + C2))
 * at every position where the window lies inside the image, averaged.  All
 * arithmetic in FP64. */
int orc_ssim(const float* x, const float* y, int N, double L, double* ssim)
{
    enum { W = 11, R = 5 };
    if (N < W || !(L > 0.0)) return ORC_EINVAL;
    double w[W][W], sum = 0.0;
    for (int i = 0; i < W; i++)
        for (int j = 0; j < W; j++) {
            const double d2 = (double)((i - R) * (i - R) + (j - R) * (j - R));
            w[i][j] = exp(-d2 / (2.0 * 1.5 * 1.5));
            sum += w[i][j];
        }
    for (int i = 0; i < W; i++)
        for (int j = 0; j < W; j++) w[i][j] /= sum;
    const double C1 = (0.01 * L) * (0.01 * L), C2 = (0.03 * L) * (0.03 * L);
    double total = 0.0;
    for (int r = R; r < N - R; r++)
        for (int c = R; c < N - R; c++) {
            double mx = 0, my = 0, xx = 0, yy = 0, xy = 0;
            for (int i = 0; i < W; i++)
                for (int j = 0; j < W; j++) {
                    const double a = x[(long)(r + i - R) * N + (c + j - R)];
                    const double b = y[(long)(r + i - R) * N + (c + j - R)];
                    mx += w[i][j] * a;
                    my += w[i][j] * b;
                    xx += w[i][j] * a * a;
                    yy += w[i][j] * b * b;
                    xy += w[i][j] * a * b;
                }
            const double sx = xx - mx * mx, sy = yy - my * my, sxy = xy - mx * my;
            total += ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sx + sy + C2));
        }
    *ssim = total / ((double)(N - 2 * R) * (N - 2 * R));
    return ORC_OK;
}
