// mxfft_kernels.hip -- gfx950 kernels of the MX-scaled mixed-precision 2D FFT.
//
//  k_stats_part / k_stats_final : global power-of-two prescale of each slice
//            (Alg. 1), exact: chunk statistics, then one work-group per slice.
//  k_lines : one radix-2 decimation-in-time pass over the rows or the columns
//            of every slice, with per-block MX encoding of the pass input and
//            the MX-scaled butterfly of Alg. 2 at every stage (or the plain
//            FP32 butterfly for the comparison form).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "mx_device.hpp"
#include "mxfft_internal.hpp"

namespace mxk {

// ---------------------------------------------------------------------------
// Alg. 1: prescale statistics and exponent
// ---------------------------------------------------------------------------

// round(log2(T / a)) exactly for T, a > 0.  With R = (T/a)^2 and
// l = floor(log2 R) the result is floor((l + 1) / 2): log2(T/a) lies in
// [l/2, (l+1)/2), and a tie would need T/a to be an odd power of sqrt 2.
__device__ int round_log2_ratio(double T, double a)
{
    int eT, ea;
    const double fT = frexp(T, &eT), fa = frexp(a, &ea);
    const unsigned long long MT = (unsigned long long)ldexp(fT, 53);
    const unsigned long long Ma = (unsigned long long)ldexp(fa, 53);
    const unsigned __int128 A = (unsigned __int128)MT * MT;
    const unsigned __int128 C = (unsigned __int128)Ma * Ma;
    int j;  // floor(log2(A / C)), A / C in (1/4, 4)
    if (A >= (C << 1)) j = 1;
    else if (A >= C) j = 0;
    else if ((A << 1) >= C) j = -1;
    else j = -2;
    const int l = 2 * (eT - ea) + j;
    return (l + 1) >> 1;
}

// Statistics of one chunk of one slice: binade histogram of |x|, count of
// nonzero values, max |x|^2, max part, non-finite flag.
// The histogram has one copy per lane of a half-wave (bin * 32 + lane % 32):
// data concentrated in a few binades would otherwise serialise the LDS
// atomics of a wave on one address; this way the two lanes sharing a copy
// are the only possible collision, which the 32-bank LDS pays anyway.
constexpr int kHistCopies = 32;
__global__ __launch_bounds__(256) void k_stats_part(const float2* __restrict__ x, int nn, int chunk,
                                                     int chunks, StatPart* __restrict__ parts,
                                                     const unsigned long long* __restrict__ slice_off)
{
    __shared__ __align__(16) uint32_t hist[kStatsBins * kHistCopies];
    __shared__ unsigned long long s_m2;
    __shared__ uint32_t s_count, s_maxc, s_nonfin;
    const int tid = threadIdx.x, slice = blockIdx.y, copy = tid & (kHistCopies - 1);
    const float2* xs = x + mxd::slice_base(slice_off, slice, (size_t)nn);

    for (int i = tid; i < kStatsBins * kHistCopies / 4; i += blockDim.x) ((uint4*)hist)[i] = make_uint4(0, 0, 0, 0);
    if (tid == 0) { s_m2 = 0; s_count = 0; s_maxc = 0; s_nonfin = 0; }
    __syncthreads();

    unsigned long long mm = 0;
    uint32_t cnt = 0, mc = 0, nf = 0;
    const int beg = blockIdx.x * chunk, end = min(beg + chunk, nn);
    // one element: non-finite flag, largest part, |x|^2 in FP64 (both squares
    // exact, the sum rounded once), count, max and binade histogram of |x|
    auto elem = [&](float re, float im) {
        const uint32_t br = __float_as_uint(re), bi = __float_as_uint(im);
        const uint32_t bad = ((br & 0x7f800000u) == 0x7f800000u) | ((bi & 0x7f800000u) == 0x7f800000u);
        nf |= bad;
        mc = max(mc, max(br & 0x7fffffffu, bi & 0x7fffffffu));
        const double m2 = (double)re * (double)re + (double)im * (double)im;
        const unsigned long long b = (unsigned long long)__double_as_longlong(m2);
        if (!bad && m2 > 0.0) {
            cnt++;
            mm = max(mm, b);
            // floor(log2 |x|) = floor(floor(log2 |x|^2) / 2): sqrt is monotone and
            // correctly rounded, so it never crosses a power of two
            atomicAdd(&hist[(((((int)(b >> 52)) - 1023) >> 1) + kBinOffset) * kHistCopies + copy], 1u);
        }
    };
    if (((end - beg) & 1) == 0 && ((((uintptr_t)(xs + beg)) & 15) == 0)) {
        // two complex values per 16-byte load, four loads in flight per thread
        const float4* x4 = (const float4*)(xs + beg);
        const int nv = (end - beg) >> 1;
        for (int base = 0; base < nv; base += 4 * (int)blockDim.x) {
            float4 q[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int i = base + u * (int)blockDim.x + tid;
                q[u] = i < nv ? x4[i] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int u = 0; u < 4; u++) {
                elem(q[u].x, q[u].y);
                elem(q[u].z, q[u].w);
            }
        }
    } else {
        for (int i = beg + tid; i < end; i += blockDim.x) elem(xs[i].x, xs[i].y);
    }
    // reduced over the wave first: one LDS atomic per wave and value instead
    // of 64 on one address
    for (int o = 32; o; o >>= 1) {
        mm = max(mm, (unsigned long long)__shfl_xor((long long)mm, o, 64));
        cnt += (uint32_t)__shfl_xor((int)cnt, o, 64);
        mc = max(mc, (uint32_t)__shfl_xor((int)mc, o, 64));
        nf |= (uint32_t)__shfl_xor((int)nf, o, 64);
    }
    if ((tid & 63) == 0) {
        atomicMax(&s_m2, mm);
        atomicAdd(&s_count, cnt);
        atomicMax(&s_maxc, mc);
        atomicOr(&s_nonfin, nf);
    }
    __syncthreads();

    StatPart* pt = parts + (size_t)slice * chunks + blockIdx.x;
    // sum the copies of bin i four at a time, the quads in the order q ^ i so
    // a wave's reads fall in different banks (one address operation per read)
    constexpr int NQ = kHistCopies / 4;
    for (int i = tid; i < kStatsBins; i += blockDim.x) {
        const uint32_t a0 = (uint32_t)(i * kHistCopies * 4) | ((uint32_t)(i & (NQ - 1)) << 4);
        uint32_t h = 0;
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            const uint4 u = *(const uint4*)((const char*)hist + (a0 ^ ((uint32_t)q << 4)));
            h += u.x + u.y + u.z + u.w;
        }
        pt->hist[i] = h;
    }
    if (tid == 0) {
        pt->max_m2 = s_m2;
        pt->count = s_count;
        pt->max_comp = s_maxc;
        pt->nonfinite = s_nonfin;
        pt->emin = 0;
        pt->emax = 0;
    }
}

// Shared state of Alg. 1 for one slice, worked on by one 256-thread work-group.
struct Alg1Smem {
    uint32_t hist[kStatsBins];        // nonzero finite |x| per binade floor(log2 |x|) + kBinOffset
    unsigned long long m2, lo_max, hi_min, m2_cut;
    uint32_t count, maxc, nonfin, below;
    int refine, thresh, bin_lo, bin_hi, emin, emax;
    double tp;
    uint32_t wave[16];
    int32_t k, st;                    // result: prescale exponent and status
};

// Clear the statistics (every thread; the caller synchronises afterwards).
__device__ void alg1_init(Alg1Smem& S)
{
    if (threadIdx.x == 0) {
        S.m2 = 0; S.count = 0; S.maxc = 0; S.nonfin = 0; S.refine = 0; S.thresh = 0;
        S.emin = 0; S.emax = 0; S.bin_lo = -1; S.bin_hi = -1; S.k = 0; S.st = 0;
    }
    for (int i = threadIdx.x; i < kStatsBins; i += blockDim.x) S.hist[i] = 0;
}

// Alg. 1 from complete statistics in S (hist, count, m2, maxc, nonfin):
// the tau-percentile's order statistics located in the histogram, refined
// exactly from the slice xs[0..nn) when needed, then k = clip(max(k1, k2)).
// Every thread of the work-group (64 to 1024 threads) calls it; S.k and S.st
// hold the result for all of them on return.
__device__ void alg1_finish(Alg1Smem& S, const float2* __restrict__ xs, int nn, const PrescaleArgs& pa)
{
#pragma clang fp contract(off)
    const int tid = threadIdx.x;
    const uint32_t n = S.count;
    const double pos = ((double)(n ? n - 1 : 0) * pa.tau) / 100.0;
    long long ri = (long long)floor(pos);
    if (n && ri > (long long)n - 1) ri = (long long)n - 1;
    const double fr = pos - (double)ri;
    if (n && !S.nonfin) {
        // binades holding the order statistics ri and ri + 1 (S[n] := S[n-1]):
        // the bin b with (count below b) <= r < (count up to b).  Each thread
        // owns bpt consecutive bins; their counts are prefix-summed over the
        // work-group (wave scans, then the wave totals)
        constexpr int MAXBPT = (kStatsBins + 63) / 64;
        const int bpt = ((int)kStatsBins + (int)blockDim.x - 1) / (int)blockDim.x;
        const long long r1 = (ri + 1 < (long long)n) ? ri + 1 : ri;
        const int b0 = tid * bpt;
        uint32_t h[MAXBPT], mine = 0;
        for (int j = 0; j < MAXBPT; j++) {
            h[j] = (j < bpt && b0 + j < kStatsBins) ? S.hist[b0 + j] : 0u;
            mine += h[j];
        }
        uint32_t incl = mine;                        // inclusive scan within the wave
        const int lane = tid & 63, wave = tid >> 6;
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t o = __shfl_up(incl, d, 64);
            if (lane >= d) incl += o;
        }
        if (lane == 63) S.wave[wave] = incl;
        __syncthreads();
        uint32_t below = incl - mine;                // counts of all lower bins
        for (int w = 0; w < wave; w++) below += S.wave[w];
        long long cum = below;
        for (int j = 0; j < MAXBPT; j++) {
            if (cum <= ri && ri < cum + (long long)h[j]) S.bin_lo = b0 + j;
            if (cum <= r1 && r1 < cum + (long long)h[j]) S.bin_hi = b0 + j;
            cum += h[j];
        }
    }
    __syncthreads();
    // Alg. 1's tail floor: k2 = the smallest k with max(p, 1e-30) 2^k >= tau_min,
    // i.e. min(k2(p), k2(1e-30)).  With p = fp 2^ep and tau_min = ft 2^et
    // (frexp mantissas in [1/2, 1)), k2(p) = et - ep + (fp < ft).  The binade of
    // p gives ep; fp < ft is needed only when tau_min is not a power of two.
    int et;
    const double ft = frexp(pa.tau_min, &et);
    if (tid == 0 && n && !S.nonfin) {
        S.refine = (S.bin_lo != S.bin_hi) && (fr != 0.0);
        S.thresh = !S.refine && ft != 0.5;
        S.lo_max = 0;
        S.hi_min = ~0ull;
        S.below = 0;
        S.m2_cut = 0;
        if (S.thresh) {
            // p lies in binade S.bin_lo; T' = ft 2^ep is the threshold in it, and
            // m = RN(sqrt(m2)) < T' iff m2 < the smallest FP64 x with
            // RN(sqrt(x)) >= T' (sqrt and rounding are monotone)
            const double tp = ldexp(ft, S.bin_lo - kBinOffset + 1);
            double xq = tp * tp;
            if (__dsqrt_rn(xq) >= tp) {
                for (int it = 0; it < 64; it++) {
                    const double y = __longlong_as_double(__double_as_longlong(xq) - 1);
                    if (__dsqrt_rn(y) >= tp) xq = y;
                    else break;
                }
            } else {
                for (int it = 0; it < 64 && __dsqrt_rn(xq) < tp; it++)
                    xq = __longlong_as_double(__double_as_longlong(xq) + 1);
            }
            S.m2_cut = (unsigned long long)__double_as_longlong(xq);
            S.tp = tp;
        }
    }
    __syncthreads();
    if (S.refine) {
        // the two order statistics sit in different binades: S[ri] is the largest
        // value of the lower one and S[ri+1] the smallest of the upper one
        for (int i = tid; i < nn; i += blockDim.x) {
            const float2 v = xs[i];
            const double m2 = (double)v.x * (double)v.x + (double)v.y * (double)v.y;
            const unsigned long long b = (unsigned long long)__double_as_longlong(m2);
            if (m2 > 0.0) {
                const int bin = ((((int)(b >> 52)) - 1023) >> 1) + kBinOffset;
                if (bin == S.bin_lo) atomicMax(&S.lo_max, b);
                if (bin == S.bin_hi) atomicMin(&S.hi_min, b);
            }
        }
        __syncthreads();
    } else if (S.thresh) {
        // count the values below T', with the largest below and the smallest
        // at or above it (the two order statistics when T' falls between them)
        const unsigned long long cut = S.m2_cut;
        uint32_t below = 0;
        for (int i = tid; i < nn; i += blockDim.x) {
            const float2 v = xs[i];
            const double m2 = (double)v.x * (double)v.x + (double)v.y * (double)v.y;
            const unsigned long long b = (unsigned long long)__double_as_longlong(m2);
            if (m2 > 0.0) {
                if (b < cut) {
                    below++;
                    atomicMax(&S.lo_max, b);
                } else {
                    atomicMin(&S.hi_min, b);
                }
            }
        }
        atomicAdd(&S.below, below);
        __syncthreads();
    }
    if (tid == 0) {
        int32_t k = 0, st = 0;
        if (S.nonfin) {
            st = -4;  // MXFFT_ENONFINITE
        } else if (n) {
            const double amax = __dsqrt_rn(__longlong_as_double((long long)S.m2));
            const int k1 = round_log2_ratio(pa.target, amax > 1e-30 ? amax : 1e-30);
            // k2(v) for v > 0
            auto k2_of = [&](double v) -> long long {
                int ev;
                const double fv = frexp(v, &ev);
                return (long long)et - ev + (fv < ft ? 1 : 0);
            };
            long long k2p;
            if (S.refine) {
                const double lo = __dsqrt_rn(__longlong_as_double((long long)S.lo_max));
                const double hi = __dsqrt_rn(__longlong_as_double((long long)S.hi_min));
                const double d = hi - lo;
                const double fd = fr * d;
                k2p = k2_of(lo + fd);
            } else {
                // p in binade lp: fp >= 1/2 >= ft for a power-of-two tau_min
                const int lp = S.bin_lo - kBinOffset;
                bool under = false;  // p < T' (i.e. fp < ft)
                if (S.thresh) {
                    const long long c = S.below;
                    const long long r1 = (ri + 1 < (long long)n) ? ri + 1 : ri;
                    if (fr == 0.0 || r1 == ri) {
                        under = c >= ri + 1;             // p = S[ri]
                    } else if (c <= ri) {
                        under = false;                   // T' <= S[ri] <= p
                    } else if (c >= ri + 2) {
                        under = true;                    // p <= S[ri+1] < T'
                    } else {
                        // S[ri] < T' <= S[ri+1]: p exactly
                        const double lo = __dsqrt_rn(__longlong_as_double((long long)S.lo_max));
                        const double hi = __dsqrt_rn(__longlong_as_double((long long)S.hi_min));
                        const double d = hi - lo;
                        const double fd = fr * d;
                        under = (lo + fd) < S.tp;
                    }
                }
                k2p = (long long)et - (lp + 1) + (under ? 1 : 0);
            }
            const long long k2 = min(k2p, k2_of(1e-30));
            long long kk = max((long long)k1, k2);
            kk = min(max(kk, (long long)pa.k_min), (long long)pa.k_max);
            k = (int32_t)kk;
            // every component scaled by 2^k must stay finite in FP32
            if (S.maxc) {
                const int e = __builtin_amdgcn_frexp_expf(__uint_as_float(S.maxc)) - 1;
                if ((long long)e + kk > 127) st = -5;  // MXFFT_ERANGE
            }
        }
        S.k = st ? INT32_MIN : k;
        S.st = st;
    }
    __syncthreads();
}

// Alg. 1 for one slice from its chunk statistics (one work-group per slice).
// With kadd given (chunk statistics from the row pass, which ran unscaled):
// also decide whether that row pass stands for the scaled one -- every block
// exponent it used, and that exponent plus kp, inside [kEquivLo, kEquivHi] --
// and list the slice for a redo otherwise.
__global__ __launch_bounds__(256) void k_stats_final(const float2* __restrict__ x, int nn, int chunks,
                                                      const StatPart* __restrict__ parts,
                                                      int32_t* __restrict__ kp, int32_t* __restrict__ slice_status,
                                                      PrescaleArgs pa, int32_t* __restrict__ kadd,
                                                      int32_t* __restrict__ fix_list, int32_t* __restrict__ fix_count,
                                                      int32_t* __restrict__ k_out,
                                                      const unsigned long long* __restrict__ slice_off)
{
    __shared__ Alg1Smem S;
    const int tid = threadIdx.x, slice = blockIdx.x;
    const float2* xs = x + mxd::slice_base(slice_off, slice, (size_t)nn);
    const StatPart* pt = parts + (size_t)slice * chunks;
    alg1_init(S);
    __syncthreads();
    // histograms of all chunks, read as one coalesced sweep of 16-byte loads
    // (several in flight per thread) and summed per bin in LDS
    {
        static_assert(kStatsBins % 4 == 0 && sizeof(StatPart) % 16 == 0, "histograms in 16-byte quads");
        constexpr int QB = kStatsBins / 4;
        const int total = chunks * QB;
        uint32_t cnt = 0;
#pragma unroll 4
        for (int w = tid; w < total; w += blockDim.x) {
            const int c = w / QB, q = w - c * QB;
            const uint4 h = *(const uint4*)&pt[c].hist[4 * q];
            if (h.x) atomicAdd(&S.hist[4 * q], h.x);
            if (h.y) atomicAdd(&S.hist[4 * q + 1], h.y);
            if (h.z) atomicAdd(&S.hist[4 * q + 2], h.z);
            if (h.w) atomicAdd(&S.hist[4 * q + 3], h.w);
            cnt += h.x + h.y + h.z + h.w;
        }
        for (int o = 32; o; o >>= 1) cnt += (uint32_t)__shfl_xor((int)cnt, o, 64);
        if ((tid & 63) == 0) atomicAdd(&S.count, cnt);
    }
    for (int c = tid; c < chunks; c += blockDim.x) {
        atomicMax(&S.m2, pt[c].max_m2);
        atomicMax(&S.maxc, pt[c].max_comp);
        atomicOr(&S.nonfin, pt[c].nonfinite);
        atomicMin(&S.emin, pt[c].emin);
        atomicMax(&S.emax, pt[c].emax);
    }
    __syncthreads();
    alg1_finish(S, xs, nn, pa);
    if (tid == 0) {
        const int32_t k = S.k, st = S.st;
        kp[slice] = k;
        slice_status[slice] = st;
        if (k_out) k_out[slice] = k;
        if (kadd) {
            const bool inside = S.emin >= kEquivLo && S.emax <= kEquivHi && S.emin + (long long)k >= kEquivLo &&
                                S.emax + (long long)k <= kEquivHi;
            if (st == 0 && !inside) {
                kadd[slice] = 0;
                fix_list[atomicAdd(fix_count, 1)] = slice;
            } else {
                kadd[slice] = st ? 0 : k;
            }
        }
    }
}

int stats_chunks(int n, int batch)
{
    const long nn = (long)n * n;
    long want = (4096 + batch - 1) / batch;       // work-groups per slice to fill the chip
    const long most = nn / 8192;                  // at least 8192 elements per chunk
    if (want > most) want = most;
    if (want < 1) want = 1;
    long c = 1;
    while (c * 2 <= want) c *= 2;                 // a power of two divides n^2
    return (int)c;
}

size_t stats_parts(int n, int max_batch)
{
    (void)n;
    return (size_t)max_batch + 4096;              // batch * chunks <= batch + 4096
}

hipError_t launch_stats(const float2* x, int n, int batch, StatPart* parts, int32_t* kp,
                        int32_t* slice_status, const PrescaleArgs& pa, const unsigned long long* slice_off,
                        int chunks, hipStream_t s)
{
    const int nn = n * n;
    if (chunks <= 0 || nn % chunks != 0) chunks = stats_chunks(n, batch);
    hipLaunchKernelGGL(k_stats_part, dim3(chunks, batch), dim3(256), 0, s, x, nn, nn / chunks, chunks, parts,
                       slice_off);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_stats_final, dim3(batch), dim3(256), 0, s, x, nn, chunks, parts, kp, slice_status, pa,
                       nullptr, nullptr, nullptr, nullptr, slice_off);
    return hipGetLastError();
}

hipError_t launch_stats_final(const float2* x, int n, int batch, int chunks, const StatPart* parts, int32_t* kp,
                              int32_t* slice_status, const PrescaleArgs& pa, int32_t* kadd, int32_t* fix_list,
                              int32_t* fix_count, int32_t* k_out, const unsigned long long* slice_off,
                              hipStream_t s)
{
    hipLaunchKernelGGL(k_stats_final, dim3(batch), dim3(256), 0, s, x, n * n, chunks, parts, kp, slice_status, pa,
                       kadd, fix_list, fix_count, k_out, slice_off);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// One radix-2 pass over lines held in LDS
// ---------------------------------------------------------------------------

// Element values (qx, qy) of v in a block of shared exponent E (the encode of
// EncodeBlockMX, by the scaled conversions after the saturating clamp).
template <int F>
__device__ __forceinline__ void mx_encode_value(float2 v, int E, float& qx, float& qy)
{
    const mxd::Blk b = mxd::blk<F>(E);
    const float2 c = mxd::clamp2(mxd::mulp<F>(v, b.pre), mxd::mulp1<F>(mxd::lim_of<F>(E), b.pre));
    const float2 q = mxd::dec2<F, false>(mxd::enc2<F, false>(0u, c.x, c.y, b.s), mxd::unit_scale<F>());
    qx = q.x;
    qy = q.y;
}

// Alg. 2's product of one butterfly in mantissa space: v encoded with its
// block's exponent Ev (clamped first: the scaled conversions do not
// saturate), its element values times the twiddle's (products of 8-bit and
// 6-bit elements are exact in FP32).
template <int F>
__device__ __forceinline__ float2 mx_mant_product(float2 w, float2 v, int Ev)
{
    const mxd::Blk bv = mxd::blk<F>(Ev);
    const float2 vc = mxd::clamp2(mxd::mulp<F>(v, bv.pre), mxd::mulp1<F>(mxd::lim_of<F>(Ev), bv.pre));
    const float2 y = mxd::dec2<F, false>(mxd::enc2<F, false>(0u, vc.x, vc.y, bv.s), mxd::unit_scale<F>());
    return make_float2(w.x * y.x - w.y * y.y, w.x * y.y + w.y * y.x);
}

// The renormalised product block's value: the mantissa-space product q
// encoded with 2^kr (no clamp needed) and decoded with its scale 2^Eo, or (a
// scale outside the E8M0 range) decoded and then ldexp.
template <int F>
__device__ __forceinline__ float2 mx_product_value(float2 q, int kr, int Eo)
{
    constexpr int OFF = mxd::Hw<F>::OFF;
    const uint32_t cp = mxd::enc2<F, false>(0u, q.x, q.y, mxd::e8(kr + OFF));
    if ((OFF == 0) ? (Eo >= -127) : (Eo + OFF >= -127 && Eo + OFF <= 127))
        return mxd::dec2<F, false>(cp, mxd::e8(Eo + OFF));
    const float2 d = mxd::dec2<F, false>(cp, mxd::unit_scale<F>());
    return make_float2(ldexpf(d.x, Eo), ldexpf(d.y, Eo));
}

// tr (MX, nullable): receives the block's (E_v, k_r, E_out) of Alg. 2.
template <int MODE>
__device__ __forceinline__ void butterfly(const LineArgs& a, int s, int j, float2 u, float2 v,
                                          float2& y0, float2& y1, int32_t* tr = nullptr)
{
    const int h = 1 << (s - 1);
    float2 w = a.tw[h - 1 + j];
    if (a.inverse) w.y = -w.y;
    float pr, pi;
    if constexpr (MODE == MODE_FP32) {
        pr = w.x * v.x - w.y * v.y;
        pi = w.x * v.y + w.y * v.x;
    } else if constexpr (MODE == MODE_FP16 || MODE == MODE_BF16) {
        // 16-bit form: v rounded to the format, each product and each sum of
        // the complex product rounded to the format (twiddles are format values)
        const float vr = mxd::round16<MODE>(v.x), vi = mxd::round16<MODE>(v.y);
        const float rr = mxd::mul16<MODE>(w.x, vr), ii = mxd::mul16<MODE>(w.y, vi);
        const float ri = mxd::mul16<MODE>(w.x, vi), ir = mxd::mul16<MODE>(w.y, vr);
        pr = mxd::add16<MODE>(rr, -ii);
        pi = mxd::add16<MODE>(ri, ir);
    } else {
        constexpr int F = MODE;
        // twiddle block: min(cb, h) consecutive j share one exponent
        const int Ew = a.tw_exp[a.tw_exp_off[s] + (a.cb <= h ? (j >> a.logcb) : 0)];
        // operand v: EncodeBlockMX over the cb butterflies of this block (cb
        // lanes), element values from the scaled conversions (clamped first:
        // they do not saturate)
        const uint32_t av = mxd::group_max(max(mxd::abs_key(v.x), mxd::abs_key(v.y)), a.cb);
        const int Ev = mxd::block_exp<F>(av);
        const float2 q = mx_mant_product<F>(w, v, Ev);
        // renormalise the product block when it exceeds the element range
        const uint32_t ap = mxd::group_max(max(mxd::abs_key(q.x), mxd::abs_key(q.y)), a.cb);
        const int kr = mxd::renorm_exp<F>(ap);
        const int Eo = Ew + Ev + kr;
        if (tr) {
            tr[0] = Ev;
            tr[1] = kr;
            tr[2] = Eo;
        }
        const float2 p = mx_product_value<F>(q, kr, Eo);
        pr = p.x;
        pi = p.y;
    }
    y0 = make_float2(u.x + pr, u.y + pi);
    y1 = make_float2(u.x - pr, u.y - pi);
}

// Blocks of more than 64 butterflies (B > 128): a block spans several waves
// (or several steps of a thread's loop), so its maxima go through LDS.  At
// most R N / 128 <= 64 blocks per work-group (R N <= 8192).
constexpr int kBigBlocks = 64;

// The stages of a pass with blocks of more than 64 butterflies: per stage,
// (1) the v maxima of every block by LDS atomics, (2) each butterfly's
// mantissa-space product, stored over its v, and the product maxima, (3) the
// renormalised products and u +/- p.  The same arithmetic as butterfly();
// every barrier is outside the per-thread loops.
template <int MODE>
__device__ void big_block_stages(const LineArgs& a, float2* lds, uint32_t (*s_bm)[kBigBlocks], int slice, int line0,
                                 int R)
{
    constexpr int F = MODE;
    const int N = a.n, logn = a.logn, tid = threadIdx.x, half = N >> 1, nbf = (R * N) >> 1;
    const int nblk = nbf >> a.logcb;
    for (int s = 1; s <= logn; s++) {
        const int h = 1 << (s - 1);
        auto where = [&](int b, int& iu, int& iv, int& j, int& t, int& r) {
            r = b >> (logn - 1);
            t = b & (half - 1);
            const int g = t >> (s - 1);
            j = t & (h - 1);
            iu = r * N + (g << s) + j;
            iv = iu + h;
        };
        for (int i = tid; i < nblk; i += blockDim.x) {
            s_bm[0][i] = 0u;
            s_bm[1][i] = 0u;
        }
        __syncthreads();
        for (int b = tid; b < nbf; b += blockDim.x) {
            int iu, iv, j, t, r;
            where(b, iu, iv, j, t, r);
            const float2 v = lds[iv];
            atomicMax(&s_bm[0][b >> a.logcb], max(mxd::abs_key(v.x), mxd::abs_key(v.y)));
        }
        __syncthreads();
        for (int b = tid; b < nbf; b += blockDim.x) {
            int iu, iv, j, t, r;
            where(b, iu, iv, j, t, r);
            float2 w = a.tw[h - 1 + j];
            if (a.inverse) w.y = -w.y;
            const float2 q = mx_mant_product<F>(w, lds[iv], mxd::block_exp<F>(s_bm[0][b >> a.logcb]));
            lds[iv] = q;
            atomicMax(&s_bm[1][b >> a.logcb], max(mxd::abs_key(q.x), mxd::abs_key(q.y)));
        }
        __syncthreads();
        for (int b = tid; b < nbf; b += blockDim.x) {
            int iu, iv, j, t, r;
            where(b, iu, iv, j, t, r);
            const int Ew = a.tw_exp[a.tw_exp_off[s] + (a.cb <= h ? (j >> a.logcb) : 0)];
            const int Ev = mxd::block_exp<F>(s_bm[0][b >> a.logcb]);
            const int kr = mxd::renorm_exp<F>(s_bm[1][b >> a.logcb]);
            const int Eo = Ew + Ev + kr;
            if (a.cap_trace && a.axis == 0 && line0 + r == 0 && (t & (a.cb - 1)) == 0) {
                int32_t* tr = a.cap_trace + ((size_t)slice * logn + (s - 1)) * 3 * (half >> a.logcb) + 3 * (t >> a.logcb);
                tr[0] = Ev;
                tr[1] = kr;
                tr[2] = Eo;
            }
            const float2 p = mx_product_value<F>(lds[iv], kr, Eo);
            const float2 u = lds[iu];
            lds[iu] = make_float2(u.x + p.x, u.y + p.y);
            lds[iv] = make_float2(u.x - p.x, u.y - p.y);
        }
        __syncthreads();
    }
}

template <int MODE>
__global__ __launch_bounds__(256) void k_lines(LineArgs a)
{
    extern __shared__ float2 lds[];
    __shared__ uint32_t s_bm[2][kBigBlocks];   // block maxima of v and of the products (B > 128)
    const int N = a.n, logn = a.logn, R = a.lines, tid = threadIdx.x;
    const int slice = blockIdx.y;
    const size_t sbase = mxd::slice_base(a.slice_off, slice, (size_t)N * N);       // slice in src
    const size_t dbase = mxd::slice_base(a.slice_off_out, slice, (size_t)N * N);   // slice in dst
    const size_t cbase = (size_t)slice * N * N;                               // slice in the capture
    const int line0 = blockIdx.x * R;
    int kp = a.kp ? a.kp[slice] : 0;
    if (kp == INT32_MIN) kp = 0;  // failed slice: output undefined, keep it finite-safe
    const int kin = a.kin_mul * kp, kout = a.kout_mul * kp + a.kout_add;
    if (a.k_out && blockIdx.x == 0 && tid == 0) a.k_out[slice] = a.kp ? a.kp[slice] : 0;
    const int total = R * N;

    // load (coalesced along the contiguous axis), apply the prescale
    for (int idx = tid; idx < total; idx += blockDim.x) {
        int r, e;
        size_t g;
        if (a.axis == 0) {
            r = idx >> logn;
            e = idx & (N - 1);
            g = sbase + (size_t)(line0 + r) * N + e;
        } else {
            e = idx / R;
            r = idx & (R - 1);
            g = sbase + (size_t)e * N + line0 + r;
        }
        float2 v = a.src[g];
        v.x = ldexpf(v.x, kin);
        v.y = ldexpf(v.y, kin);
        lds[r * N + e] = v;
    }
    __syncthreads();

    if constexpr (MODE == MODE_FP16 || MODE == MODE_BF16) {
        // pass input rounded to the format
        for (int idx = tid; idx < total; idx += blockDim.x) {
            const float2 v = lds[idx];
            lds[idx] = make_float2(mxd::round16<MODE>(v.x), mxd::round16<MODE>(v.y));
        }
        __syncthreads();
    } else if constexpr (MODE != MODE_FP32) {
        if (a.encode) {
            // pass input: blocks of cb consecutive values along the line
            const bool big = a.cb > 64;
            if (big) {
                for (int i = tid; i < (total >> a.logcb); i += blockDim.x) s_bm[0][i] = 0u;
                __syncthreads();
                for (int idx = tid; idx < total; idx += blockDim.x) {
                    const float2 v = lds[idx];
                    atomicMax(&s_bm[0][idx >> a.logcb], max(mxd::abs_key(v.x), mxd::abs_key(v.y)));
                }
                __syncthreads();
            }
            for (int idx = tid; idx < total; idx += blockDim.x) {
                float2 v = lds[idx];
                const uint32_t am = big ? s_bm[0][idx >> a.logcb]
                                        : mxd::group_max(max(mxd::abs_key(v.x), mxd::abs_key(v.y)), a.cb);
                const int E = mxd::block_exp<MODE>(am);
                float qx, qy;
                mx_encode_value<MODE>(v, E, qx, qy);
                if (a.cap_mant && a.axis == 1) {
                    // debug capture of the column pass input: line r is column
                    // line0 + r, element e its row
                    const int r = idx >> logn, e = idx & (N - 1), col = line0 + r;
                    a.cap_mant[cbase + (size_t)e * N + col] = make_float2(qx, qy);
                    if ((e & (a.cb - 1)) == 0)
                        a.cap_exp[((size_t)slice * N + col) * (N >> a.logcb) + (e >> a.logcb)] = E;
                }
                v.x = ldexpf(qx, E);
                v.y = ldexpf(qy, E);
                lds[idx] = v;
            }
            __syncthreads();
        }
    }

    // bit reversal (decimation in time)
    for (int idx = tid; idx < total; idx += blockDim.x) {
        const int r = idx >> logn, e = idx & (N - 1);
        const int rev = (int)(__brev((unsigned)e) >> (32 - logn));
        if (rev > e) {
            const float2 t = lds[r * N + e];
            lds[r * N + e] = lds[r * N + rev];
            lds[r * N + rev] = t;
        }
    }
    __syncthreads();

    const int half = N >> 1, nbf = total >> 1;
    bool big = false;
    if constexpr (MODE != MODE_FP32 && MODE != MODE_FP16 && MODE != MODE_BF16) big = a.cb > 64;
    if (big) {
        if constexpr (MODE != MODE_FP32 && MODE != MODE_FP16 && MODE != MODE_BF16)
            big_block_stages<MODE>(a, lds, s_bm, slice, line0, R);
    } else {
        for (int s = 1; s <= logn; s++) {
            const int h = 1 << (s - 1);
            for (int b = tid; b < nbf; b += blockDim.x) {
                const int r = b >> (logn - 1);
                const int t = b & (half - 1);
                const int g = t >> (s - 1), j = t & (h - 1);
                const int iu = r * N + (g << s) + j, iv = iu + h;
                float2 y0, y1;
                // debug capture: the block exponents of line 0 of the row pass
                int32_t* tr = nullptr;
                if (a.cap_trace && a.axis == 0 && line0 + r == 0 && (t & (a.cb - 1)) == 0)
                    tr = a.cap_trace + ((size_t)slice * logn + (s - 1)) * 3 * (half >> a.logcb) + 3 * (t >> a.logcb);
                butterfly<MODE>(a, s, j, lds[iu], lds[iv], y0, y1, tr);
                lds[iu] = y0;
                lds[iv] = y1;
            }
            __syncthreads();
        }
    }

    for (int idx = tid; idx < total; idx += blockDim.x) {
        int r, e;
        size_t g;
        if (a.axis == 0) {
            r = idx >> logn;
            e = idx & (N - 1);
            g = dbase + (size_t)(line0 + r) * N + e;
        } else {
            e = idx / R;
            r = idx & (R - 1);
            g = dbase + (size_t)e * N + line0 + r;
        }
        float2 v = lds[r * N + e];
        if constexpr (MODE == MODE_FP16 || MODE == MODE_BF16) {
            // the 16-bit form ends each pass rounded to the format (a column
            // pass input would be rounded anyway; the output must be)
            v = make_float2(mxd::round16<MODE>(v.x), mxd::round16<MODE>(v.y));
        }
        v.x = ldexpf(v.x, kout);
        v.y = ldexpf(v.y, kout);
        a.dst[g] = v;
    }
}

// Debug capture from the register-resident MX intermediate.  Its layout:
// codes[slice][16-column group][row][8 words], the word of the group's
// columns 2w, 2w + 1 at w ^ (((row >> 2) & 3) << 1), holding (re, im) of the
// even column in its low half and of the odd one in its high half;
// exps[slice][row block][column] as E + 127 (E offset by -kadd[slice] when
// the row pass ran on the unscaled input).  One thread per (slice, row,
// column pair).  MXFP6 codes travel as FP8 codes of the value times 2^-OFF.
typedef float capf2 __attribute__((ext_vector_type(2)));
__global__ void k_capture_mx(int fmt8, int off, int n, int logcb, const uint32_t* __restrict__ codes,
                             const uint8_t* __restrict__ exps, const int32_t* __restrict__ kadd, long pairs,
                             float2* __restrict__ mant, int32_t* __restrict__ cap_exp)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= pairs) return;
    const int half = n >> 1;
    const long slice = i / ((long)n * half);
    const int rem = (int)(i - slice * (long)n * half);
    const int row = rem / half, c2 = 2 * (rem - row * half);
    const uint32_t w = codes[(size_t)slice * n * n / 2 + ((size_t)(c2 >> 4) * n + row) * 8 +
                             (((c2 & 15) >> 1) ^ (((row >> 2) & 3) << 1))];
    const float us = __uint_as_float((uint32_t)(off + 127) << 23);   // 2^OFF
    capf2 lo, hi;
    if (fmt8 == 0) {
        lo = __builtin_amdgcn_cvt_scalef32_pk_f32_fp8(w, us, false);
        hi = __builtin_amdgcn_cvt_scalef32_pk_f32_fp8(w, us, true);
    } else {
        lo = __builtin_amdgcn_cvt_scalef32_pk_f32_bf8(w, us, false);
        hi = __builtin_amdgcn_cvt_scalef32_pk_f32_bf8(w, us, true);
    }
    float2* m = mant + ((size_t)slice * n + row) * n + c2;
    m[0] = make_float2(lo.x, lo.y);
    m[1] = make_float2(hi.x, hi.y);
    if ((row & ((1 << logcb) - 1)) == 0) {
        const int nb = n >> logcb, rb = row >> logcb;
        const int add = kadd ? kadd[slice] : 0;
        const uint8_t* ex = exps + ((size_t)slice * nb + rb) * n + c2;
        int32_t* o = cap_exp + ((size_t)slice * n + c2) * nb + rb;
        o[0] = (int32_t)ex[0] - 127 + add;
        o[nb] = (int32_t)ex[1] - 127 + add;
    }
}

hipError_t launch_capture_mx(int mode, int n, int cb, const uint32_t* codes, const uint8_t* exps,
                             const int32_t* kadd, int batch, float2* mant, int32_t* cap_exp, hipStream_t s)
{
    const int fmt8 = (mode == MODE_E5M2 || mode == MODE_E3M2) ? 1 : 0;
    const int off = (mode == MODE_E2M3) ? 6 : (mode == MODE_E3M2) ? 12 : 0;
    int logcb = 0;
    while ((1 << logcb) < cb) logcb++;
    const long pairs = (long)batch * n * (n / 2);
    hipLaunchKernelGGL(k_capture_mx, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, s, fmt8, off, n, logcb,
                       codes, exps, kadd, pairs, mant, cap_exp);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Single-launch transform of small slices (n <= 64): one work-group per slice
// holds the slice in LDS (row pitch n + 1, so column accesses spread over the
// banks) and runs Alg. 1, every 1D pass (rows, then columns; both halves of a
// round trip) and the output scaling with the same per-element arithmetic as
// the line kernels.
// ---------------------------------------------------------------------------

constexpr int kSmallMaxN = kSmallN;

// One 1D pass over the n lines of the slice in buf: rows (element e of line r
// at r * pitch + e) or columns (at e * pitch + r).  encode: MX-encode the
// pass input (blocks of cb consecutive values along the line); the 16-bit
// forms round it to the format instead, and round the pass result.  With
// cap_mant set, the encoded input's element values and block exponents are
// recorded (debug capture of the forward's column pass).
template <int MODE>
__device__ void small_pass(const LineArgs& a, float2* buf, bool cols, bool encode, float2* cap_mant,
                           int32_t* cap_exp, int32_t* cap_trace, int slice)
{
    const int N = a.n, logn = a.logn, tid = threadIdx.x, total = N * N, pitch = N + 1;
    auto at = [&](int r, int e) -> float2& { return cols ? buf[e * pitch + r] : buf[r * pitch + e]; };
    if constexpr (MODE == MODE_FP16 || MODE == MODE_BF16) {
        for (int idx = tid; idx < total; idx += blockDim.x) {
            float2& v = at(idx >> logn, idx & (N - 1));
            v = make_float2(mxd::round16<MODE>(v.x), mxd::round16<MODE>(v.y));
        }
        __syncthreads();
    } else if constexpr (MODE != MODE_FP32) {
        if (encode) {
            for (int idx = tid; idx < total; idx += blockDim.x) {
                const int r = idx >> logn, e = idx & (N - 1);
                float2 v = at(r, e);
                const uint32_t am = mxd::group_max(max(mxd::abs_key(v.x), mxd::abs_key(v.y)), a.cb);
                const int E = mxd::block_exp<MODE>(am);
                float qx, qy;
                mx_encode_value<MODE>(v, E, qx, qy);
                if (cap_mant) {
                    // line r is column r, element e its row
                    cap_mant[((size_t)slice * N + e) * N + r] = make_float2(qx, qy);
                    if ((e & (a.cb - 1)) == 0)
                        cap_exp[((size_t)slice * N + r) * (N >> a.logcb) + (e >> a.logcb)] = E;
                }
                at(r, e) = make_float2(ldexpf(qx, E), ldexpf(qy, E));
            }
            __syncthreads();
        }
    }
    // bit reversal (decimation in time)
    for (int idx = tid; idx < total; idx += blockDim.x) {
        const int r = idx >> logn, e = idx & (N - 1);
        const int rev = (int)(__brev((unsigned)e) >> (32 - logn));
        if (rev > e) {
            const float2 t = at(r, e);
            at(r, e) = at(r, rev);
            at(r, rev) = t;
        }
    }
    __syncthreads();
    const int half = N >> 1, nbf = total >> 1;
    for (int st = 1; st <= logn; st++) {
        const int h = 1 << (st - 1);
        for (int b = tid; b < nbf; b += blockDim.x) {
            const int r = b >> (logn - 1);
            const int t = b & (half - 1);
            const int g = t >> (st - 1), j = t & (h - 1);
            const int iu = (g << st) + j, iv = iu + h;
            float2 y0, y1;
            int32_t* tr = nullptr;   // debug capture: the block exponents of line 0
            if (cap_trace && r == 0 && (t & (a.cb - 1)) == 0)
                tr = cap_trace + ((size_t)slice * logn + (st - 1)) * 3 * (half >> a.logcb) + 3 * (t >> a.logcb);
            butterfly<MODE>(a, st, j, at(r, iu), at(r, iv), y0, y1, tr);
            at(r, iu) = y0;
            at(r, iv) = y1;
        }
        __syncthreads();
    }
    if constexpr (MODE == MODE_FP16 || MODE == MODE_BF16) {
        for (int idx = tid; idx < total; idx += blockDim.x) {
            float2& v = at(idx >> logn, idx & (N - 1));
            v = make_float2(mxd::round16<MODE>(v.x), mxd::round16<MODE>(v.y));
        }
        __syncthreads();
    }
}

template <int MODE>
__global__ __launch_bounds__(1024) void k_small(SmallArgs g)
{
    extern __shared__ float2 buf[];     // n x (n + 1) complex values
    __shared__ Alg1Smem S;
    // the plan's twiddles (n - 1 values) and MX twiddle block exponents, read
    // by every stage: staged in LDS once
    __shared__ float2 s_tw[kSmallMaxN];
    __shared__ int32_t s_twe[kSmallMaxN];
    const int tid = threadIdx.x, slice = blockIdx.x, N = g.a.n, logn = g.a.logn, nn = N * N, pitch = N + 1;
    const float2* xs = g.a.src + mxd::slice_base(g.a.slice_off, slice, (size_t)nn);
    constexpr bool MXM = MODE != MODE_FP32 && MODE != MODE_FP16 && MODE != MODE_BF16;
    if (N >= 2) {
        for (int i = tid; i < N - 1; i += blockDim.x) s_tw[i] = g.a.tw[i];
        if constexpr (MXM) {
            // stage s holds (n/2 of the last stage) / min(cb, h) exponents from tw_exp_off[s]
            const int h = N >> 1, ne = g.a.tw_exp_off[logn] + h / min(g.a.cb, h);
            for (int i = tid; i < ne; i += blockDim.x) s_twe[i] = g.a.tw_exp[i];
        }
    }
    if (g.stats) {
        alg1_init(S);
        __syncthreads();
    }
    // load; Alg. 1's statistics on the way (|x|^2 in FP64, binade histogram,
    // maximum, largest part, non-finite check)
    {
        unsigned long long mm = 0;
        uint32_t cnt = 0, mc = 0, nf = 0;
        for (int i = tid; i < nn; i += blockDim.x) {
            const float2 v = xs[i];
            buf[(i >> logn) * pitch + (i & (N - 1))] = v;
            if (g.stats) {
                const uint32_t br = __float_as_uint(v.x), bi = __float_as_uint(v.y);
                const uint32_t bad = ((br & 0x7f800000u) == 0x7f800000u) | ((bi & 0x7f800000u) == 0x7f800000u);
                nf |= bad;
                mc = max(mc, max(br & 0x7fffffffu, bi & 0x7fffffffu));
                const double m2 = (double)v.x * (double)v.x + (double)v.y * (double)v.y;
                const unsigned long long b = (unsigned long long)__double_as_longlong(m2);
                if (!bad && m2 > 0.0) {
                    cnt++;
                    mm = max(mm, b);
                    atomicAdd(&S.hist[((((int)(b >> 52)) - 1023) >> 1) + kBinOffset], 1u);
                }
            }
        }
        if (g.stats) {
            // reduced over the wave first: one LDS atomic per wave and value
            // instead of 64 on one address
            for (int o = 32; o; o >>= 1) {
                mm = max(mm, (unsigned long long)__shfl_xor((long long)mm, o, 64));
                cnt += (uint32_t)__shfl_xor((int)cnt, o, 64);
                mc = max(mc, (uint32_t)__shfl_xor((int)mc, o, 64));
                nf |= (uint32_t)__shfl_xor((int)nf, o, 64);
            }
            if ((tid & 63) == 0) {
                atomicMax(&S.m2, mm);
                atomicAdd(&S.count, cnt);
                atomicMax(&S.maxc, mc);
                atomicOr(&S.nonfin, nf);
            }
        }
    }
    __syncthreads();
    int k = 0;
    if (g.stats) {
        alg1_finish(S, xs, nn, g.pa);
        k = S.k;
        if (tid == 0) {
            if (g.kp) g.kp[slice] = k;
            if (g.status) g.status[slice] = S.st;
            if (g.a.k_out) g.a.k_out[slice] = k;
        }
    } else {
        k = g.k_in ? g.k_in[slice] : 0;
        if (tid == 0 && g.a.k_out) g.a.k_out[slice] = k;
    }
    if (k == INT32_MIN) k = 0;  // failed slice: output undefined, keep it finite-safe
    const int kin = g.kin_mul * k;
    if (kin) {
        for (int i = tid; i < nn; i += blockDim.x) {
            float2& v = buf[(i >> logn) * pitch + (i & (N - 1))];
            v = make_float2(ldexpf(v.x, kin), ldexpf(v.y, kin));
        }
        __syncthreads();
    }
    constexpr bool MX = MXM;
    LineArgs a = g.a;
    a.inverse = g.op == 1;
    if (N >= 2) {
        a.tw = s_tw;
        if constexpr (MX) a.tw_exp = s_twe;
    }
    small_pass<MODE>(a, buf, false, MX, nullptr, nullptr, g.op == 0 ? g.a.cap_trace : nullptr, slice);
    small_pass<MODE>(a, buf, true, MX, g.op == 0 ? g.a.cap_mant : nullptr, g.a.cap_exp, nullptr, slice);
    if (g.op == 2) {
        a.inverse = 1;
        small_pass<MODE>(a, buf, false, MX && !g.raw_inverse_rows, nullptr, nullptr, nullptr, slice);
        small_pass<MODE>(a, buf, true, MX, nullptr, nullptr, nullptr, slice);
    }
    const int kout = g.kout_mul * k + g.kout_add;
    float2* ys = g.a.dst + mxd::slice_base(g.a.slice_off_out, slice, (size_t)nn);
    for (int i = tid; i < nn; i += blockDim.x) {
        const float2 v = buf[(i >> logn) * pitch + (i & (N - 1))];
        ys[i] = make_float2(ldexpf(v.x, kout), ldexpf(v.y, kout));
    }
}

// Threads per work-group of the single-launch kernel (results do not depend
// on it).  While the batch gives a CU at most one slice, 16 waves per slice;
// with more slices per CU, 16 waves shared among the slices a CU holds at
// once (at most 8 per slice), so that each thread runs several butterflies of
// a stage and a barrier spans fewer waves.  Never more than one thread per
// butterfly, never less than one wave.
int small_block(int n, int batch, int cus, int lds_per_cu)
{
    const int bf = n * n / 2;
    const long lds = (long)n * (n + 1) * (long)sizeof(float2);
    const int fit = std::max(1, (int)(lds_per_cu / lds));
    const int per_cu = (batch + std::max(cus, 1) - 1) / std::max(cus, 1);
    int waves = 16 / std::min(std::min(fit, per_cu), 16);
    if (fit > 1 && per_cu > 1) waves = std::min(waves, 8);
    waves = std::max(1, std::min(waves, bf / 64));
    return 64 * waves;
}

hipError_t launch_small(int mode, const SmallArgs& g, int batch, int cus, int lds_per_cu, hipStream_t s)
{
    if (g.a.n > kSmallMaxN) return hipErrorInvalidValue;
    // the slice in LDS with a row pitch of n + 1 (132 KiB at 128^2)
    const dim3 grid(batch), block(small_block(g.a.n, batch, cus, lds_per_cu));
    const size_t lds = (size_t)g.a.n * (g.a.n + 1) * sizeof(float2);
    switch (mode) {
    case MODE_E4M3: hipLaunchKernelGGL(k_small<MODE_E4M3>, grid, block, lds, s, g); break;
    case MODE_E5M2: hipLaunchKernelGGL(k_small<MODE_E5M2>, grid, block, lds, s, g); break;
    case MODE_E2M3: hipLaunchKernelGGL(k_small<MODE_E2M3>, grid, block, lds, s, g); break;
    case MODE_E3M2: hipLaunchKernelGGL(k_small<MODE_E3M2>, grid, block, lds, s, g); break;
    case MODE_FP16: hipLaunchKernelGGL(k_small<MODE_FP16>, grid, block, lds, s, g); break;
    case MODE_BF16: hipLaunchKernelGGL(k_small<MODE_BF16>, grid, block, lds, s, g); break;
    case MODE_FP32: hipLaunchKernelGGL(k_small<MODE_FP32>, grid, block, lds, s, g); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Output quantisation (MXFFT_QUANTIZE_OUTPUT): one thread per (slice, row
// block, column), consecutive threads on consecutive columns, so every row of
// a block is read and written as whole row segments.  The block's exponent
// from its maximum, then each value re-encoded with it (the same encode as
// the passes' input encode).
template <int MODE>
__global__ void k_quantize_out(float2* __restrict__ out, const unsigned long long* __restrict__ off, int n,
                               int logcb, long total)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int cb = 1 << logcb, nb = n >> logcb;
    const long per_slice = (long)nb * n;
    const long slice = i / per_slice;
    const int rem = (int)(i - slice * per_slice), rb = rem / n, col = rem - rb * n;
    float2* y = out + mxd::slice_base(off, slice, (size_t)n * n) + (size_t)rb * cb * n + col;
    uint32_t am = 0;
    for (int r = 0; r < cb; r++) {
        const float2 v = y[(size_t)r * n];
        am = max(am, max(mxd::abs_key(v.x), mxd::abs_key(v.y)));
    }
    const int E = mxd::block_exp<MODE>(am);
    for (int r = 0; r < cb; r++) {
        float qx, qy;
        mx_encode_value<MODE>(y[(size_t)r * n], E, qx, qy);
        y[(size_t)r * n] = make_float2(ldexpf(qx, E), ldexpf(qy, E));
    }
}

hipError_t launch_quantize_out(int mode, float2* out, const unsigned long long* off, int n, int logcb, int batch,
                               hipStream_t s)
{
    const long total = (long)batch * (n >> logcb) * n;
    const dim3 grid((unsigned)((total + 255) / 256)), block(256);
    switch (mode) {
    case MODE_E4M3: hipLaunchKernelGGL(k_quantize_out<MODE_E4M3>, grid, block, 0, s, out, off, n, logcb, total); break;
    case MODE_E5M2: hipLaunchKernelGGL(k_quantize_out<MODE_E5M2>, grid, block, 0, s, out, off, n, logcb, total); break;
    case MODE_E2M3: hipLaunchKernelGGL(k_quantize_out<MODE_E2M3>, grid, block, 0, s, out, off, n, logcb, total); break;
    case MODE_E3M2: hipLaunchKernelGGL(k_quantize_out<MODE_E3M2>, grid, block, 0, s, out, off, n, logcb, total); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

__global__ void k_scatter_k(const int32_t* __restrict__ src, const int32_t* __restrict__ idx,
                            int32_t* __restrict__ dst, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[idx[i]] = src[i];
}

hipError_t launch_scatter_k(const int32_t* src, const int32_t* idx, int32_t* dst, int count, hipStream_t s)
{
    hipLaunchKernelGGL(k_scatter_k, dim3((count + 255) / 256), dim3(256), 0, s, src, idx, dst, count);
    return hipGetLastError();
}

// Synthetic data for launch tuning: both parts uniform in [-1, 1) from a
// counter hash (timing only; the values do not matter beyond being finite).
__global__ void k_fill(float2* x, size_t count, uint32_t seed)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
        uint32_t h = (uint32_t)i * 0x9E3779B1u ^ seed;
        h ^= h >> 16; h *= 0x7FEB352Du; h ^= h >> 15; h *= 0x846CA68Bu; h ^= h >> 16;
        const uint32_t g = h * 0x2C1B3C6Du + 0x297A2D39u;
        x[i] = make_float2((float)(int32_t)h * 0x1p-31f, (float)(int32_t)g * 0x1p-31f);
    }
}

hipError_t launch_fill(float2* x, size_t count, uint32_t seed, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, s, x, count, seed);
    return hipGetLastError();
}

// Root-sum-of-squares coil combine of finished transforms (Eq. 1): T holds
// [recon][coils][nn] complex values; rss[r][i] = (sum_c |T|^2)^(1/2) in FP32,
// each square and their sum rounded, the coils in order, correctly rounded
// square root (the arithmetic of the fused column-pass epilogue).
__global__ void k_rss(const float2* __restrict__ T, int coils, size_t nn, size_t total, float* __restrict__ rss)
{
#pragma clang fp contract(off)
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (size_t)gridDim.x * blockDim.x) {
        const size_t r = q / nn, i = q % nn;
        const float2* t = T + r * coils * nn + i;
        float acc = 0.0f;
        for (int c = 0; c < coils; c++) {
            const float2 v = t[(size_t)c * nn];
            const float re2 = v.x * v.x;
            const float im2 = v.y * v.y;
            const float m2 = re2 + im2;
            acc = acc + m2;
        }
        rss[q] = sqrtf(acc);
    }
}

hipError_t launch_rss(const float2* T, int coils, size_t nn, long recon, float* rss, hipStream_t s)
{
    const size_t total = nn * (size_t)recon;
    const size_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(k_rss, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, s, T, coils, nn, total,
                       rss);
    return hipGetLastError();
}

// Mean SSIM of image x against reference y per image (Wang, Bovik, Sheikh
// and Simoncelli 2004): local means, variances and covariance under an
// 11 x 11 Gaussian window of standard deviation 1.5 normalised to unit sum,
// C1 = (0.01 L)^2, C2 = (0.03 L)^2 with L = max(y), the index at every
// position where the window lies inside the image, averaged.  FP64.  One
// work-group per image; the sums are reduced in a fixed order.
__global__ __launch_bounds__(1024) void k_ssim(const float* __restrict__ x, const float* __restrict__ y, int n,
                                               double* __restrict__ out)
{
    __shared__ double w[121];
    __shared__ double red[16];
    __shared__ float fred[16];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const size_t nn = (size_t)n * n;
    const float* X = x + blockIdx.x * nn;
    const float* Y = y + blockIdx.x * nn;
    if (tid < 121) {
        const int i = tid / 11 - 5, j = tid % 11 - 5;
        w[tid] = exp(-(double)(i * i + j * j) / (2.0 * 1.5 * 1.5));
    }
    float m = -INFINITY;
    for (size_t i = tid; i < nn; i += 1024) m = fmaxf(m, Y[i]);
    for (int o = 32; o; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if (lane == 0) fred[wv] = m;
    __syncthreads();
    if (tid == 0) {
        double sum = 0.0;
        for (int k = 0; k < 121; k++) sum += w[k];
        for (int k = 0; k < 121; k++) w[k] /= sum;
        float mm = fred[0];
        for (int k = 1; k < 16; k++) mm = fmaxf(mm, fred[k]);
        fred[0] = mm;
    }
    __syncthreads();
    const double L = fred[0];
    const double C1 = (0.01 * L) * (0.01 * L), C2 = (0.03 * L) * (0.03 * L);
    const int V = n - 10;
    double acc = 0.0;
    for (int p = tid; p < V * V; p += 1024) {
        const int r = p / V, c = p % V;           // window origin (top-left)
        double mx = 0, my = 0, xx = 0, yy = 0, xy = 0;
        for (int i = 0; i < 11; i++) {
            const float* xr = X + (size_t)(r + i) * n + c;
            const float* yr = Y + (size_t)(r + i) * n + c;
            for (int j = 0; j < 11; j++) {
                const double a = xr[j], b = yr[j], wt = w[i * 11 + j];
                mx += wt * a;
                my += wt * b;
                xx += wt * a * a;
                yy += wt * b * b;
                xy += wt * a * b;
            }
        }
        const double sx = xx - mx * mx, sy = yy - my * my, sxy = xy - mx * my;
        acc += ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sx + sy + C2));
    }
    for (int o = 32; o; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) red[wv] = acc;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int k = 0; k < 16; k++) t += red[k];
        out[blockIdx.x] = t / ((double)V * V);
    }
}

hipError_t launch_ssim(const float* x, const float* y, int n, int count, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_ssim, dim3(count), dim3(1024), 0, s, x, y, n, out);
    return hipGetLastError();
}

int line_lines_per_group(int n)
{
    int r = 8192 / n;
    if (r > n) r = n;
    if (r < 1) r = 1;
    return r;
}

hipError_t launch_lines(int mode, const LineArgs& a, int batch, hipStream_t s)
{
    const dim3 grid(a.n / a.lines, batch), block(256);
    const size_t lds = (size_t)a.lines * a.n * sizeof(float2);
    switch (mode) {
    case MODE_E4M3: hipLaunchKernelGGL(k_lines<MODE_E4M3>, grid, block, lds, s, a); break;
    case MODE_E5M2: hipLaunchKernelGGL(k_lines<MODE_E5M2>, grid, block, lds, s, a); break;
    case MODE_FP16: hipLaunchKernelGGL(k_lines<MODE_FP16>, grid, block, lds, s, a); break;
    case MODE_BF16: hipLaunchKernelGGL(k_lines<MODE_BF16>, grid, block, lds, s, a); break;
    case MODE_FP32: hipLaunchKernelGGL(k_lines<MODE_FP32>, grid, block, lds, s, a); break;
    case MODE_E2M3: hipLaunchKernelGGL(k_lines<MODE_E2M3>, grid, block, lds, s, a); break;
    case MODE_E3M2: hipLaunchKernelGGL(k_lines<MODE_E3M2>, grid, block, lds, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mxk
