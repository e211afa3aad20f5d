// mxfft_fast.hip -- dispatch of the register-resident 512^2 passes.
#define MXF_LOGN 9
#define MXF_NS mxf
#include "mxfft_fast.hpp"

namespace mxk {

hipError_t launch_fast_e4m3(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_e5m2(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_fp32(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_fp16(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_bf16(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_e2m3(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_e2m3_128(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_e2m3_256(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_e2m3_1024(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_e3m2(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_e3m2_128(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_e3m2_256(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_e3m2_1024(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_fp16_128(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_bf16_128(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_fp16_256(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_bf16_256(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_fp16_1024(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_bf16_1024(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_e4m3_128(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_e5m2_128(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_e4m3_256(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_e5m2_256(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_e4m3_1024(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_e5m2_1024(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_wide_256(int mode, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_wide_512(int mode, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);
hipError_t launch_fast_wide_1024(int mode, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s);

bool fast_supported(int mode, int n, int cb)
{
    // MXFP6 is instantiated for blocks of 16 and 32 only; MXFP8 blocks of 64
    // (32 complex values) at 256^2 and above
    if (fast_wide(mode, n, cb)) return true;
    const bool mx = ((mode == MODE_E4M3 || mode == MODE_E5M2) && cb >= 2 && cb <= 16) ||
                    ((mode == MODE_E2M3 || mode == MODE_E3M2) && (cb == 8 || cb == 16));
    if (n == 512) return mx || mode == MODE_FP32 || mode == MODE_FP16 || mode == MODE_BF16;
    return (n == 128 || n == 256 || n == 1024) && (mx || mode == MODE_FP16 || mode == MODE_BF16);
}

bool fast_wide(int mode, int n, int cb)
{
    return (mode == MODE_E4M3 || mode == MODE_E5M2) && cb == 32 && (n == 256 || n == 512 || n == 1024);
}

bool fast_fused_stats(int mode, int n)
{
    // the statistics histogram lives in the exchange planes of the row pass
    // (4 copies at 128^2, 16 at 256^2, 32 above)
    return is_mx_mode(mode) && (n == 128 || n == 256 || n == 512 || n == 1024);
}

int fast_row_tiles(int mode, int n, int cb)
{
    // 16 lines per work-group at every size; 32 for MXFP8 blocks of 64
    return fast_wide(mode, n, cb) ? n / 32 : n / 16;
}

hipError_t launch_fast(int mode, int n, int cb, bool row, bool inverse, int kind, const FastPassArgs& p,
                       int batch, hipStream_t s)
{
    mxf::FastArgs g{};
    g.src = p.src;
    g.dst = p.dst;
    g.codes = p.codes;
    g.exps = p.exps;
    g.kp = p.kp;
    g.k_out = p.k_out;
    g.kin_mul = p.kin_mul;
    g.kout_mul = p.kout_mul;
    g.kout_add = p.kout_add;
    g.tw = p.tw;
    g.tw_exp = p.tw_exp;
    for (int i = 0; i < 16; i++) g.tw_off[i] = p.tw_off[i];
    g.parts = p.parts;
    g.kadd = p.kadd;
    g.fix_list = p.fix_list;
    g.fix_count = p.fix_count;
    g.tw16 = p.tw16;
    g.rss = p.rss;
    g.coils = p.coils;
    g.slice_off = p.slice_off;
    g.slice_off_out = p.slice_off_out;
    // the redo pass strides over its list: tiles of at most 64 slices in the grid
    if (row && kind == ROW_FIX && batch > 64) batch = 64;
    if (fast_wide(mode, n, cb)) {
        switch (n) {
        case 256: return launch_fast_wide_256(mode, row, inverse, kind, g, batch, s);
        case 512: return launch_fast_wide_512(mode, row, inverse, kind, g, batch, s);
        default: return launch_fast_wide_1024(mode, row, inverse, kind, g, batch, s);
        }
    }
    switch (mode * 4096 + n) {
    case MODE_E4M3 * 4096 + 512: return launch_fast_e4m3(cb, row, inverse, kind, g, batch, s);
    case MODE_E5M2 * 4096 + 512: return launch_fast_e5m2(cb, row, inverse, kind, g, batch, s);
    case MODE_FP32 * 4096 + 512: return launch_fast_fp32(cb, row, inverse, kind, g, batch, s);
    case MODE_FP16 * 4096 + 512: return launch_fast_fp16(cb, row, inverse, kind, g, batch, s);
    case MODE_BF16 * 4096 + 512: return launch_fast_bf16(cb, row, inverse, kind, g, batch, s);
    case MODE_FP16 * 4096 + 128: return launch_fast_fp16_128(cb, row, inverse, kind, g, batch, s);
    case MODE_BF16 * 4096 + 128: return launch_fast_bf16_128(cb, row, inverse, kind, g, batch, s);
    case MODE_FP16 * 4096 + 256: return launch_fast_fp16_256(cb, row, inverse, kind, g, batch, s);
    case MODE_BF16 * 4096 + 256: return launch_fast_bf16_256(cb, row, inverse, kind, g, batch, s);
    case MODE_FP16 * 4096 + 1024: return launch_fast_fp16_1024(cb, row, inverse, kind, g, batch, s);
    case MODE_BF16 * 4096 + 1024: return launch_fast_bf16_1024(cb, row, inverse, kind, g, batch, s);
    case MODE_E2M3 * 4096 + 128: return launch_fast_e2m3_128(cb, row, inverse, kind, g, batch, s);
    case MODE_E2M3 * 4096 + 256: return launch_fast_e2m3_256(cb, row, inverse, kind, g, batch, s);
    case MODE_E2M3 * 4096 + 512: return launch_fast_e2m3(cb, row, inverse, kind, g, batch, s);
    case MODE_E2M3 * 4096 + 1024: return launch_fast_e2m3_1024(cb, row, inverse, kind, g, batch, s);
    case MODE_E3M2 * 4096 + 128: return launch_fast_e3m2_128(cb, row, inverse, kind, g, batch, s);
    case MODE_E3M2 * 4096 + 256: return launch_fast_e3m2_256(cb, row, inverse, kind, g, batch, s);
    case MODE_E3M2 * 4096 + 512: return launch_fast_e3m2(cb, row, inverse, kind, g, batch, s);
    case MODE_E3M2 * 4096 + 1024: return launch_fast_e3m2_1024(cb, row, inverse, kind, g, batch, s);
    case MODE_E4M3 * 4096 + 128: return launch_fast_e4m3_128(cb, row, inverse, kind, g, batch, s);
    case MODE_E5M2 * 4096 + 128: return launch_fast_e5m2_128(cb, row, inverse, kind, g, batch, s);
    case MODE_E4M3 * 4096 + 256: return launch_fast_e4m3_256(cb, row, inverse, kind, g, batch, s);
    case MODE_E5M2 * 4096 + 256: return launch_fast_e5m2_256(cb, row, inverse, kind, g, batch, s);
    case MODE_E4M3 * 4096 + 1024: return launch_fast_e4m3_1024(cb, row, inverse, kind, g, batch, s);
    case MODE_E5M2 * 4096 + 1024: return launch_fast_e5m2_1024(cb, row, inverse, kind, g, batch, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mxk
