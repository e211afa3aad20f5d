// fast_wide_256.hip -- instantiations of the register-resident 256^2 passes for MX blocks of
// 64 values (32 butterflies) in E4M3 and E5M2: row tiles of 32 lines, so that a column block's 32
// rows are encoded inside one work-group.
#define MXF_LOGN 8
#define MXF_NS mxf256
#include "mxfft_fast.hpp"

namespace mxk {

hipError_t launch_fast_wide_256(int mode, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch,
                               hipStream_t s)
{
    // row tiles of 32 lines (twice the threads of a 16-line tile); column groups of 16
    const dim3 rgrid((mxf256::N / mxf256::row_lines<0, 5>()) * batch), rblock(mxf256::row_threads<0, 5>());
    const dim3 cgrid((mxf256::N / mxf256::LINES) * batch), cblock(mxf256::THREADS);
#define MXF_CASE(FF, INV)                                                                                    \
    if (!row && kind == COL_RSS) hipLaunchKernelGGL((mxf256::k_col_rss<FF, 5, INV>), cgrid, cblock, 0, s, g);     \
    else if (!row) hipLaunchKernelGGL((mxf256::k_col<FF, 5, INV>), cgrid, cblock, 0, s, g);                      \
    else if (kind == ROW_RAW) hipLaunchKernelGGL((mxf256::k_row<FF, 5, INV, ROW_RAW>), rgrid, rblock, 0, s, g);     \
    else if (kind == ROW_STATS) hipLaunchKernelGGL((mxf256::k_row<FF, 5, INV, ROW_STATS>), rgrid, rblock, 0, s, g); \
    else if (kind == ROW_FIX) hipLaunchKernelGGL((mxf256::k_row_fix<FF, 5, INV>), rgrid, rblock, 0, s, g);         \
    else hipLaunchKernelGGL((mxf256::k_row<FF, 5, INV, ROW_PLAIN>), rgrid, rblock, 0, s, g);
    switch ((mode == MODE_E5M2 ? 2 : mode == MODE_E4M3 ? 0 : 4) + (inverse ? 1 : 0)) {
    case 0: MXF_CASE(0, false) break;
    case 1: MXF_CASE(0, true) break;
    case 2: MXF_CASE(1, false) break;
    case 3: MXF_CASE(1, true) break;
    default: return hipErrorInvalidValue;
    }
#undef MXF_CASE
    return hipGetLastError();
}

}  // namespace mxk
