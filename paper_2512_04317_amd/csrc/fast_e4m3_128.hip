// fast_e4m3_128.hip -- instantiations of the register-resident 128^2 passes for MXFP8-E4M3.
#define MXF_LOGN 7
#define MXF_NS mxf128
#include "mxfft_fast.hpp"

namespace mxk {

hipError_t launch_fast_e4m3_128(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch,
                               hipStream_t s)
{
    const dim3 grid((mxf128::N / mxf128::LINES) * batch), block(mxf128::THREADS);
#define MXF_CASE(CC, INV)                                                                                  \
    if (!row && kind == COL_RSS) hipLaunchKernelGGL((mxf128::k_col_rss<0, CC, INV>), grid, block, 0, s, g); \
    else if (!row) hipLaunchKernelGGL((mxf128::k_col<0, CC, INV>), grid, block, 0, s, g);                  \
    else if (kind == ROW_RAW) hipLaunchKernelGGL((mxf128::k_row<0, CC, INV, ROW_RAW>), grid, block, 0, s, g); \
    else if (kind == ROW_STATS) hipLaunchKernelGGL((mxf128::k_row<0, CC, INV, ROW_STATS>), grid, block, 0, s, g); \
    else if (kind == ROW_FIX) hipLaunchKernelGGL((mxf128::k_row_fix<0, CC, INV>), grid, block, 0, s, g);         \
    else hipLaunchKernelGGL((mxf128::k_row<0, CC, INV, ROW_PLAIN>), grid, block, 0, s, g);
    switch (cb * 2 + (inverse ? 1 : 0)) {
    case 4: MXF_CASE(1, false) break;
    case 5: MXF_CASE(1, true) break;
    case 8: MXF_CASE(2, false) break;
    case 9: MXF_CASE(2, true) break;
    case 16: MXF_CASE(3, false) break;
    case 17: MXF_CASE(3, true) break;
    case 32: MXF_CASE(4, false) break;
    case 33: MXF_CASE(4, true) break;
    default: return hipErrorInvalidValue;
    }
#undef MXF_CASE
    return hipGetLastError();
}

}  // namespace mxk
