// fast_wide_256.hip -- instantiations of the register-resident 256^2 passes for MX blocks of
// 64 values (32 butterflies) in E4M3 and E5M2: the row pass stores FP32, the column pass encodes
// its input as it loads it.
#define MXF_LOGN 8
#define MXF_NS mxf256
#include "mxfft_fast.hpp"

namespace mxk {

hipError_t launch_fast_wide_256(int mode, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch,
                               hipStream_t s)
{
    const dim3 grid((mxf256::N / mxf256::LINES) * batch), block(mxf256::THREADS);
#define MXF_CASE(FF, INV)                                                                                 \
    if (!row && kind == COL_RSS) hipLaunchKernelGGL((mxf256::k_col_rss<FF, 5, INV>), grid, block, 0, s, g); \
    else if (!row) hipLaunchKernelGGL((mxf256::k_col<FF, 5, INV>), grid, block, 0, s, g);                  \
    else if (kind == ROW_RAW) hipLaunchKernelGGL((mxf256::k_row<FF, 5, INV, ROW_RAW>), grid, block, 0, s, g); \
    else if (kind != ROW_PLAIN) return hipErrorInvalidValue;                                           \
    else hipLaunchKernelGGL((mxf256::k_row<FF, 5, INV, ROW_PLAIN>), grid, block, 0, s, g);
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
