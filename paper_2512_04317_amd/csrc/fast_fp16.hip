// fast_fp16.hip -- instantiations of the register-resident 512^2 passes for the FP16 form.
#define MXF_LOGN 9
#define MXF_NS mxf
#include "mxfft_fast.hpp"

namespace mxk {

hipError_t launch_fast_fp16(int cb, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch,
                          hipStream_t s)
{
    if (row && kind != ROW_PLAIN) return hipErrorInvalidValue;   // statistics ride on the MX row pass only
    const dim3 grid((mxf::N / mxf::LINES) * batch), block(256);
#define MXF_CASE(INV)                                                                          \
    if (row) hipLaunchKernelGGL((mxf::k_row<mxf::FP16, 1, INV, ROW_PLAIN>), grid, block, 0, s, g); \
    else if (kind == COL_RSS) hipLaunchKernelGGL((mxf::k_col_rss<mxf::FP16, 1, INV>), grid, block, 0, s, g); \
    else hipLaunchKernelGGL((mxf::k_col<mxf::FP16, 1, INV>), grid, block, 0, s, g);
    (void)cb;
    if (inverse) { MXF_CASE(true) }
    else { MXF_CASE(false) }
#undef MXF_CASE
    return hipGetLastError();
}

}  // namespace mxk
