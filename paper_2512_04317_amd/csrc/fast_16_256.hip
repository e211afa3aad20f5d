// fast_16_256.hip -- instantiations of the register-resident 256^2 passes for the FP16 and BF16 forms.
#define MXF_LOGN 8
#define MXF_NS mxf256
#include "mxfft_fast.hpp"

namespace mxk {

namespace {

template <int F>
hipError_t launch16(bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s)
{
    if (row && kind != ROW_PLAIN) return hipErrorInvalidValue;   // statistics ride on the MX row pass only
    const dim3 grid((mxf256::N / mxf256::LINES) * batch), block(mxf256::THREADS);
    if (row) {
        if (inverse) hipLaunchKernelGGL((mxf256::k_row<F, 1, true, ROW_PLAIN>), grid, block, 0, s, g);
        else hipLaunchKernelGGL((mxf256::k_row<F, 1, false, ROW_PLAIN>), grid, block, 0, s, g);
    } else if (kind == COL_RSS) {
        if (inverse) hipLaunchKernelGGL((mxf256::k_col_rss<F, 1, true>), grid, block, 0, s, g);
        else hipLaunchKernelGGL((mxf256::k_col_rss<F, 1, false>), grid, block, 0, s, g);
    } else {
        if (inverse) hipLaunchKernelGGL((mxf256::k_col<F, 1, true>), grid, block, 0, s, g);
        else hipLaunchKernelGGL((mxf256::k_col<F, 1, false>), grid, block, 0, s, g);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fast_fp16_256(int, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s)
{
    return launch16<mxf::FP16>(row, inverse, kind, g, batch, s);
}

hipError_t launch_fast_bf16_256(int, bool row, bool inverse, int kind, const mxf::FastArgs& g, int batch, hipStream_t s)
{
    return launch16<mxf::BF16>(row, inverse, kind, g, batch, s);
}

}  // namespace mxk
