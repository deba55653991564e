// Decode fused with a table-lookup consumer, N = 32 or 64 interleaved
// coders: output element i is lut[symbol i], 2 or 4 bytes (the kernel is in
// decode64_impl.h).
#include "decode64_impl.h"

namespace rans {

hipError_t launch_decode64_lut(const DecodeArgs& a, int R, Layout layout, hipStream_t stream)
{
    if (a.n_chunks == 0)
        return hipSuccess;
    if (a.lut_w == 2)
        return run_r<2>(a, R, 1, layout, stream);
    if (a.lut_w == 4)
        return run_r<4>(a, R, 1, layout, stream);
    return hipErrorInvalidValue;
}

}  // namespace rans
