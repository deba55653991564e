// Single-buffer decode for N = 32 or 64 interleaved coders, symbol output
// (the kernel is in decode64_impl.h).
#include "decode64_impl.h"

namespace rans {

uint32_t decode64_lds_per_wave(Layout layout) { return c64::wave_lds_bytes(layout); }

uint32_t decode_seg_lds_per_wave(Layout layout, uint32_t N)
{
    switch (layout) {
    case kFused: return N == 32 ? c64::seg_wave_lds_bytes(kFused, 32) : c64::seg_wave_lds_bytes(kFused, 64);
    case kPacked: return N == 32 ? c64::seg_wave_lds_bytes(kPacked, 32) : c64::seg_wave_lds_bytes(kPacked, 64);
    default: return N == 32 ? c64::seg_wave_lds_bytes(kTwoLevel, 32) : c64::seg_wave_lds_bytes(kTwoLevel, 64);
    }
}

hipError_t launch_decode64(const DecodeArgs& a, int R, int W, Layout layout, hipStream_t stream)
{
    if (a.n_chunks == 0)
        return hipSuccess;
    return run_r<0>(a, R, W, layout, stream);
}

}  // namespace rans
