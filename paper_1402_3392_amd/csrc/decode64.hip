// Single-buffer decode kernel for N = 32 or 64 interleaved coders: one wave
// per chunk, tables staged in LDS once per block; the chunk coder itself is
// c64::decode_chunk.
#include "coder64.h"

namespace rans {
namespace {

template <int R, int W, int SW, int LAYOUT, int NL, bool BF>
__global__ void __launch_bounds__(1024) k_decode64(const DecodeArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    // symbol map first (small immediate offsets), then the entries; the
    // fused layout has no separate symbol map
    const void* symsrc = LAYOUT == kPacked ? a.tab1 : (LAYOUT == kFused ? nullptr : a.tab0);
    const void* ent = LAYOUT == kPacked ? a.tab0 : (LAYOUT == kFused ? a.tab0 : a.tab1);
    const uint32_t sym_bytes = LAYOUT == kPacked ? a.tab1_bytes : (LAYOUT == kFused ? 0 : a.tab0_bytes);
    const uint32_t ent_bytes = LAYOUT == kPacked ? a.tab0_bytes : (LAYOUT == kFused ? a.tab0_bytes : a.tab1_bytes);
    // the waves' rings and output blocks first (low LDS addresses for the
    // direct-to-LDS loads), the tables after them
    uint8_t* tab = lds + c64::uni(blockDim.x >> 6) * c64::wave_lds_bytes(LAYOUT);
    c64::stage2(tab, symsrc, sym_bytes, ent, ent_bytes);
    __syncthreads();
    // wave-uniform by construction; readfirstlane lets the compiler keep
    // everything derived from it in SGPRs
    const uint32_t wave = c64::uni(threadIdx.x >> 6);
    const uint64_t chunk = uint64_t(blockIdx.x) * (blockDim.x >> 6) + wave;
    if (chunk >= a.n_chunks)
        return;  // no barrier follows
    c64::decode_chunk<R, W, SW, LAYOUT, NL, BF>(a.in, a.in_len, a.n_chunks, chunk, a.C, a.n, a.out, a.k, a.l, tab,
                                        reinterpret_cast<const uint32_t*>(tab + sym_bytes),
                                        lds + wave * c64::wave_lds_bytes(LAYOUT), a.status);
}

template <int R, int W, int SW, int LAYOUT, int NL, bool BF>
hipError_t run(const DecodeArgs& a, hipStream_t st)
{
    const uint32_t wpb = a.n_chunks < 16 ? a.n_chunks : 16;
    const uint32_t blocks = (a.n_chunks + wpb - 1) / wpb;
    const uint32_t lds = a.tab0_bytes + a.tab1_bytes + wpb * c64::wave_lds_bytes(LAYOUT);
    auto kern = k_decode64<R, W, SW, LAYOUT, NL, BF>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * wpb), lds, st, a);
    return hipGetLastError();
}

template <int R, int W, int SW, int LAYOUT, bool BF>
hipError_t run_n(const DecodeArgs& a, hipStream_t st)
{
    return a.N == 32 ? run<R, W, SW, LAYOUT, 32, BF>(a, st) : run<R, W, SW, LAYOUT, 64, BF>(a, st);
}

template <int R, int W, int SW, bool BF>
hipError_t run_l(const DecodeArgs& a, Layout layout, hipStream_t st)
{
    if (SW == 1 && layout == kFused)
        return run_n<R, W, 1, kFused, BF>(a, st);
    return layout == kPacked ? run_n<R, W, SW, kPacked, BF>(a, st) : run_n<R, W, SW, kTwoLevel, BF>(a, st);
}

template <int R, bool BF>
hipError_t run_w(const DecodeArgs& a, int W, Layout layout, hipStream_t st)
{
    if (W == 1)
        return run_l<R, 1, 1, BF>(a, layout, st);
    if (a.alphabet <= 256)
        return run_l<R, 2, 1, BF>(a, layout, st);
    return run_l<R, 2, 2, BF>(a, layout, st);
}

}  // namespace

uint32_t decode64_lds_per_wave(Layout layout) { return c64::wave_lds_bytes(layout); }

hipError_t launch_decode64(const DecodeArgs& a, int R, int W, Layout layout, hipStream_t stream)
{
    if (a.n_chunks == 0)
        return hipSuccess;
    // 16-bit digits: one digit per step at most (b >= M), both orders coincide
    if (R == 16)
        return run_w<16, false>(a, W, layout, stream);
    return a.bf ? run_w<8, true>(a, W, layout, stream) : run_w<8, false>(a, W, layout, stream);
}

}  // namespace rans
