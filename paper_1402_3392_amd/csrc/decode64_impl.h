// Single-buffer decode kernel for N = 32 or 64 interleaved coders: one wave
// per chunk, tables staged in LDS once per block; the chunk coder itself is
// c64::decode_chunk.  LW = 0 writes the symbols; LW = 2 or 4 writes
// lut[symbol] (a consumer fused into the decoder); ESC decodes escape-coded
// 16-bit symbols.  Included by the translation units that instantiate each
// output kind.
#pragma once

#include "decode_seg.h"

namespace rans {
namespace {

// Copies `count` LUT elements of T to LDS (element-wise: the caller's buffer
// holds exactly count elements).
template <typename T>
__device__ __forceinline__ void stage_lut(uint8_t* lds, const void* src, uint32_t count)
{
    const T* s = static_cast<const T*>(src);
    T* d = reinterpret_cast<T*>(lds);
    for (uint32_t i = threadIdx.x; i < count; i += blockDim.x)
        d[i] = s[i];
}

template <int R, int W, int SW, int LAYOUT, int NL, bool BF, int LW, bool ESC, bool PFX>
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
    // direct-to-LDS loads), the tables after them, then the LUT
    uint8_t* tab = lds + c64::uni(blockDim.x >> 6) * c64::wave_lds_bytes(LAYOUT);
    uint8_t* lut = tab + sym_bytes + ent_bytes;
    c64::stage2(tab, symsrc, sym_bytes, ent, ent_bytes);
    if (LW == 2)
        stage_lut<uint16_t>(lut, a.lut, a.alphabet);
    else if (LW == 4)
        stage_lut<uint32_t>(lut, a.lut, a.alphabet);
    __syncthreads();
    // wave-uniform by construction; readfirstlane lets the compiler keep
    // everything derived from it in SGPRs
    const uint32_t wave = c64::uni(threadIdx.x >> 6);
    const uint64_t chunk = uint64_t(blockIdx.x) * (blockDim.x >> 6) + wave;
    if (chunk >= a.n_chunks)
        return;  // no barrier follows
    c64::decode_chunk<R, W, SW, LAYOUT, NL, BF, LW, ESC, PFX>(
        a.in, a.in_len, a.n_chunks, chunk, a.C, a.n, a.out, a.k, a.l, tab,
        reinterpret_cast<const uint32_t*>(tab + sym_bytes), lds + wave * c64::wave_lds_bytes(LAYOUT),
        a.status, lut, a.alphabet);
}

// Symbol output, rANS without escapes: 64 / NL chunks per wave (no lane
// idles with N = 32), the decoder in decode_seg.h.
template <int R, int W, int SW, int LAYOUT, int NL, bool BF, bool ONE>
__global__ void __launch_bounds__(1024) k_decode64_seg(const DecodeArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    constexpr uint32_t SEG = c64::seg_count(NL);
    const void* symsrc = LAYOUT == kPacked ? a.tab1 : (LAYOUT == kFused ? nullptr : a.tab0);
    const void* ent = LAYOUT == kPacked ? a.tab0 : (LAYOUT == kFused ? a.tab0 : a.tab1);
    const uint32_t sym_bytes = LAYOUT == kPacked ? a.tab1_bytes : (LAYOUT == kFused ? 0 : a.tab0_bytes);
    const uint32_t ent_bytes = LAYOUT == kPacked ? a.tab0_bytes : (LAYOUT == kFused ? a.tab0_bytes : a.tab1_bytes);
    uint8_t* tab = lds + c64::uni(blockDim.x >> 6) * c64::seg_wave_lds_bytes(LAYOUT, NL);
    c64::stage2(tab, symsrc, sym_bytes, ent, ent_bytes);
    __syncthreads();
    const uint32_t wave = c64::uni(threadIdx.x >> 6);
    const uint64_t chunk0 = (uint64_t(blockIdx.x) * (blockDim.x >> 6) + wave) * SEG;
    if (chunk0 >= a.n_chunks)
        return;  // no barrier follows
    uint8_t* wave_lds = lds + wave * c64::seg_wave_lds_bytes(LAYOUT, NL);
    if constexpr (SEG == 1)
        c64::decode_chunk<R, W, SW, LAYOUT, NL, BF, 0, false, false, ONE>(
            a.in, a.in_len, a.n_chunks, chunk0, a.C, a.n, a.out, a.k, a.l, tab,
            reinterpret_cast<const uint32_t*>(tab + sym_bytes), wave_lds, a.status);
    else
        c64::decode_seg<R, W, SW, LAYOUT, NL, BF, ONE>(a.in, a.in_len, a.n_chunks, chunk0, a.C, a.n, a.out, a.k,
                                                       a.l, tab, reinterpret_cast<const uint32_t*>(tab + sym_bytes),
                                                       wave_lds, a.status);
}

// Waves per block: 16 when the tables leave room for them, fewer otherwise.
template <int R, int W, int SW, int LAYOUT, int NL, bool BF, int LW, bool ESC, bool PFX = false>
hipError_t run(const DecodeArgs& a, hipStream_t st)
{
    constexpr bool SEGK = LW == 0 && !ESC && !PFX;  // the segment decoder
    constexpr uint32_t SEG = SEGK ? c64::seg_count(NL) : 1;
    const uint32_t tabs = a.tab0_bytes + a.tab1_bytes + lut_lds_bytes(a.alphabet, LW);
    const uint32_t per = SEGK ? c64::seg_wave_lds_bytes(LAYOUT, NL) : c64::wave_lds_bytes(LAYOUT);
    const uint32_t maxl = static_cast<uint32_t>(max_lds_bytes());
    const uint32_t fit = tabs + per <= maxl ? (maxl - tabs) / per : 0;
    if (fit == 0)
        return hipErrorInvalidValue;
    const uint32_t waves = (a.n_chunks + SEG - 1) / SEG;
    uint32_t wpb = waves < 16 ? waves : 16;
    wpb = wpb < fit ? wpb : fit;
    const uint32_t blocks = (waves + wpb - 1) / wpb;
    const uint32_t lds = tabs + wpb * per;
    if constexpr (SEGK) {
        // byte digits with a one-digit table: the single-byte refill (for
        // either digit order: no lane reads a second byte)
        auto kern = R == 8 && a.one ? k_decode64_seg<R, W, SW, LAYOUT, NL, BF, true>
                                    : k_decode64_seg<R, W, SW, LAYOUT, NL, BF, false>;
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * wpb), lds, st, a);
        return hipGetLastError();
    }
    auto kern = k_decode64<R, W, SW, LAYOUT, NL, BF, LW, ESC, PFX>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * wpb), lds, st, a);
    return hipGetLastError();
}

template <int R, int W, int SW, int LAYOUT, bool BF, int LW, bool ESC>
hipError_t run_n(const DecodeArgs& a, hipStream_t st)
{
    return a.N == 32 ? run<R, W, SW, LAYOUT, 32, BF, LW, ESC>(a, st)
                     : run<R, W, SW, LAYOUT, 64, BF, LW, ESC>(a, st);
}

template <int R, int W, int SW, bool BF, int LW, bool ESC = false>
hipError_t run_l(const DecodeArgs& a, Layout layout, hipStream_t st)
{
    if (SW == 1 && layout == kFused)
        return run_n<R, W, 1, kFused, BF, LW, ESC>(a, st);
    return layout == kPacked ? run_n<R, W, SW, kPacked, BF, LW, ESC>(a, st)
                             : run_n<R, W, SW, kTwoLevel, BF, LW, ESC>(a, st);
}

template <int R, bool BF, int LW>
hipError_t run_w(const DecodeArgs& a, int W, Layout layout, hipStream_t st)
{
    const bool wide_map = a.alphabet > 256;  // u16 slot -> symbol map
    if constexpr (LW != 0) {
        // the output is lut[symbol]: only the symbol map's width matters
        (void)W;
        return wide_map ? run_l<R, 1, 2, BF, LW>(a, layout, st) : run_l<R, 1, 1, BF, LW>(a, layout, st);
    } else {
        if (W == 1)  // 8-bit symbols come from tables of at most 256 symbols
            return run_l<R, 1, 1, BF, LW>(a, layout, st);
        return wide_map ? run_l<R, 2, 2, BF, LW>(a, layout, st) : run_l<R, 2, 1, BF, LW>(a, layout, st);
    }
}

// escape coding: 16-bit symbols, depth-first, symbol output
template <int R>
hipError_t run_esc(const DecodeArgs& a, Layout layout, hipStream_t st)
{
    return a.alphabet > 256 ? run_l<R, 2, 2, false, 0, true>(a, layout, st)
                            : run_l<R, 2, 1, false, 0, true>(a, layout, st);
}

// prefix-code family: 16-bit words, its lookup table staged as the packed
// layout's entries (no symbol map)
template <int W>
hipError_t run_pfx(const DecodeArgs& a, hipStream_t st)
{
    return a.N == 32 ? run<16, W, 1, kPacked, 32, false, 0, false, true>(a, st)
                     : run<16, W, 1, kPacked, 64, false, 0, false, true>(a, st);
}

template <int LW>
hipError_t run_r(const DecodeArgs& a, int R, int W, Layout layout, hipStream_t st)
{
    if constexpr (LW == 0) {
        if (a.pfx)
            return W == 1 ? run_pfx<1>(a, st) : run_pfx<2>(a, st);
        if (a.esc)
            return R == 16 ? run_esc<16>(a, layout, st) : run_esc<8>(a, layout, st);
    }
    // 16-bit digits: one digit per step at most (b >= M), both orders coincide
    if (R == 16)
        return run_w<16, false, LW>(a, W, layout, st);
    return a.bf ? run_w<8, true, LW>(a, W, layout, st) : run_w<8, false, LW>(a, W, layout, st);
}

}  // namespace
}  // namespace rans
