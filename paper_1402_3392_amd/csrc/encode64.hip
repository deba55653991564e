// Single-buffer encode kernel for N = 32 or 64 interleaved coders: one wave
// per chunk, encoder entries staged in LDS once per block; the chunk coder is
// c64::encode_chunk and the chunk is placed into the container in the same
// kernel by c64::place_chunk.
#include "encode_seg.h"

namespace rans {
namespace {

// Chunk indices come from a ticket in start order so that every look-back
// only waits on chunks that are already running.
template <int R, int W, int NL, bool BF, bool ESC, bool ONE>
__global__ void __launch_bounds__(1024) k_encode64_place(const EncodeArgs a, const PlaceArgs p)
{
    // LDS: the waves' digit rings from address 0 (the kernel has no static
    // LDS, so each ring's address is a multiple of its size), their symbol
    // areas, then the encoder entries
    extern __shared__ __align__(16) uint8_t lds[];
    const uint32_t nw = c64::uni(blockDim.x >> 6);
    const uint32_t wave = c64::uni(threadIdx.x >> 6);
    uint8_t* ring = lds + wave * c64::kEncRing;
    uint8_t* sbuf = lds + nw * c64::kEncRing + wave * c64::kEncSymArea;
    uint8_t* tab = lds + nw * c64::kEncWaveLds;
    c64::stage_enc(tab, a.enc, a.enc_bytes, a.l + R - a.k, ESC ? a.alphabet - 1 : ~0u,
                   enc_lds_bytes(a.enc_bytes, W) / 16);
    __syncthreads();
    uint32_t t = 0;
    if ((threadIdx.x & 63) == 0)
        t = atomicAdd(p.ticket, 1u);
    if constexpr (NL == 32 && !ESC) {
        // two chunks per wave: lanes 0-31 code chunk 2t, lanes 32-63 chunk 2t + 1
        const uint32_t chunk = 2 * c64::uni(t);
        if (chunk >= a.n_chunks)
            return;
        uint8_t* s0 = a.slots + uint64_t(chunk) * a.slot_stride;
        uint8_t* s1 = s0 + a.slot_stride;
        uint32_t x = 0, nd[2];
        c64::encode_seg<R, W, BF, ONE>(a.syms, a.n, a.C, chunk, a.n_chunks, a.l, a.alphabet,
                                  reinterpret_cast<const uint4*>(tab), s0, s1, a.slot_bytes, ring, sbuf,
                                  a.status, &x, nd);
        // the lower chunk first: the upper one's look-back waits on it
        const uint32_t nd0 = c64::uni(nd[0]), nd1 = c64::uni(nd[1]);
        const uint32_t x1 = static_cast<uint32_t>(__shfl(static_cast<int>(x), static_cast<int>((threadIdx.x & 63) | 32)));
        const bool two = chunk + 1 < a.n_chunks;
        c64::publish_chunk<R, 32>(chunk, nd0, p);
        if (two)
            c64::publish_chunk<R, 32>(chunk + 1, nd1, p);
        bool t0 = false, t1 = false;
        const uint64_t l0 = c64::chunk_local<R, 32>(chunk, a.n_chunks, nd0, p, t0);
        const uint64_t l1 = two ? c64::chunk_local<R, 32>(chunk + 1, a.n_chunks, nd1, p, t1) : 0;
        c64::place_chunk<R, 32>(chunk, a.n_chunks, x, nd0, s0 + a.slot_bytes - uint64_t(nd0) * (R / 8), p,
                                a.status, true, l0, t0);
        if (two)
            c64::place_chunk<R, 32>(chunk + 1, a.n_chunks, x1, nd1, s1 + a.slot_bytes - uint64_t(nd1) * (R / 8),
                                    p, a.status, true, l1, t1);
        return;
    }
    const uint32_t chunk = c64::uni(t);
    if (chunk >= a.n_chunks)
        return;
    uint8_t* slot = a.slots + uint64_t(chunk) * a.slot_stride;
    uint32_t x = 0, nd = 0;
    c64::encode_chunk<R, W, NL, BF, ESC, ONE>(a.syms, a.n, a.C, chunk, a.k, a.l, a.alphabet,
                                reinterpret_cast<const uint4*>(tab), slot, a.slot_bytes, ring, sbuf,
                                nullptr, nullptr, a.status,
                                &x, &nd);
    // the digits end at slot + slot_bytes; the slot padding after it absorbs
    // the copy's reads past them
    c64::place_chunk<R, NL>(chunk, a.n_chunks, x, c64::uni(nd),
                            slot + a.slot_bytes - uint64_t(c64::uni(nd)) * (R / 8), p, a.status);
}

template <int R, int W, int NL, bool BF, bool ESC = false, bool ONE = false>
hipError_t run_place(const EncodeArgs& a, const PlaceArgs& p, hipStream_t st)
{
    const uint32_t per = NL == 32 && !ESC ? 2 : 1;  // chunks per wave
    const uint32_t waves = (a.n_chunks + per - 1) / per;
    const uint32_t wpb = waves < 16 ? waves : 16;
    const uint32_t blocks = (waves + wpb - 1) / wpb;
    const uint32_t lds = enc_lds_bytes(a.enc_bytes, W) + wpb * c64::kEncWaveLds;
    auto kern = k_encode64_place<R, W, NL, BF, ESC, ONE>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * wpb), lds, st, a, p);
    return hipGetLastError();
}

template <int NL>
hipError_t run_n(const EncodeArgs& a, const PlaceArgs& p, int R, int W, hipStream_t st)
{
    if (a.esc)  // escape coding: 16-bit symbols, depth-first
        return R == 16 ? run_place<16, 2, NL, false, true>(a, p, st) : run_place<8, 2, NL, false, true>(a, p, st);
    // 16-bit digits: one digit per step at most (b >= M), both orders coincide
    if (R == 16)
        return W == 1 ? run_place<16, 1, NL, false>(a, p, st) : run_place<16, 2, NL, false>(a, p, st);
    // byte digits with a one-digit table: the single-digit step (both
    // orders write the same bytes then)
    if (a.one)
        return W == 1 ? run_place<8, 1, NL, false, false, true>(a, p, st)
                      : run_place<8, 2, NL, false, false, true>(a, p, st);
    if (a.bf)
        return W == 1 ? run_place<8, 1, NL, true>(a, p, st) : run_place<8, 2, NL, true>(a, p, st);
    return W == 1 ? run_place<8, 1, NL, false>(a, p, st) : run_place<8, 2, NL, false>(a, p, st);
}

// Prefix-code family (Section 4's multiplexer): one wave per chunk, code
// entries staged in LDS, words stored at their multiplexed positions in the
// chunk's slot, then placed like the rANS chunks (the NL bit counts take the
// place of the states).
template <int W, int NL>
__global__ void __launch_bounds__(1024) k_pfx_encode64(const EncodeArgs a, const PlaceArgs p)
{
    extern __shared__ __align__(16) uint8_t lds[];
    c64::stage2(lds, a.enc, a.enc_bytes, nullptr, 0);
    __syncthreads();
    uint32_t t = 0;
    if ((threadIdx.x & 63) == 0)
        t = atomicAdd(p.ticket, 1u);
    const uint32_t chunk = c64::uni(t);
    if (chunk >= a.n_chunks)
        return;
    uint8_t* slot = a.slots + uint64_t(chunk) * a.slot_stride;
    uint32_t x = 0, nd = 0;
    c64::encode_chunk_pfx<W, NL>(a.syms, a.n, a.C, chunk, a.alphabet, reinterpret_cast<const uint32_t*>(lds),
                                 reinterpret_cast<uint16_t*>(slot), a.status, &x, &nd);
    c64::wait_vm<0>();  // the words are in memory before other lanes copy them
    c64::place_chunk<16, NL>(chunk, a.n_chunks, x, c64::uni(nd), slot, p, a.status);
}

template <int W, int NL>
hipError_t run_pfx(const EncodeArgs& a, const PlaceArgs& p, hipStream_t st)
{
    const uint32_t wpb = a.n_chunks < 16 ? a.n_chunks : 16;
    const uint32_t blocks = (a.n_chunks + wpb - 1) / wpb;
    hipLaunchKernelGGL((k_pfx_encode64<W, NL>), dim3(blocks), dim3(64 * wpb), a.enc_bytes, st, a, p);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_pfx_encode64(const EncodeArgs& a, const PlaceArgs& p, int W, hipStream_t stream)
{
    if (a.n_chunks == 0)
        return hipSuccess;
    if (a.N == 32)
        return W == 1 ? run_pfx<1, 32>(a, p, stream) : run_pfx<2, 32>(a, p, stream);
    return W == 1 ? run_pfx<1, 64>(a, p, stream) : run_pfx<2, 64>(a, p, stream);
}

hipError_t launch_encode64_place(const EncodeArgs& a, const PlaceArgs& p, int R, int W,
                                 hipStream_t stream)
{
    if (a.n_chunks == 0)
        return hipSuccess;
    return a.N == 32 ? run_n<32>(a, p, R, W, stream) : run_n<64>(a, p, R, W, stream);
}

}  // namespace rans
