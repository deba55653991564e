// Fast chunk encoder for N = 64 (one coder per lane of a wave64).
//
// Same arithmetic as the generic encoder (Algorithm 1's Encode with rANS's
// C, walking the chunk backwards, digits prepended; Section 6's ballot and
// prefix count give each emitting lane its slot), organised for latency:
//  * symbols arrive in 1 KiB blocks (16 steps of uint8, 8 of uint16), one
//    16-byte load per lane issued a block ahead, transposed through LDS;
//  * every step issues exactly one digit store per lane (two for byte
//    digits): lanes that emit nothing store to a junk area past the slot.
//    With a fixed number of memory operations per block the compiler's wait
//    for the next symbol block never has to drain recent stores.
#include <hip/hip_runtime.h>

#include "rans_internal.h"

namespace rans {
namespace {

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ uint32_t mbcnt(uint64_t m, uint32_t acc)
{
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), acc));
}

struct Coder {
    uint32_t x;       // state (per lane)
    uint32_t wpos;    // next free digit index + 1, counting down (uniform)
    bool nosym;
};

// One encode step for all 64 lanes; `s` is the lane's symbol, `act` whether
// the lane codes a symbol in this step.  Exactly R==16 ? 1 : 2 stores.
template <int R>
__device__ __forceinline__ void enc_step(Coder& c, uint32_t s, bool act, const uint4* l_enc,
                                         uint32_t alphabet, uint32_t sh, uint8_t* slot,
                                         uint32_t junk, uint32_t lane)
{
    const uint4 e = l_enc[min(s, alphabet)];
    const uint32_t f = e.y & 0xFFFFu, cum = e.y >> 16;
    c.nosym |= act && f == 0;
    const bool e1 = act && (c.x >> sh) >= f;
    if (R == 16) {
        const uint64_t m = ballot(e1);
        c.wpos -= __popcll(m);
        const uint32_t idx = mbcnt(m, c.wpos);
        const uint32_t o = e1 ? 2 * idx : junk + 2 * lane;
        *reinterpret_cast<uint16_t*>(slot + o) = static_cast<uint16_t>(c.x);
        c.x = e1 ? c.x >> 16 : c.x;
    } else {
        const bool e2 = act && (c.x >> (sh + 8)) >= f;
        const uint64_t m1 = ballot(e1), m2 = ballot(e2);
        c.wpos -= __popcll(m1) + __popcll(m2);
        const uint32_t idx = mbcnt(m2, mbcnt(m1, c.wpos));
        const uint32_t o1 = e1 ? idx : junk + lane;
        const uint32_t o2 = e2 ? idx + 1 : junk + 64 + lane;
        slot[o1] = static_cast<uint8_t>(e2 ? c.x >> 8 : c.x);
        slot[o2] = static_cast<uint8_t>(c.x);
        c.x = e2 ? c.x >> 16 : (e1 ? c.x >> 8 : c.x);
    }
    if (act) {
        const uint32_t th = __umulhi(e.x, c.x);
        const uint32_t q = (th + ((c.x - th) >> (e.z & 0xFFu))) >> (e.z >> 8);
        c.x = c.x + __umul24(q, e.w) + cum;
    }
}

template <int R, int W>
__global__ void __launch_bounds__(1024) k_encode64(const EncodeArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    {
        const uint4* s = a.enc;
        uint4* d = reinterpret_cast<uint4*>(lds);
        for (uint32_t i = threadIdx.x; i < a.enc_bytes / 16; i += blockDim.x)
            d[i] = s[i];
    }
    __syncthreads();
    const uint4* l_enc = reinterpret_cast<const uint4*>(lds);
    using InT = typename std::conditional<W == 1, uint8_t, uint16_t>::type;
    constexpr uint32_t SPB = 16 / W;  // steps per 1 KiB symbol block

    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint8_t* sbuf = lds + a.enc_bytes + wave * 1024;
    const uint64_t chunk = uint64_t(blockIdx.x) * (blockDim.x >> 6) + wave;
    if (chunk >= a.n_chunks)
        return;
    const uint64_t first = chunk * a.C;
    const uint32_t nsym = __builtin_amdgcn_readfirstlane(
        static_cast<uint32_t>(a.n - first < a.C ? a.n - first : a.C));
    const InT* in = static_cast<const InT*>(a.syms) + first;
    uint8_t* slot = a.slots + chunk * a.slot_stride;
    const uint32_t junk = static_cast<uint32_t>(a.slot_bytes);  // byte offset of the junk area
    const uint32_t sh = a.l + R - a.k;
    const uint32_t steps = (nsym + 63) / 64;
    const uint32_t nblk = nsym / (64 * SPB);  // whole blocks
    Coder c{1u << a.l, static_cast<uint32_t>(a.slot_bytes / (R / 8)), false};

    // steps above the whole blocks (the partial tail), one at a time
    for (uint32_t t = steps; t-- > nblk * SPB;) {
        const uint64_t i = uint64_t(t) * 64 + lane;
        const bool act = i < nsym;
        const uint32_t s = act ? static_cast<uint32_t>(in[i]) : 0u;
        enc_step<R>(c, s, act, l_enc, a.alphabet, sh, slot, junk, lane);
    }

    if (nblk > 0) {
        // block b = symbols [b*64*SPB, (b+1)*64*SPB); lane loads 16 bytes
        const uint4* blk = reinterpret_cast<const uint4*>(in) + lane;
        auto load_blk = [&](int64_t b) { return blk[(b < 0 ? 0 : b) * 64]; };
        auto run_blk = [&](uint4 v, uint32_t b) {
            *reinterpret_cast<uint4*>(sbuf + 16 * lane) = v;
            const InT* sb = reinterpret_cast<const InT*>(sbuf) + lane;
#pragma unroll
            for (int q = SPB - 1; q >= 0; --q)
                enc_step<R>(c, sb[q * 64], true, l_enc, a.alphabet, sh, slot, junk, lane);
            (void)b;
        };
        int64_t b = int64_t(nblk) - 1;
        uint4 A = load_blk(b);
        uint4 B = load_blk(b - 1);
        run_blk(A, uint32_t(b));
        A = load_blk(b - 2);
        --b;
        while (b >= 0) {
            run_blk(B, uint32_t(b));
            B = load_blk(b - 2);
            if (--b < 0)
                break;
            run_blk(A, uint32_t(b));
            A = load_blk(b - 2);
            --b;
        }
    }
    a.states[chunk * 64 + lane] = c.x;
    if (lane == 0)
        a.ndig[chunk] = static_cast<uint32_t>(a.slot_bytes / (R / 8)) - c.wpos;
    if (ballot(c.nosym) && lane == 0)
        atomicMin(a.status, RANS_ENOSYM);
}

template <int R, int W>
hipError_t run(const EncodeArgs& a, hipStream_t st)
{
    const uint32_t wpb = a.n_chunks < 16 ? a.n_chunks : 16;
    const uint32_t blocks = (a.n_chunks + wpb - 1) / wpb;
    const uint32_t lds = a.enc_bytes + wpb * 1024;
    auto kern = k_encode64<R, W>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * wpb), lds, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_encode64(const EncodeArgs& a, int R, int W, hipStream_t stream)
{
    if (a.n_chunks == 0)
        return hipSuccess;
    if (R == 16)
        return W == 1 ? run<16, 1>(a, stream) : run<16, 2>(a, stream);
    return W == 1 ? run<8, 1>(a, stream) : run<8, 2>(a, stream);
}

}  // namespace rans
