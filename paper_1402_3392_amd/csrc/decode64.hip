// Fast chunk decoder for N = 64 (one coder per lane of a wave64).
//
// Per step and lane this is the same decode as the generic kernel (rANS D,
// then Algorithm 1's refill with the ballot/prefix offsets of Section 6);
// what changes is where the bytes come from and go to:
//  * the chunk's digit stream is read from a per-wave LDS ring of 4 windows
//    of 256 bytes; the windows are fetched from HBM four windows ahead of the
//    one being read, with loads whose completion the kernel awaits
//    explicitly (s_waitcnt vmcnt) just before a window enters the ring, so the
//    refill never waits on HBM latency;
//  * decoded symbols go to a per-wave LDS block of 1 KiB and leave as one
//    16-byte store per lane (coalesced 1 KiB per wave).
// The state chain per step is: slot -> LDS table read -> multiply-add ->
// compare (ballot) -> mbcnt -> LDS ring read -> shift-or.
#include <hip/hip_runtime.h>

#include "rans_internal.h"

namespace rans {
namespace {

constexpr uint32_t kWaveLds = 2048;  // ring (1 KiB) + output block (1 KiB)
constexpr uint32_t kWin = 256;       // window bytes

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Issues a 4-byte global load whose completion the caller awaits with
// wait_windows<>() before reading the result.
__device__ __forceinline__ uint32_t async_load(const uint8_t* p)
{
    uint32_t v;
    asm volatile("global_load_dword %0, %1, off" : "=v"(v) : "v"(p) : "memory");
    return v;
}

// All but the `n` most recent vector-memory operations of this wave have
// completed (they complete in issue order).
template <int n>
__device__ __forceinline__ void wait_vm()
{
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(n) : "memory");
}

template <int R, int W, int SW, int LAYOUT>
__global__ void __launch_bounds__(1024) k_decode64(const DecodeArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    // tables: symbol map first (small immediate offsets), then the per-slot
    // entries (kPacked) or the per-symbol entries (kTwoLevel)
    const void* symsrc = LAYOUT == kPacked ? a.tab1 : a.tab0;
    const void* ent = LAYOUT == kPacked ? a.tab0 : a.tab1;
    const uint32_t sym_bytes = LAYOUT == kPacked ? a.tab1_bytes : a.tab0_bytes;
    const uint32_t ent_bytes = LAYOUT == kPacked ? a.tab0_bytes : a.tab1_bytes;
    {
        const uint4* s0 = static_cast<const uint4*>(symsrc);
        const uint4* s1 = static_cast<const uint4*>(ent);
        uint4* d = reinterpret_cast<uint4*>(lds);
        const uint32_t n0 = sym_bytes / 16, n1 = ent_bytes / 16;
        for (uint32_t i = threadIdx.x; i < n0 + n1; i += blockDim.x)
            d[i] = i < n0 ? s0[i] : s1[i - n0];
    }
    __syncthreads();

    using SymT = typename std::conditional<SW == 1, uint8_t, uint16_t>::type;
    using OutT = typename std::conditional<W == 1, uint8_t, uint16_t>::type;
    const SymT* l_sym = reinterpret_cast<const SymT*>(lds);
    const uint32_t* l_ent = reinterpret_cast<const uint32_t*>(lds + sym_bytes);

    const uint32_t lane = threadIdx.x & 63;
    // wave-uniform by construction; readfirstlane lets the compiler keep
    // everything derived from it (chunk, positions, step counters) in SGPRs
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint8_t* ring = lds + sym_bytes + ent_bytes + wave * kWaveLds;
    uint8_t* obuf = ring + 1024;
    const uint64_t chunk = uint64_t(blockIdx.x) * (blockDim.x >> 6) + wave;
    if (chunk >= a.n_chunks)
        return;  // no barrier follows

    const uint8_t* de = a.in + kHeaderBytes + kDirEntryBytes * chunk;
    // directory values are the same for the whole wave: keep them scalar
    const uint64_t off_v = *reinterpret_cast<const uint64_t*>(de);
    const uint64_t off = (uint64_t(__builtin_amdgcn_readfirstlane(uint32_t(off_v >> 32))) << 32) |
                         __builtin_amdgcn_readfirstlane(uint32_t(off_v));
    const uint32_t len = __builtin_amdgcn_readfirstlane(*reinterpret_cast<const uint32_t*>(de + 8));
    const uint64_t first = chunk * a.C;
    const uint32_t nsym = __builtin_amdgcn_readfirstlane(
        static_cast<uint32_t>(a.n - first < a.C ? a.n - first : a.C));
    const uint64_t data0 = (kHeaderBytes + uint64_t(kDirEntryBytes) * a.n_chunks + 15) & ~15ull;
    if ((off & 15) || off < data0 || off > a.in_len || len > a.in_len - off || len < 256 ||
        ((len - 256) % (R / 8)) != 0) {
        if (lane == 0)
            atomicMin(a.status, RANS_ECORRUPT);
        return;
    }
    const uint32_t ndig = (len - 256) / (R / 8);
    const uint32_t L = 1u << a.l, k = a.k, mask = (1u << k) - 1;

    // window w = payload bytes [w*256, w*256+256); lane reads 4 of them.
    // Addresses past the container are clamped to its last whole dword:
    // every load is issued (the wait counts rely on that) and stays inside.
    const uint8_t* pay = a.in + off + 256 + 4 * lane;
    const uint64_t room = a.in_len >= 4 ? ((a.in_len - 4) & ~3ull) : 0;
    const uint64_t pay_off = off + 256 + 4 * lane;
    auto waddr = [&](uint32_t w) -> const uint8_t* {
        const uint64_t o = pay_off + uint64_t(w) * kWin;
        return o <= room ? pay + uint64_t(w) * kWin : a.in + room;
    };
    uint32_t* ring32 = reinterpret_cast<uint32_t*>(ring) + lane;
    uint32_t x = async_load(a.in + off + 4 * lane);  // coder `lane`'s initial state
    uint32_t p0 = async_load(waddr(0));
    uint32_t p1 = async_load(waddr(1));
    uint32_t p2 = async_load(waddr(2));
    uint32_t p3 = async_load(waddr(3));
    wait_vm<2>();
    ring32[0] = p0;
    ring32[64] = p1;
    p0 = async_load(waddr(4));
    p1 = async_load(waddr(5));
    // ring holds windows kw, kw+1; p[(kw+2)%4..] hold kw+2 .. kw+5 in flight

    constexpr uint32_t WD = kWin / (R / 8);           // digits per window
    constexpr uint32_t SPB = 1024 / (64 * W);         // steps per output block
    const uint32_t full = nsym / 64;                  // steps with all lanes active
    const uint32_t steps = (nsym + 63) / 64;
    OutT* out = static_cast<OutT*>(a.out) + first;
    OutT* ob = reinterpret_cast<OutT*>(obuf) + lane;

    uint32_t pos = 0, kw = 0, wend = WD, t = 0;

    auto decode_one = [&](uint32_t& s) {
        const uint32_t slot = x & mask;
        if (LAYOUT == kPacked) {
            const uint32_t e = l_ent[slot];
            s = l_sym[slot];
            x = __umul24(e >> 16, x >> k) + (e & 0xFFFFu);
        } else {
            s = l_sym[slot];
            const uint32_t fc = l_ent[s];
            x = __umul24(fc & 0xFFFFu, x >> k) + slot - (fc >> 16);
        }
    };
    auto refill = [&](bool act) {
        const bool n1 = act && x < L;
        const uint64_t m1 = ballot(n1);
        if (R == 16) {
            if (m1) {
                const uint32_t idx = __builtin_amdgcn_mbcnt_hi(
                    static_cast<uint32_t>(m1 >> 32), __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m1), pos));
                if (n1)
                    x = (x << 16) | reinterpret_cast<const uint16_t*>(ring)[idx & 511];
                pos += __popcll(m1);
            }
        } else {
            const bool n2 = act && x < (L >> 8);
            const uint64_t m2 = ballot(n2);
            if (m1) {
                uint32_t idx = __builtin_amdgcn_mbcnt_hi(
                    static_cast<uint32_t>(m1 >> 32), __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m1), pos));
                idx = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m2 >> 32),
                                                __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m2), idx));
                if (n1) {
                    x = (x << 8) | ring[idx & 1023];
                    if (n2)
                        x = (x << 8) | ring[(idx + 1) & 1023];
                }
                pos += __popcll(m1) + __popcll(m2);
            }
        }
    };
    auto flush = [&](uint32_t tb) {  // output block starting at step tb
        const uint4 v = *reinterpret_cast<const uint4*>(obuf + 16 * lane);
        *reinterpret_cast<uint4*>(reinterpret_cast<uint8_t*>(out + uint64_t(tb) * 64) + 16 * lane) = v;
    };
    auto step = [&]() {
        uint32_t s;
        decode_one(s);
        refill(true);
        ob[(t % SPB) * 64] = static_cast<OutT>(s);
        if (t % SPB == SPB - 1)
            flush(t - (SPB - 1));
        ++t;
    };

    bool done = false;
#define RANS_PHASE(PREG)                                                   \
    if (!done) {                                                           \
        while (t < full && pos < wend)                                     \
            step();                                                        \
        if (t >= full) {                                                   \
            done = true;                                                   \
        } else {                                                           \
            wait_vm<3>();                                                  \
            ring32[((kw + 2) & 3) * 64] = PREG;                            \
            PREG = async_load(waddr(kw + 6));                              \
            ++kw;                                                          \
            wend += WD;                                                    \
        }                                                                  \
    }
    while (!done) {
        RANS_PHASE(p2)
        RANS_PHASE(p3)
        RANS_PHASE(p0)
        RANS_PHASE(p1)
    }
#undef RANS_PHASE
    // last, partial step: only lanes below nsym % 64 take part; its reads lie
    // in windows kw, kw+1 (pos < wend + WD/2 and a step reads < WD/2 digits)
    if (t < steps) {
        const bool act = lane < nsym - t * 64;
        uint32_t s = 0;
        if (act)
            decode_one(s);
        refill(act);
        ob[(t % SPB) * 64] = static_cast<OutT>(s);
        ++t;
    }
    // partial output block: whole 16-byte lane pieces, then the ragged lane
    const uint32_t tb = t - t % SPB;
    if (t % SPB != 0) {
        const uint32_t nbytes = (nsym - tb * 64) * W;  // valid bytes of this block
        uint8_t* dst = reinterpret_cast<uint8_t*>(out + uint64_t(tb) * 64);
        if (16 * lane + 16 <= nbytes) {
            *reinterpret_cast<uint4*>(dst + 16 * lane) = *reinterpret_cast<const uint4*>(obuf + 16 * lane);
        } else if (16 * lane < nbytes) {
            for (uint32_t b = 16 * lane; b < nbytes; ++b)
                dst[b] = obuf[b];
        }
    }
    wait_vm<0>();
    const bool bad = x != L || pos != ndig;
    if (ballot(bad) && lane == 0)
        atomicMin(a.status, RANS_ECORRUPT);
}

template <int R, int W, int SW, int LAYOUT>
hipError_t run(const DecodeArgs& a, hipStream_t st)
{
    const uint32_t wpb = a.n_chunks < 16 ? a.n_chunks : 16;
    const uint32_t blocks = (a.n_chunks + wpb - 1) / wpb;
    const uint32_t lds = a.tab0_bytes + a.tab1_bytes + wpb * kWaveLds;
    auto kern = k_decode64<R, W, SW, LAYOUT>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * wpb), lds, st, a);
    return hipGetLastError();
}

template <int R, int W, int SW>
hipError_t run_l(const DecodeArgs& a, Layout layout, hipStream_t st)
{
    return layout == kPacked ? run<R, W, SW, kPacked>(a, st) : run<R, W, SW, kTwoLevel>(a, st);
}

template <int R>
hipError_t run_w(const DecodeArgs& a, int W, Layout layout, hipStream_t st)
{
    if (W == 1)
        return run_l<R, 1, 1>(a, layout, st);
    if (a.alphabet <= 256)
        return run_l<R, 2, 1>(a, layout, st);
    return run_l<R, 2, 2>(a, layout, st);
}

}  // namespace

uint32_t decode64_lds_per_wave() { return kWaveLds; }

hipError_t launch_decode64(const DecodeArgs& a, int R, int W, Layout layout, hipStream_t stream)
{
    if (a.n_chunks == 0)
        return hipSuccess;
    return R == 16 ? run_w<16>(a, W, layout, stream) : run_w<8>(a, W, layout, stream);
}

}  // namespace rans
