// Device functions that code one chunk with all 64 lanes of a wave (N = 64),
// shared by the single-buffer kernels and the persistent batched kernels.
//
// Decode (rANS D, then Algorithm 1's refill; offsets from a ballot of the
// refilling lanes plus mbcnt, Section 6):
//  * the chunk's digit stream is read from a per-wave LDS ring of four
//    256-byte windows; windows are fetched from HBM four windows ahead of
//    the one being read, with loads whose completion the code awaits
//    explicitly (s_waitcnt vmcnt) just before a window enters the ring, so a
//    refill never waits on HBM latency;
//  * decoded symbols go to a per-wave 1 KiB LDS block and leave as one
//    16-byte store per lane.
// Encode (Algorithm 1's Encode with rANS's C, walking backwards):
//  * symbols arrive in 1 KiB blocks, one 16-byte load per lane issued a block
//    ahead and transposed through LDS;
//  * every step issues exactly one digit store per lane (two for byte
//    digits); lanes with nothing to emit store into a junk area past the
//    slot.  A fixed number of memory operations per block lets the
//    compiler's wait for the next block leave recent stores in flight.
#pragma once

#include <hip/hip_runtime.h>

#include "rans_internal.h"

namespace rans {
namespace c64 {

constexpr uint32_t kWaveLds = 2048;  // per wave: decode ring 1 KiB + output block 1 KiB
constexpr uint32_t kWin = 256;       // stream window bytes

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ uint32_t mbcnt(uint64_t m, uint32_t acc)
{
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), acc));
}

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint64_t uni64(uint64_t v)
{
    return (uint64_t(uni(uint32_t(v >> 32))) << 32) | uni(uint32_t(v));
}

// Issues a 4-byte global load whose completion the caller awaits with
// wait_vm<>() before using the result.
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

// Copies two tables (byte counts multiples of 16) into LDS, back to back.
__device__ __forceinline__ void stage2(uint8_t* lds, const void* a, uint32_t abytes, const void* b,
                                       uint32_t bbytes)
{
    const uint4* s0 = static_cast<const uint4*>(a);
    const uint4* s1 = static_cast<const uint4*>(b);
    uint4* d = reinterpret_cast<uint4*>(lds);
    const uint32_t n0 = abytes / 16, n1 = bbytes / 16;
    for (uint32_t i = threadIdx.x; i < n0 + n1; i += blockDim.x)
        d[i] = i < n0 ? s0[i] : s1[i - n0];
}

// Decodes chunk `chunk` of the container `in` (n_chunks chunks of C symbols,
// n in total) into out_base (the container's symbol 0).  l_sym / l_ent are
// the LDS tables (symbol map first, then the packed per-slot entries or the
// per-symbol f|cum entries), wave_lds this wave's 2 KiB.  Every argument
// must be wave-uniform.
template <int R, int W, int SW, int LAYOUT>
__device__ __forceinline__ void decode_chunk(const uint8_t* in, uint64_t in_len, uint32_t n_chunks,
                                             uint64_t chunk, uint32_t C, uint64_t n, void* out_base,
                                             uint32_t k_, uint32_t l, const void* l_sym_v,
                                             const uint32_t* l_ent, uint8_t* wave_lds,
                                             int32_t* status)
{
    using SymT = typename std::conditional<SW == 1, uint8_t, uint16_t>::type;
    using OutT = typename std::conditional<W == 1, uint8_t, uint16_t>::type;
    const SymT* l_sym = static_cast<const SymT*>(l_sym_v);
    const uint32_t lane = threadIdx.x & 63;
    uint8_t* ring = wave_lds;
    uint8_t* obuf = wave_lds + 1024;
    const uint8_t* de = in + kHeaderBytes + kDirEntryBytes * chunk;
    // directory values are the same for the whole wave: keep them scalar
    const uint64_t off = uni64(*reinterpret_cast<const uint64_t*>(de));
    const uint32_t len = uni(*reinterpret_cast<const uint32_t*>(de + 8));
    const uint64_t first = chunk * C;
    const uint32_t nsym = uni(static_cast<uint32_t>(n - first < C ? n - first : C));
    const uint64_t data0 = (kHeaderBytes + uint64_t(kDirEntryBytes) * n_chunks + 15) & ~15ull;
    if ((off & 15) || off < data0 || off > in_len || len > in_len - off || len < 256 ||
        ((len - 256) % (R / 8)) != 0) {
        if (lane == 0)
            atomicMin(status, RANS_ECORRUPT);
        return;
    }
    const uint32_t ndig = (len - 256) / (R / 8);
    const uint32_t L = 1u << l, k = k_, mask = (1u << k) - 1;

    // window w = payload bytes [w*256, w*256+256); lane reads 4 of them.
    // Addresses past the container are clamped to its last whole dword:
    // every load is issued (the wait counts rely on that) and stays inside.
    const uint8_t* pay = in + off + 256 + 4 * lane;
    const uint64_t room = in_len >= 4 ? ((in_len - 4) & ~3ull) : 0;
    const uint64_t pay_off = off + 256 + 4 * lane;
    auto waddr = [&](uint32_t w) -> const uint8_t* {
        const uint64_t o = pay_off + uint64_t(w) * kWin;
        return o <= room ? pay + uint64_t(w) * kWin : in + room;
    };
    uint32_t* ring32 = reinterpret_cast<uint32_t*>(ring) + lane;
    uint32_t x = async_load(in + off + 4 * lane);  // coder `lane`'s initial state
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
    OutT* out = static_cast<OutT*>(out_base) + first;
    OutT* ob = reinterpret_cast<OutT*>(obuf) + lane;

    uint32_t pos = 0, kw = 0, wend = WD, t = 0;

    auto decode_one = [&](uint32_t& s) {
        const uint32_t slot = x & mask;
        if (LAYOUT == kFused) {
            // low 24 bits of e.y are f: what the 24-bit multiply-add reads
            const uint2 e = reinterpret_cast<const uint2*>(l_ent)[slot];
            s = e.y >> 24;
            x = __umul24(e.y, x >> k) + e.x;
        } else if (LAYOUT == kPacked) {
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
    // Blocks that ended inside the full steps were flushed by step(); the
    // rest, [tb, steps), holds the ragged end: whole 16-byte lane pieces,
    // then the one lane that straddles the end byte by byte.
    const uint32_t tb = (full / SPB) * SPB;
    if (tb < steps) {
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
        atomicMin(status, RANS_ECORRUPT);
}

// Encodes chunk `chunk` of syms_base (n symbols, C per chunk) into the digit
// slot `slot` (digits end at slot + slot_bytes; 128 junk bytes follow),
// writes the 64 final states to states_out and the digit count to *ndig_out.
// l_enc: LDS encoder entries (alphabet + 1), wave_lds: this wave's 1 KiB.
template <int R>
__device__ __forceinline__ void enc_step(uint32_t& x, uint32_t& wpos, bool& nosym, uint32_t s, bool act,
                                         const uint4* l_enc, uint32_t alphabet, uint32_t sh,
                                         uint8_t* slot, uint32_t junk, uint32_t lane)
{
    const uint4 e = l_enc[min(s, alphabet)];
    const uint32_t f = e.y & 0xFFFFu, cum = e.y >> 16;
    nosym |= act && f == 0;
    const bool e1 = act && (x >> sh) >= f;
    if (R == 16) {
        const uint64_t m = ballot(e1);
        wpos -= __popcll(m);
        const uint32_t idx = mbcnt(m, wpos);
        const uint32_t o = e1 ? 2 * idx : junk + 2 * lane;
        *reinterpret_cast<uint16_t*>(slot + o) = static_cast<uint16_t>(x);
        x = e1 ? x >> 16 : x;
    } else {
        const bool e2 = act && (x >> (sh + 8)) >= f;
        const uint64_t m1 = ballot(e1), m2 = ballot(e2);
        wpos -= __popcll(m1) + __popcll(m2);
        const uint32_t idx = mbcnt(m2, mbcnt(m1, wpos));
        const uint32_t o1 = e1 ? idx : junk + lane;
        const uint32_t o2 = e2 ? idx + 1 : junk + 64 + lane;
        slot[o1] = static_cast<uint8_t>(e2 ? x >> 8 : x);
        slot[o2] = static_cast<uint8_t>(x);
        x = e2 ? x >> 16 : (e1 ? x >> 8 : x);
    }
    if (act) {
        const uint32_t th = __umulhi(e.x, x);
        const uint32_t q = (th + ((x - th) >> (e.z & 0xFFu))) >> (e.z >> 8);
        x = x + __umul24(q, e.w) + cum;
    }
}

template <int R, int W>
__device__ __forceinline__ void encode_chunk(const void* syms_base, uint64_t n, uint32_t C, uint64_t chunk,
                                             uint32_t k, uint32_t l, uint32_t alphabet,
                                             const uint4* l_enc, uint8_t* slot, uint64_t slot_bytes,
                                             uint8_t* sbuf, uint32_t* states_out, uint32_t* ndig_out,
                                             int32_t* status)
{
    using InT = typename std::conditional<W == 1, uint8_t, uint16_t>::type;
    constexpr uint32_t SPB = 16 / W;  // steps per 1 KiB symbol block
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t first = chunk * C;
    const uint32_t nsym = uni(static_cast<uint32_t>(n - first < C ? n - first : C));
    const InT* in = static_cast<const InT*>(syms_base) + first;
    const uint32_t junk = static_cast<uint32_t>(slot_bytes);  // byte offset of the junk area
    const uint32_t sh = l + R - k;
    const uint32_t steps = (nsym + 63) / 64;
    const uint32_t nblk = nsym / (64 * SPB);  // whole blocks
    uint32_t x = 1u << l;
    uint32_t wpos = uni(static_cast<uint32_t>(slot_bytes / (R / 8)));
    bool nosym = false;

    // steps above the whole blocks (the partial tail), one at a time
    for (uint32_t t = steps; t-- > nblk * SPB;) {
        const uint64_t i = uint64_t(t) * 64 + lane;
        const bool act = i < nsym;
        const uint32_t s = act ? static_cast<uint32_t>(in[i]) : 0u;
        enc_step<R>(x, wpos, nosym, s, act, l_enc, alphabet, sh, slot, junk, lane);
    }

    if (nblk > 0) {
        // block b = symbols [b*64*SPB, (b+1)*64*SPB); lane loads 16 bytes
        const uint4* blk = reinterpret_cast<const uint4*>(in) + lane;
        auto load_blk = [&](int64_t b) { return blk[(b < 0 ? 0 : b) * 64]; };
        auto run_blk = [&](uint4 v) {
            *reinterpret_cast<uint4*>(sbuf + 16 * lane) = v;
            const InT* sb = reinterpret_cast<const InT*>(sbuf) + lane;
#pragma unroll
            for (int q = SPB - 1; q >= 0; --q)
                enc_step<R>(x, wpos, nosym, sb[q * 64], true, l_enc, alphabet, sh, slot, junk, lane);
        };
        int64_t b = int64_t(nblk) - 1;
        uint4 A = load_blk(b);
        uint4 B = load_blk(b - 1);
        run_blk(A);
        A = load_blk(b - 2);
        --b;
        while (b >= 0) {
            run_blk(B);
            B = load_blk(b - 2);
            if (--b < 0)
                break;
            run_blk(A);
            A = load_blk(b - 2);
            --b;
        }
    }
    states_out[lane] = x;
    if (lane == 0)
        *ndig_out = static_cast<uint32_t>(slot_bytes / (R / 8)) - wpos;
    if (ballot(nosym) && lane == 0)
        atomicMin(status, RANS_ENOSYM);
}

}  // namespace c64
}  // namespace rans
