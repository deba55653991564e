// Device functions that code one chunk with all 64 lanes of a wave (N = 64),
// shared by the single-buffer kernels and the persistent batched kernels.
//
// Decode (rANS D, then Algorithm 1's refill; offsets from a ballot of the
// refilling lanes plus mbcnt, Section 6):
//  * the chunk's digit stream reaches a per-wave LDS ring of 256-byte
//    windows (4 or 8 slots) by direct global-to-LDS loads issued ahead of
//    the read position; no register ever holds a load in flight, and the
//    code awaits completion explicitly (s_waitcnt vmcnt) when the read
//    position enters a new window, so a refill rarely waits on HBM latency;
//  * decoded symbols go to a per-wave LDS block and leave as one 8- or
//    16-byte store per lane.
// Encode (Algorithm 1's Encode with rANS's C, walking backwards):
//  * symbols arrive in 1 KiB blocks, one 16-byte load per lane issued a block
//    ahead and transposed through LDS;
//  * digits go to a per-wave LDS ring at positions from a ballot prefix and
//    reach HBM a 1 KiB window at a time, one coalesced 16-byte store per
//    lane, instead of a scattered 2-byte store per lane and step.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "rans_internal.h"

// The direct-to-LDS load takes its LDS address in M0, which inline assembly
// has to name as clobbered; clang warns that M0 is reserved.  These kernels
// make no other use of M0.
#pragma clang diagnostic ignored "-Winline-asm"

namespace rans {
namespace c64 {

constexpr uint32_t kWin = 256;  // stream window: one 4-byte load per lane

// Per-wave LDS geometry by table layout.  The fused table (M * 8 bytes)
// leaves about 2 KiB per wave for 16 waves: 4 ring slots tested every 2
// steps and a 512-byte output block.  The smaller tables take 8 slots tested
// every 4 steps and a 1 KiB output block.  One more slot after the ring
// holds a copy of slot 0.
constexpr uint32_t ring_slots(int layout) { return layout == kFused ? 4 : 8; }
constexpr uint32_t test_steps(int layout) { return layout == kFused ? 2 : 4; }
constexpr uint32_t obuf_bytes(int layout) { return layout == kFused ? 512 : 1024; }
constexpr uint32_t wave_lds_bytes(int layout)
{
    return obuf_bytes(layout) + (ring_slots(layout) + 1) * kWin;
}
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

// LDS byte address of a pointer into this block's shared memory.
__device__ __forceinline__ uint32_t lds_addr(const void* p)
{
    typedef __attribute__((address_space(3))) const uint8_t* lds_ptr;
    return uni(static_cast<uint32_t>(reinterpret_cast<uintptr_t>((lds_ptr)p)));
}

// Direct global-to-LDS copy of 256 bytes: lane i moves the 4 bytes at
// base + voff (its own offset) to LDS address dst + 4 i.  base and dst are
// wave-uniform.  No register receives the data; the caller awaits completion
// with wait_vm<>() before reading the LDS bytes.  M0 carries dst and must be
// set one instruction ahead of the load.
__device__ __forceinline__ void dma256(const uint8_t* base, uint32_t voff, uint32_t dst)
{
    asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dword %0, %1"
                 :
                 : "v"(voff), "s"(base), "s"(dst)
                 : "memory", "m0");
}

// Lanes of a wave hand data to each other through LDS (a lane reads bytes
// another lane wrote).  The hardware runs a wave's LDS operations in order,
// but the compiler reasons per lane and may move a read above a write it
// proves cannot touch the same lane's bytes; this compiler barrier keeps
// every LDS access on its side.
__device__ __forceinline__ void lane_fence() { asm volatile("" ::: "memory"); }

// Per lane: b where the lane's bit of mask m is set, a elsewhere (one
// v_cndmask on the ballot mask, no exec-mask branch).
__device__ __forceinline__ uint32_t select_mask(uint64_t m, uint32_t a, uint32_t b)
{
    uint32_t r;
    asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(m));
    return r;
}

// Per lane, x > y as the wave's mask (returned), and *xs = x >> 16 where it
// holds, x elsewhere.  The compare writes vcc, the one mask an SDWA select
// reads, and the select takes x's upper half in place: one instruction
// fewer than a shift and a select.
__device__ __forceinline__ uint64_t gt_shift16(uint32_t x, uint32_t y, uint32_t* xs)
{
    uint64_t m;
    uint32_t r;
    asm("v_cmp_gt_u32_e32 vcc, %2, %3\n\t"
        "s_mov_b64 %0, vcc\n\t"
        "v_cndmask_b32_sdwa %1, %2, %2, vcc dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_1"
        : "=s"(m), "=v"(r)
        : "v"(x), "v"(y)
        : "vcc");
    *xs = r;
    return m;
}

// A wave-uniform value in a vector register (a VOP3 operation reads at most
// one scalar register on this chip; a loop-invariant copy frees the slot).
__device__ __forceinline__ uint32_t in_vgpr(uint32_t s)
{
    uint32_t r;
    asm("v_mov_b32 %0, %1" : "=v"(r) : "s"(s));
    return r;
}

// A digit's ring store by the lanes of m: at LDS address a on those lanes,
// at junk (a per-lane address nothing reads) on the others -- a select, not
// an exec-mask branch, and a store the compiler counts when it waits for
// the step's LDS reads.
template <int B>
__device__ __forceinline__ void ring_store(uint64_t m, uint32_t a, uint32_t junk, uint32_t v)
{
    const uint32_t o = select_mask(m, junk, a);
    if constexpr (B == 2)
        *(__attribute__((address_space(3))) uint16_t*)(o) = static_cast<uint16_t>(v);
    else
        *(__attribute__((address_space(3))) uint8_t*)(o) = static_cast<uint8_t>(v);
}

// The same address as a pointer into global memory.  Accesses through it are
// global_* instructions, which count in vmcnt only and complete in issue
// order, so the compiler waits for exactly the load it needs.  Through a
// generic pointer (one read from a job descriptor, say) they are flat_*
// instructions, which also count in lgkmcnt and may target LDS: the
// compiler then waits for every outstanding memory operation, loads just
// issued ahead and stores included, before an LDS result or a prefetched
// register is used.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p)
{
    return (__attribute__((address_space(1))) T*)p;
}

typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));

// 8- and 16-byte global stores and a 16-byte global load (the HIP vector
// classes have no assignment across address spaces)
__device__ __forceinline__ void gstore(void* p, const uint4& v)
{
    v4u t;
    t.x = v.x;
    t.y = v.y;
    t.z = v.z;
    t.w = v.w;
    *gmem(static_cast<v4u*>(p)) = t;
}
__device__ __forceinline__ void gstore(void* p, const uint2& v)
{
    v2u t;
    t.x = v.x;
    t.y = v.y;
    *gmem(static_cast<v2u*>(p)) = t;
}
__device__ __forceinline__ uint4 gload16(const void* p)
{
    const v4u t = *gmem(static_cast<const v4u*>(p));
    return make_uint4(t.x, t.y, t.z, t.w);
}

// All but the `n` most recent vector-memory operations of this wave have
// completed (loads and stores complete in issue order).
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
// n in total, NL = 32 or 64 interleaved coders: lanes NL.. of the wave stay
// idle) into out_base (the container's symbol 0).  l_sym / l_ent are
// the LDS tables (symbol map first, then the packed per-slot entries, the
// per-symbol f|cum entries or the fused entries), wave_lds this wave's
// wave_lds_bytes(LAYOUT) bytes.  Every argument must be wave-uniform.  When
// it returns, every load it issued has completed, so wave_lds can be reused.
// BF: the chunk's digits are in breadth-first order (Section 5; only byte
// digits can differ from depth-first).  LW = 2 or 4: a consumer fused into
// the decoder -- output element i is l_lut[symbol i] (LW bytes, staged in
// LDS), so the symbols never reach memory; W is then irrelevant.  ESC
// (16-bit symbols, depth-first): escape coding -- the table's last symbol
// E = alphabet - 1 is followed in its coder's share of the step by 16 / R
// raw digits that hold the output value (Section 3's raw data mixed into
// the stream).  PFX (R = 16): the chunk holds the prefix-code family
// multiplexed as Section 4 describes -- NL bit counts at the head, then the
// 16-bit words in the order the decoders read them; each lane reads one word
// before a symbol whenever it holds fewer than 16 bits, then looks the
// symbol up by its next k_ (the longest code length) bits in l_ent (u16
// entries symbol | length << 12); the end check compares the bits each lane
// consumed with its count.
template <int R, int W, int SW, int LAYOUT, int NL, bool BF = false, int LW = 0, bool ESC = false,
          bool PFX = false, bool ONE = false>
__device__ __forceinline__ void decode_chunk(const uint8_t* in, uint64_t in_len, uint32_t n_chunks,
                                             uint64_t chunk, uint32_t C, uint64_t n, void* out_base,
                                             uint32_t k_, uint32_t l, const void* l_sym_v,
                                             const uint32_t* l_ent, uint8_t* wave_lds,
                                             int32_t* status, const void* l_lut = nullptr,
                                             uint32_t alphabet = 0)
{
    static_assert(!ESC || (W == 2 && !BF && LW == 0), "escape coding: 16-bit symbols, depth-first");
    static_assert(!PFX || (R == 16 && !BF && !ESC && LW == 0), "prefix-code family: 16-bit words");
    const uint32_t E = alphabet - 1;  // the escape symbol (ESC)
    using SymT = typename std::conditional<SW == 1, uint8_t, uint16_t>::type;
    using SymOutT = typename std::conditional<W == 1, uint8_t, uint16_t>::type;
    using LutT = typename std::conditional<LW == 4, uint32_t, uint16_t>::type;
    using OutT = typename std::conditional<LW == 0, SymOutT, LutT>::type;
    constexpr uint32_t OW = sizeof(OutT);  // output bytes per symbol
    const LutT* lut = static_cast<const LutT*>(l_lut);
    // what a decoded symbol becomes in the output
    auto emit = [&](uint32_t s) -> OutT {
        if (LW == 0)
            return static_cast<OutT>(s);
        return static_cast<OutT>(lut[s]);
    };
    const SymT* l_sym = static_cast<const SymT*>(l_sym_v);
    const uint32_t lane = threadIdx.x & 63;
    constexpr uint32_t OB = obuf_bytes(LAYOUT);
    uint8_t* obuf = wave_lds;              // output block (first: the initial states)
    constexpr uint32_t S = ring_slots(LAYOUT), TB = test_steps(LAYOUT);
    // a block of TB steps reads at most MAXB TB bytes starting below the end
    // of window kw, so windows kw .. kw + RES - 1 must have landed; the
    // loads of the other S - RES slots may still be in flight.  A step reads
    // at most 2 digit bytes per coder, 4 with escapes (a renormalisation
    // digit and a raw digit of 16 bits, or two bytes of each).
    constexpr uint32_t MAXB = ESC ? 256 : 128;
    constexpr uint32_t RES = 1 + TB * MAXB / kWin;
    constexpr int AHEAD = static_cast<int>(S - RES);
    const uint8_t* ring = wave_lds + OB;   // S windows + copy of slot 0
    const uint8_t* de = in + kHeaderBytes + kDirEntryBytes * chunk;
    // directory values are the same for the whole wave: keep them scalar
    const uint64_t off = uni64(*reinterpret_cast<const uint64_t*>(de));
    const uint32_t len = uni(*reinterpret_cast<const uint32_t*>(de + 8));
    const uint64_t first = chunk * C;
    const uint32_t nsym = uni(static_cast<uint32_t>(n - first < C ? n - first : C));
    const uint64_t data0 = (kHeaderBytes + uint64_t(kDirEntryBytes) * n_chunks + 15) & ~15ull;
    if ((off & 15) || off < data0 || off > in_len || len > in_len - off || len < 4 * NL ||
        ((len - 4 * NL) % (R / 8)) != 0) {
        if (lane == 0)
            atomicMin(status, RANS_ECORRUPT);
        return;
    }
    const bool live = NL == 64 || lane < NL;
    const uint32_t plen = len - 4 * NL;  // digit bytes after the NL states
    const uint32_t L = 1u << l, k = k_, mask = (1u << k) - 1;

    // Window w = digit bytes [256 w, 256 w + 256) sits in ring slot w % S;
    // windows 0, S, 2S, ... go to one more slot after the last as well, so a
    // read that starts in slot S - 1 runs on into the next window unwrapped.
    // Lane addresses past the container (whole 4-byte words) are pulled back
    // to its last word; such bytes are never used.
    const uint64_t room = (in_len - 4) & ~3ull;  // in_len >= 176 here
    const uint32_t lds_ob = lds_addr(obuf), lds_ring = lds_ob + OB, lane4 = 4 * lane;
    auto fetch = [&](uint64_t src, uint32_t dst) {  // 256 container bytes from src
        uint32_t vo = lane4;
        if (src + kWin > room + 4) {
            if (src > room)
                src = room;
            vo = min(lane4, static_cast<uint32_t>(room - src));
        }
        dma256(in + src, vo, dst);
    };
    const uint64_t pay = off + 4 * NL;
    const uint32_t nwin = (plen + kWin - 1) / kWin;
    // windows below wfast lie wholly inside the container: no clamping
    const uint32_t wfast =
        uni(room + 4 >= pay + kWin ? static_cast<uint32_t>((room + 4 - pay - kWin) / kWin) + 1 : 0u);
    // Vector-memory operations (these loads and the output stores) complete
    // in issue order.  The wait after a window load leaves in flight the
    // operations issued after the load of window kw + RES - 1: the AHEAD
    // window loads after it plus the stores and slot-0 copies among them,
    // counted per window interval in hist[] (oldest first) and cur (since the
    // newest window load).
    uint32_t hist[AHEAD > 0 ? AHEAD : 1] = {};
    uint32_t cur = 0;
    auto fetch_win = [&](uint32_t w, uint32_t dst) {
        const uint64_t src = pay + uint64_t(w) * kWin;
        if (w < wfast)
            dma256(in + src, lane4, dst);
        else
            fetch(src, dst);
    };
    auto issue = [&](uint32_t w) {
        if (w % S == 0) {  // the copy goes first, so it lands no later than the window
            fetch_win(w, lds_ring + S * kWin);
            ++cur;
        }
        fetch_win(w, lds_ring + (w % S) * kWin);
#pragma unroll
        for (int i = 0; i + 1 < AHEAD; ++i)
            hist[i] = hist[i + 1];
        hist[AHEAD - 1] = cur;
        cur = 0;
    };
    fetch(off, lds_ob);  // coder i's initial state: bytes 4 i .. 4 i + 3 (i < NL)
#pragma unroll
    for (uint32_t w = 0; w < S; ++w)
        if (w < nwin)
            issue(w);
    // windows 0 .. RES - 1 (and window 0's copy, issued before window 0)
    // are in once at most S - RES later loads are pending
    if (nwin >= S)
        wait_vm<AHEAD>();
    else
        wait_vm<0>();
#pragma unroll
    for (int i = 0; i < AHEAD; ++i)
        hist[i] = 0;
    cur = 0;
    uint32_t x = reinterpret_cast<const uint32_t*>(obuf)[lane];
    lane_fence();  // the output block is reused for symbols
    if (!live)
        x = PFX ? 0u : L;  // idle lanes stay at L and never refill (PFX: count 0)
    uint32_t pbuf = 0, pnb = 0, pused = 0;  // PFX: bit buffer (MSB first), its bits, bits used

    constexpr uint32_t SPB = OB / (NL * OW);   // steps per output block
    constexpr uint32_t PIECE = OB / 64;         // bytes each lane moves per block
    constexpr uint32_t DB = R / 8;                 // bytes per digit
    constexpr uint32_t DMASK = S * kWin / DB - 1;  // ring size in digits, minus 1
    constexpr uint32_t WD = kWin / DB;             // digits per window
    using Piece = typename std::conditional<PIECE == 16, uint4, uint2>::type;
    const uint32_t full = nsym / NL;           // steps with every coder active
    const uint32_t steps = (nsym + NL - 1) / NL;
    OutT* out = static_cast<OutT*>(out_base) + first;
    OutT* ob = reinterpret_cast<OutT*>(obuf) + lane;

    // pos: next digit; wend: digits up to the end of window kw
    uint32_t pos = 0, kw = 0, wend = WD, t = 0;
    const uint32_t ndig = plen / DB;

    auto decode_one = [&](uint32_t& s) {
        const uint32_t x0 = x;
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
        if (!live)
            x = x0;
    };
    // Refill: every lane reads the ring at its would-be digit (the ring
    // position, a scalar, plus the prefix count of refilling lanes below it)
    // and a select on the ballot keeps the digit in the lanes that need it.
    // With byte digits a lane may read two: depth-first they are adjacent
    // (after the digits of the lanes below); breadth-first the first digits
    // of all reading lanes come first, then the second digits.  Either way
    // the step reads digits [pos, pos + |m1| + |m2|).
    // In sparse chunks the step is skipped as a whole when no lane refills;
    // in dense ones (dense = std::true_type) it runs unconditionally, which
    // takes a branch off every step's dependency chain.
    auto refill = [&](bool act, auto dense) {
        const bool n1 = act && x < L;
        const uint64_t m1 = ballot(n1);
        if (R == 16) {
            if (dense || m1) {
                const uint16_t* rp = reinterpret_cast<const uint16_t*>(ring) + (pos & DMASK);
                const uint32_t v = rp[mbcnt(m1, 0)];
                x = select_mask(m1, x, (x << 16) | v);
                pos += __popcll(m1);
            }
        } else if (ONE) {
            // a one-digit table: no state falls below L / 256, one byte per
            // refilling lane (both digit orders read the same bytes then)
            if (dense || m1) {
                x = select_mask(m1, x, (x << 8) | ring[(pos & DMASK) + mbcnt(m1, 0)]);
                pos += __popcll(m1);
            }
        } else {
            const bool n2 = act && x < (L >> 8);
            const uint64_t m2 = ballot(n2);
            if (dense || m1) {
                const uint8_t* r = ring + (pos & DMASK);
                uint32_t x1, x2;
                if (BF) {
                    // the second digits start after every first digit: a
                    // scalar base, so each address is one mbcnt pair plus
                    // one add
                    const uint8_t* r2 = r + __popcll(m1);
                    x1 = (x << 8) | r[mbcnt(m1, 0)];
                    x2 = (x1 << 8) | r2[mbcnt(m2, 0)];
                } else {
                    // two independent prefix counts (a shorter chain than
                    // accumulating one into the other)
                    const uint8_t* q = r + (mbcnt(m1, 0) + mbcnt(m2, 0));
                    x1 = (x << 8) | q[0];
                    x2 = (x1 << 8) | q[1];
                }
                x = select_mask(m1, x, select_mask(m2, x1, x2));
                pos += __popcll(m1) + __popcll(m2);
            }
        }
    };
    // Refill with escapes: a lane's digits in the step are its
    // renormalisation digits, then (escape lanes) 16 raw bits; every lane
    // reads at the prefix count of all digits below it, the escape lanes'
    // raw digits replace the decoded symbol.
    auto refill_esc = [&](bool act, auto dense, uint32_t& s) {
        const bool n1 = act && x < L;
        const bool ne = act && s == E;
        const uint64_t m1 = ballot(n1), me = ballot(ne);
        if (R == 16) {
            if (dense || (m1 | me)) {
                const uint16_t* rp = reinterpret_cast<const uint16_t*>(ring) + (pos & DMASK);
                const uint16_t* q = rp + (mbcnt(m1, 0) + mbcnt(me, 0));
                const uint32_t v0 = q[0], v1 = q[1];
                x = select_mask(m1, x, (x << 16) | v0);
                s = select_mask(me, s, select_mask(m1, v0, v1));
                pos += __popcll(m1) + __popcll(me);
            }
        } else {
            const bool n2 = act && x < (L >> 8);
            const uint64_t m2 = ballot(n2);
            if (dense || (m1 | me)) {
                const uint8_t* q = ring + (pos & DMASK) + (mbcnt(m1, 0) + mbcnt(m2, 0) + 2 * mbcnt(me, 0));
                const uint32_t b0 = q[0], b1 = q[1], b2 = q[2], b3 = q[3];
                const uint32_t x1 = (x << 8) | b0, x2 = (x1 << 8) | b1;
                x = select_mask(m1, x, select_mask(m2, x1, x2));
                // raw value after 0, 1 or 2 renormalisation bytes
                const uint32_t r0 = (b0 << 8) | b1, r1 = (b1 << 8) | b2, r2 = (b2 << 8) | b3;
                s = select_mask(me, s, select_mask(m1, r0, select_mask(m2, r1, r2)));
                pos += __popcll(m1) + __popcll(m2) + 2 * __popcll(me);
            }
        }
    };
    // Prefix-code step: the read (one word when fewer than 16 bits are
    // buffered) comes before the symbol, so every lane reads at the prefix
    // count of the reading lanes below it, then decodes from its buffer.
    auto step_pfx = [&](bool act, auto dense, uint32_t& s) {
        const bool n1 = act && pnb < 16;
        const uint64_t m1 = ballot(n1);
        if (dense || m1) {
            const uint16_t* rp = reinterpret_cast<const uint16_t*>(ring) + (pos & DMASK);
            const uint32_t v = rp[mbcnt(m1, 0)];
            pbuf = select_mask(m1, pbuf, pbuf | (v << ((16u - pnb) & 31u)));
            pnb = select_mask(m1, pnb, pnb + 16);
            pos += __popcll(m1);
        }
        const uint32_t e = reinterpret_cast<const uint16_t*>(l_ent)[pbuf >> (32 - k)];
        s = e & 0xFFFu;
        const uint32_t len = act ? e >> 12 : 0u;
        pbuf <<= len;
        pnb -= len;
        pused += len;
    };
    auto flush = [&](uint32_t tb) {  // output block starting at step tb
        lane_fence();
        const Piece v = *reinterpret_cast<const Piece*>(obuf + PIECE * lane);
        lane_fence();
        gstore(reinterpret_cast<uint8_t*>(out + uint64_t(tb) * NL) + PIECE * lane, v);
        ++cur;  // one store instruction (more would only make waits longer)
    };
    auto step1 = [&](OutT* dst, auto dense) {
        uint32_t s;
        if (PFX) {
            step_pfx(live, dense, s);
        } else {
            decode_one(s);
            if (ESC)
                refill_esc(live, dense, s);
            else
                refill(live, dense);
        }
        if (live)
            *dst = emit(s);
    };
    // TB full steps; t is a multiple of TB here (and TB divides SPB), so the
    // output offsets are immediates and an output block ends on a test block
    auto stepblk = [&]() {
        OutT* o = ob + (t & (SPB - 1)) * NL;
#pragma unroll
        for (uint32_t i = 0; i < TB; ++i)
            step1(o + i * NL, std::false_type{});
        t += TB;
        if ((t & (SPB - 1)) == 0)
            flush(t - SPB);
    };
    auto step_single = [&]() {
        step1(ob + (t & (SPB - 1)) * NL, std::false_type{});
        ++t;
        if ((t & (SPB - 1)) == 0)
            flush(t - SPB);
    };
    // last, partial step: only lanes below nsym % NL take part
    auto partial_step = [&]() {
        const bool act = lane < nsym - t * NL;
        uint32_t s = 0;
        if (PFX) {
            step_pfx(act, std::false_type{}, s);
        } else {
            if (act)
                decode_one(s);
            if (ESC)
                refill_esc(act, std::false_type{}, s);
            else
                refill(act, std::false_type{});
        }
        if (live)
            ob[(t & (SPB - 1)) * NL] = emit(s);
        ++t;
    };
    // A step reads at most MAXB digit bytes, so TB steps that start below
    // wend = 256 (kw + 1) stay inside windows kw .. kw + RES - 1.
    // Moving kw on issues window kw + S - 1 into the slot of the window just
    // finished, then waits until at most S - RES later loads are pending:
    // window kw + RES - 1 is in.
    auto advance = [&]() {
        while (pos >= wend) {
            ++kw;
            wend += WD;
            if (kw + S - 1 < nwin) {
                issue(kw + S - 1);
                uint32_t pend = cur;
#pragma unroll
                for (int i = 0; i < AHEAD; ++i)
                    pend += hist[i];
                // more than two extra operations: waiting as if two only waits longer
                if (pend == 0)
                    wait_vm<AHEAD>();
                else if (pend == 1)
                    wait_vm<AHEAD + 1>();
                else
                    wait_vm<AHEAD + 2>();
            } else {
                wait_vm<0>();
            }
        }
    };
    static_assert(SPB % TB == 0 && MAXB * TB <= (RES - 1) * kWin && RES < S, "ring geometry");

    // whole output blocks: every offset is an immediate, one flush per block
    constexpr uint32_t NB = SPB / TB;
    auto blocks = [&](auto dense) {
        while (t + SPB <= full) {
#pragma unroll
            for (uint32_t b = 0; b < NB; ++b) {
                advance();
#pragma unroll
                for (uint32_t i = 0; i < TB; ++i)
                    step1(ob + (b * TB + i) * NL, dense);
            }
            t += SPB;
            flush(t - SPB);
        }
    };
    // dense: at least one refill per 16 coder steps (two digits per refill
    // at most with byte digits), so a step without any refill is rare
    if (uint64_t(ndig) * 16 >= uint64_t(nsym) * (R == 8 ? 2 : 1))
        blocks(std::true_type{});
    else
        blocks(std::false_type{});
    while (t + TB <= full) {  // fewer than SPB full steps remain
        advance();
        stepblk();
    }
    advance();  // fewer than TB full steps remain
    while (t < full)
        step_single();
    if (t < steps)
        partial_step();

    // Blocks that ended inside the full steps were flushed; the rest,
    // [tb, steps), holds the ragged end: whole lane pieces, then the one
    // lane that straddles the end byte by byte.
    const uint32_t tb = (full / SPB) * SPB;
    lane_fence();
    if (tb < steps) {
        const uint32_t nbytes = (nsym - tb * NL) * OW;  // valid bytes of this block
        uint8_t* dst = reinterpret_cast<uint8_t*>(out + uint64_t(tb) * NL);
        if (PIECE * lane + PIECE <= nbytes) {
            gstore(dst + PIECE * lane, *reinterpret_cast<const Piece*>(obuf + PIECE * lane));
        } else if (PIECE * lane < nbytes) {
            for (uint32_t b = PIECE * lane; b < nbytes; ++b)
                dst[b] = obuf[b];
        }
    }
    wait_vm<0>();  // windows fetched ahead land before wave_lds is reused
    const bool bad = (PFX ? pused != x : x != L) || pos != ndig;
    if (ballot(bad) && lane == 0)
        atomicMin(status, RANS_ECORRUPT);
}

// Per-wave LDS of the encoder: a 4 KiB digit ring at an LDS address that is
// a multiple of 4 KiB (a digit's ring address is its position's bits or-ed
// into the ring's), and a symbol area: a 1 KiB symbol block, then 128
// bytes where lanes with no digit to store write.  A kernel lays out the
// rings of its waves first, from LDS address 0, then their symbol areas.
constexpr uint32_t kEncRing = 4096;
constexpr uint32_t kEncSymBlock = 1024;
constexpr uint32_t kEncSymArea = kEncSymBlock + 128;
constexpr uint32_t kEncWaveLds = kEncWaveLdsBytes;
static_assert(kEncWaveLds == kEncRing + kEncSymArea, "encoder LDS layout");
// Digits leave the ring in windows of kEncWindow bytes, aligned to
// multiples of it in the slot (slot sizes are multiples of it), one 16-byte
// store per lane.  Window stores per flush: after a flush fewer than
// kEncWindow bytes stay pending, and a block of symbols (1 KiB) adds at
// most 2 KiB of digits, so a flush completes at most 2 windows.
constexpr uint32_t kEncWindow = 1024;
constexpr uint32_t kFlushStores = 2;
static_assert(kEncWindow == kSlotAlign && kSlotPad >= kEncWindow && kEncRing % kEncWindow == 0,
              "encoder windows, slots and ring");

// Stages the encoder entries of a table into LDS for one parameter set,
// sh = l + r - k.  Table entry {m, f | cum << 16, inc | dsh << 8, M - f}
// (q = x / f = mulhi(x + inc, m) >> dsh) becomes
// {m, x_max - 1, cum | dsh << 16, (M - f) | bad << 23 | inc << 24}
// with x_max = f * 2^sh the bound of Algorithm 1's renormalisation (no digit
// is emitted once x < x_max; x_max >= 2^32 is stored as 2^32 - 1, which no
// state exceeds) and bad = (f == 0), a symbol the table cannot encode.  The
// kernel then compares against x_max - 1 directly and reads every field
// with sub-dword operand selects.  esc (escape coding): the escape symbol;
// every entry the coder cannot use directly -- frequency 0, or at or above
// the escape (the extra last entry included) -- becomes a copy of the
// escape's entry with bit 31 of z set, so one LDS read gives both the entry
// to code and whether raw digits follow.  pad_to: entries staged at least
// (those past the table get frequency 0: not encodable).
__device__ __forceinline__ void stage_enc(uint8_t* lds, const uint4* src, uint32_t bytes, uint32_t sh,
                                          uint32_t esc = ~0u, uint32_t pad_to = 0)
{
    uint4* d = reinterpret_cast<uint4*>(lds);
    const uint32_t n = bytes / 16, nn = n > pad_to ? n : pad_to;
    for (uint32_t i = threadIdx.x; i < nn; i += blockDim.x) {
        uint4 e = i < n ? src[i] : make_uint4(0, 0, 0, 0);  // padding: frequency 0
        const bool raw = esc != ~0u && (i >= esc || (e.y & 0xFFFFu) == 0);
        if (raw)
            e = src[esc];
        const uint32_t f = e.y & 0xFFFFu, cum = e.y >> 16, inc = e.z & 0xFFu, dsh = e.z >> 8;
        const uint64_t xm = uint64_t(f) << sh;
        d[i] = make_uint4(e.x, (f == 0 || xm > 0xFFFFFFFFull) ? 0xFFFFFFFFu : static_cast<uint32_t>(xm - 1),
                          cum | (dsh << 16) | (raw ? 1u << 31 : 0u),
                          e.w | (f == 0 ? (1u << 23) : 0u) | (inc << 24));
    }
}

// x + cum + q (M - f) from a staged entry (cum in the low half of z, M - f in
// the low 24 bits of w): one add reading z's low half in place and one
// 24-bit multiply-add, where the compiler otherwise masks, multiplies and
// adds three operands.
__device__ __forceinline__ uint32_t c_update(uint32_t x, uint32_t q, uint32_t z, uint32_t w)
{
    uint32_t xc, xn;
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_0"
        : "=v"(xc)
        : "v"(x), "v"(z));
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(xn) : "v"(q), "v"(w), "v"(xc));
    return xn;
}

// One encoder step (Algorithm 1's Encode with rANS's C) for every lane:
// emits the digits the renormalisation drops into the wave's LDS digit ring
// (at their slot positions modulo the ring; positions from a ballot prefix,
// the stream growing downwards), then applies C.  bad collects the entries'
// bit 23 (a symbol the table cannot encode).  e: the symbol's staged entry
// (read ahead by the caller).  BF: breadth-first digit order (Section 5):
// the step's block holds the first digit of every emitting lane, then the
// second digit of every lane that emits two; depth-first keeps a lane's two
// digits together.  Either way a lane's more significant digit is read first.
// ONE (byte digits): the table is a one-digit table (every f is 0 or at least
// M / 256), so no lane emits a second digit and the step has one compare,
// one ballot, one prefix count and one store.
template <int R, bool BF = false, bool FULL = false, bool ONE = false>
__device__ __forceinline__ void enc_step(uint32_t& x, uint32_t& wpos, uint32_t& bad, const uint4& e,
                                         bool act, uint32_t ringv, uint32_t junkv)
{
    constexpr uint32_t RD = kEncRing / (R / 8);  // ring size in digits
    // idle lanes keep their state through selects, not branches (an
    // exec-mask branch per step splits the unrolled loop into blocks);
    // FULL: every lane is active
    bad |= FULL || act ? e.w : 0u;
    // the emitting lanes store, each at its digit's ring position (ringv, the
    // ring's LDS address in a vector register, is a multiple of the ring's
    // size: the position's bits are or-ed in)
    if (R == 16) {
        uint64_t m;
        uint32_t xs;
        if (FULL) {
            m = gt_shift16(x, e.y, &xs);
        } else {
            const bool e1 = act && x > e.y;
            m = ballot(e1);
            xs = e1 ? x >> 16 : x;
        }
        wpos -= __popcll(m);
        ring_store<2>(m, (((mbcnt(m, 0) + wpos) << 1) & (2 * RD - 1)) | ringv, junkv, x);
        x = xs;
    } else if (ONE) {
        const bool e1 = (FULL || act) && x > e.y;
        const uint64_t m1 = ballot(e1);
        wpos -= __popcll(m1);
        ring_store<1>(m1, ((mbcnt(m1, 0) + wpos) & (RD - 1)) | ringv, junkv, x);
        x = e1 ? x >> 8 : x;
    } else {
        const bool e1 = (FULL || act) && x > e.y;
        const bool e2 = (FULL || act) && (x >> 8) > e.y;
        const uint64_t m1 = ballot(e1), m2 = ballot(e2);
        wpos -= __popcll(m1) + __popcll(m2);
        uint32_t i1, i2;
        if (BF) {
            i1 = mbcnt(m1, 0) + wpos;
            i2 = mbcnt(m2, 0) + (wpos + __popcll(m1));
        } else {
            i1 = mbcnt(m1, mbcnt(m2, 0)) + wpos;
            i2 = i1 + 1;
        }
        ring_store<1>(m1, (i1 & (RD - 1)) | ringv, junkv, e2 ? x >> 8 : x);
        ring_store<1>(m2, (i2 & (RD - 1)) | ringv, junkv, x);
        x = e2 ? x >> 16 : (e1 ? x >> 8 : x);
    }
    // C(s, x) = M q + (x - q f) + cum = x + q (M - f) + cum, q = x / f by
    // one multiply-high (the entry's m, inc and shift); the 24-bit multiply
    // reads M - f (bit 23 is set only on entries that are errors)
    const uint32_t q = __umulhi(e.x, x + (e.w >> 24)) >> ((e.z >> 16) & 31u);
    const uint32_t xn = c_update(x, q, e.z, e.w);
    x = FULL || act ? xn : x;
}

// Encoder step with escape coding (16-bit symbols, depth-first).  The value
// v is coded as the symbol v when the table has it (v < E, f_v > 0) and as
// the escape E otherwise; an escape lane also emits 16 raw bits holding v.
// The decoder reads them after the lane's renormalisation digits, so they
// follow those digits in the stream (Section 3: the encoder sends raw data
// just before it encodes the symbol they belong to).  e: the entry staged
// for min(v, alphabet) by stage_enc with the escape, which is already the
// escape's entry, with bit 31 of z set, when v must escape.
template <int R>
__device__ __forceinline__ void enc_step_esc(uint32_t& x, uint32_t& wpos, uint32_t& bad, const uint4& e,
                                             uint32_t v, bool act, uint32_t ringv, uint32_t junkv)
{
    constexpr uint32_t RD = kEncRing / (R / 8);  // ring size in digits
    const bool esc = act && (e.z >> 31) != 0;
    bad |= act ? e.w : 0u;
    const bool e1 = act && x > e.y;
    const uint64_t m1 = ballot(e1), me = ballot(esc);
    if (R == 16) {
        wpos -= __popcll(m1) + __popcll(me);
        const uint32_t i1 = mbcnt(m1, mbcnt(me, wpos));
        ring_store<2>(m1, ((i1 << 1) & (2 * RD - 1)) | ringv, junkv, x);
        ring_store<2>(me, (((i1 + (e1 ? 1u : 0u)) << 1) & (2 * RD - 1)) | ringv, junkv, v);
        x = e1 ? x >> 16 : x;
    } else {
        const bool e2 = act && (x >> 8) > e.y;
        const uint64_t m2 = ballot(e2);
        wpos -= __popcll(m1) + __popcll(m2) + 2 * __popcll(me);
        const uint32_t i1 = wpos + (mbcnt(m1, 0) + mbcnt(m2, 0) + 2 * mbcnt(me, 0));
        const uint32_t ir = i1 + (e1 ? 1u : 0u) + (e2 ? 1u : 0u);  // raw bytes after the renormalisation bytes
        ring_store<1>(m1, (i1 & (RD - 1)) | ringv, junkv, e2 ? x >> 8 : x);
        ring_store<1>(m2, ((i1 + 1) & (RD - 1)) | ringv, junkv, x);
        ring_store<1>(me, (ir & (RD - 1)) | ringv, junkv, v >> 8);
        ring_store<1>(me, ((ir + 1) & (RD - 1)) | ringv, junkv, v);
        x = e2 ? x >> 16 : (e1 ? x >> 8 : x);
    }
    const uint32_t q = __umulhi(e.x, x + (e.w >> 24)) >> ((e.z >> 16) & 31u);
    x = act ? c_update(x, q, e.z, e.w) : x;
}

// Encodes chunk `chunk` of syms_base (n symbols, C per chunk, NL = 32 or 64
// interleaved coders) into the digit slot `slot` (digits end at slot +
// slot_bytes, a multiple of kEncWindow; kSlotPad more bytes follow), writes the NL final
// states to states_out and the digit count to *ndig_out (or to the
// caller's x_out / nd_out).  l_enc: LDS encoder entries staged by stage_enc
// (alphabet + 1 entries; 256 with 8-bit symbols, which index it unclamped);
// ring: this wave's kEncRing-byte digit ring (at an LDS address that is a
// multiple of kEncRing); sbuf: its kEncSymArea-byte symbol area.  Digits reach the slot from the
// LDS ring a window at a time, one 16-byte store per lane: after every block
// of symbols, the windows the stream has grown past, padded to kFlushStores
// stores with stores to the kSlotPad bytes after the slot.  A fixed
// number of memory operations per block lets the compiler's wait for the
// symbols of the next block leave the recent stores in flight.  BF: as in
// enc_step.  ESC: escape coding, as in enc_step_esc; l_enc staged with the
// escape (a 1 KiB block of 16-bit symbols still emits at most 2 KiB: 4
// bytes per symbol).  ONE: as in enc_step (a one-digit table, byte digits).
template <int R, int W, int NL, bool BF = false, bool ESC = false, bool ONE = false>
__device__ __forceinline__ void encode_chunk(const void* syms_base, uint64_t n, uint32_t C, uint64_t chunk,
                                             uint32_t k, uint32_t l, uint32_t alphabet,
                                             const uint4* l_enc, uint8_t* slot, uint64_t slot_bytes,
                                             uint8_t* ring, uint8_t* sbuf, uint32_t* states_out, uint32_t* ndig_out,
                                             int32_t* status, uint32_t* x_out = nullptr,
                                             uint32_t* nd_out = nullptr)
{
    static_assert(!ESC || (W == 2 && !BF), "escape coding: 16-bit symbols, depth-first");
    using InT = typename std::conditional<W == 1, uint8_t, uint16_t>::type;
    constexpr uint32_t SPB = 1024 / (W * NL);  // steps per 1 KiB symbol block
    constexpr uint32_t DB = R / 8, WD = kEncWindow / DB;  // bytes per digit, digits per window
    const uint32_t lane = threadIdx.x & 63;
    const bool live = NL == 64 || lane < NL;
    const uint8_t* dring = ring;
    const uint32_t ringv = in_vgpr(lds_addr(ring));
    const uint32_t junkv = lds_addr(sbuf) + kEncSymBlock + 2 * lane;
    const uint64_t first = chunk * C;
    const uint32_t nsym = uni(static_cast<uint32_t>(n - first < C ? n - first : C));
    const InT* in = static_cast<const InT*>(syms_base) + first;
    const uint32_t steps = (nsym + NL - 1) / NL;
    const uint32_t nblk = nsym / (NL * SPB);  // whole blocks
    const uint32_t top = uni(static_cast<uint32_t>(slot_bytes / DB));
    uint32_t x = 1u << l;
    uint32_t wpos = top;  // lowest digit written so far
    uint32_t wtop = top;  // digits from wtop up are in the slot
    uint32_t bad = 0;

    auto ring_word = [&](uint32_t lo) {  // this lane's 16 bytes of the ring window of digits [lo, lo + WD)
        return reinterpret_cast<const uint4*>(dring + ((lo * DB) & (kEncRing - 1)))[lane];
    };
    auto flush = [&]() {
        const uint32_t wc = (wpos + WD - 1) / WD * WD;  // lowest window boundary at or above wpos
        const uint32_t cnt = (wtop - wc) / WD;          // complete windows not yet stored (<= 2)
        lane_fence();
#pragma unroll
        for (uint32_t j = 0; j < kFlushStores; ++j) {
            const uint32_t lo = wtop - (j + 1) * WD;
            uint8_t* dst = j < cnt ? slot + uint64_t(lo) * DB : slot + slot_bytes;
            const uint4 v = ring_word(lo);
            gstore(reinterpret_cast<uint4*>(dst) + lane, v);
        }
        lane_fence();
        wtop = wc;
    };

    // steps above the whole blocks (the partial tail), one at a time
    for (uint32_t t = steps; t-- > nblk * SPB;) {
        const uint64_t i = uint64_t(t) * NL + lane;
        const bool act = live && i < nsym;
        const uint32_t s = act ? static_cast<uint32_t>(gmem(in)[i]) : 0u;
        if (ESC)
            enc_step_esc<R>(x, wpos, bad, l_enc[min(s, alphabet)], s, act, ringv, junkv);
        else
            enc_step<R, BF, false, ONE>(x, wpos, bad, l_enc[W == 1 ? s : min(s, alphabet)], act, ringv, junkv);
    }
    flush();  // the tail is shorter than a block: at most 2 windows

    if (nblk > 0) {
        // block b = symbols [b*NL*SPB, (b+1)*NL*SPB); lane loads 16 bytes,
        // marked non-temporal (each symbol is read once)
        const uint4* blk = reinterpret_cast<const uint4*>(in) + lane;
        auto load_blk = [&](int64_t b) {
            const v4u v = __builtin_nontemporal_load(gmem(reinterpret_cast<const v4u*>(blk + (b < 0 ? 0 : b) * 64)));
            return make_uint4(v.x, v.y, v.z, v.w);
        };
        // The block's symbols are read from LDS up front and each step's
        // entry PF steps ahead, in program order before the steps' digit
        // writes: the reads stay off the state's dependency chain.
        // A block of 32 steps (8-bit symbols, N = 32) runs as two halves of
        // 16, so that its symbols fit in registers next to the rest.
        constexpr int PF = 3;
        constexpr int HB = SPB > 16 ? 16 : int(SPB);
        auto run_blk = [&](uint4 v) {
            lane_fence();
            *reinterpret_cast<uint4*>(sbuf + 16 * lane) = v;
            lane_fence();
            const InT* sb = reinterpret_cast<const InT*>(sbuf) + lane;
#pragma unroll
            for (int h = int(SPB) / HB - 1; h >= 0; --h) {
                uint32_t sy[HB];  // entry index (ESC: the value itself)
                if (h + 1 < int(SPB) / HB)
                    lane_fence();  // read after the first half's steps
#pragma unroll
                for (int q = 0; q < HB; ++q) {
                    const uint32_t v0 = static_cast<uint32_t>(sb[(h * HB + q) * NL]);
                    sy[q] = ESC || W == 1 ? v0 : min(v0, alphabet);
                }
                lane_fence();  // the symbols are in registers before the ring writes
                auto entry = [&](int q) { return l_enc[ESC ? min(sy[q], alphabet) : sy[q]]; };
                uint4 ent[HB];
#pragma unroll
                for (int q = HB - 1; q >= HB - PF && q >= 0; --q)
                    ent[q] = entry(q);
#pragma unroll
                for (int q = HB - 1; q >= 0; --q) {
                    if (q - PF >= 0)
                        ent[q - PF] = entry(q - PF);
                    if (ESC)
                        enc_step_esc<R>(x, wpos, bad, ent[q], sy[q], live, ringv, junkv);
                    else
                        enc_step<R, BF, NL == 64, ONE>(x, wpos, bad, ent[q], live, ringv, junkv);
                }
            }
            flush();
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
    if (wpos < wtop) {  // the window holding the stream's first digits
        lane_fence();
        const uint4 v = ring_word(wtop - WD);
        gstore(reinterpret_cast<uint4*>(slot + uint64_t(wtop - WD) * DB) + lane, v);
    }
    if (states_out && live)
        states_out[lane] = x;
    if (ndig_out && lane == 0)
        *ndig_out = top - wpos;
    if (x_out)
        *x_out = x;
    if (nd_out)
        *nd_out = top - wpos;
    if (ballot((bad >> 23) & 1) && lane == 0)
        atomicMin(status, RANS_ENOSYM);
}

// 16 bytes starting `mis` bytes into the 32-byte window lo:hi (mis uniform).
__device__ __forceinline__ uint4 funnel16(const uint4& lo, const uint4& hi, uint32_t mis)
{
    uint32_t a0, a1, a2, a3, a4;
    switch (mis >> 2) {
    case 0: a0 = lo.x; a1 = lo.y; a2 = lo.z; a3 = lo.w; a4 = hi.x; break;
    case 1: a0 = lo.y; a1 = lo.z; a2 = lo.w; a3 = hi.x; a4 = hi.y; break;
    case 2: a0 = lo.z; a1 = lo.w; a2 = hi.x; a3 = hi.y; a4 = hi.z; break;
    default: a0 = lo.w; a1 = hi.x; a2 = hi.y; a3 = hi.z; a4 = hi.w; break;
    }
    const uint32_t b = mis & 3;
    return make_uint4(__builtin_amdgcn_alignbyte(a1, a0, b), __builtin_amdgcn_alignbyte(a2, a1, b),
                      __builtin_amdgcn_alignbyte(a3, a2, b), __builtin_amdgcn_alignbyte(a4, a3, b));
}

constexpr uint64_t kFlag = 1ull << 62, kValMask = kFlag - 1;

// Sum over the wave of one 64-bit value per lane.
__device__ __forceinline__ uint64_t wave_sum(uint64_t v)
{
    for (int d = 32; d >= 1; d >>= 1)
        v += static_cast<uint64_t>(__shfl_xor(static_cast<long long>(v), d));
    return v;
}

// Lane-parallel wait for a published word (flag bit set); bounded spin.
// The words carry self-contained values (lengths) and order nothing else, so
// they are relaxed device-scope atomics: coherent across the chip's L2
// slices without the whole-L2 write-back / invalidate that acquire and
// release would add to every publish and every spin iteration.
__device__ __forceinline__ uint64_t await_word(const uint64_t* w, bool& timeout)
{
    uint32_t spins = 0;
    for (;;) {
        const uint64_t v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (v & kFlag)
            return v & kValMask;
        if (++spins > (1u << 22)) {
            timeout = true;
            return 0;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

// Prefix-code encoder of one chunk (the second coder family, multiplexed as
// Section 4 describes).  Lane j codes symbols j, j + NL, ... with the
// canonical prefix code and, step by step, applies its decoder's read rule
// to its own bit count: the decoder reads one 16-bit word before a symbol
// whenever it holds fewer than 16 bits.  The lanes that read in a step take
// consecutive positions of the multiplexed stream (a ballot prefix) -- the
// order in which the instrumented decoder would copy the words -- and each
// word is stored at its position once the lane's bits complete it, at most
// two reads later (the decoder holds at most 31 bits).  penc: LDS, alphabet
// + 1 entries code | len << 16 (len 0: the symbol cannot be coded).  Words
// go to mux[0 ..) (global); the NL bit counts to *x_out (per lane), the word
// count to *nd_out.
template <int W, int NL>
__device__ __forceinline__ void encode_chunk_pfx(const void* syms_base, uint64_t n, uint32_t C, uint64_t chunk,
                                                 uint32_t alphabet, const uint32_t* penc, uint16_t* mux,
                                                 int32_t* status, uint32_t* x_out, uint32_t* nd_out)
{
    using InT = typename std::conditional<W == 1, uint8_t, uint16_t>::type;
    const uint32_t lane = threadIdx.x & 63;
    const bool live = NL == 64 || lane < NL;
    const uint64_t first = chunk * C;
    const uint32_t nsym = uni(static_cast<uint32_t>(n - first < C ? n - first : C));
    const InT* in = static_cast<const InT*>(syms_base) + first;
    const uint32_t steps = (nsym + NL - 1) / NL;
    uint64_t acc = 0;      // code bits not yet in a word (nacc of them)
    uint32_t nacc = 0;
    uint32_t nbd = 0;      // bits the lane's decoder holds
    uint32_t q0 = 0, q1 = 0, npend = 0;  // positions read, words not yet complete
    uint32_t bits = 0, wpos = 0, bad = 0;
    constexpr uint32_t PF = 16;  // symbols loaded this many steps ahead
    auto load = [&](uint32_t t) -> uint32_t {
        const uint64_t i = uint64_t(t) * NL + lane;
        return live && i < nsym ? static_cast<uint32_t>(in[i]) : 0u;
    };
    uint32_t cur[PF], nxt[PF];
#pragma unroll
    for (uint32_t q = 0; q < PF; ++q)
        cur[q] = load(q);
    for (uint32_t t0 = 0; t0 < steps; t0 += PF) {
#pragma unroll
        for (uint32_t q = 0; q < PF; ++q)
            nxt[q] = load(t0 + PF + q);
        // the block's code entries, read before its steps: the LDS latency
        // stays off the steps' chain
        uint32_t ent[PF];
#pragma unroll
        for (uint32_t q = 0; q < PF; ++q)
            ent[q] = penc[min(cur[q], alphabet)];
#pragma unroll
        for (uint32_t q = 0; q < PF; ++q) {
            const uint32_t t = t0 + q;
            const bool act = live && uint64_t(t) * NL + lane < nsym;
            const bool rd = act && nbd < 16;
            const uint64_t m = ballot(rd);
            if (rd) {
                const uint32_t pos = wpos + mbcnt(m, 0);
                if (npend == 0)
                    q0 = pos;
                else
                    q1 = pos;
                ++npend;
                nbd += 16;
            }
            wpos += __popcll(m);
            if (act) {
                const uint32_t e = ent[q];
                const uint32_t len = e >> 16;
                bad |= len == 0 ? 1u : 0u;
                acc = (acc << len) | (e & 0xFFFFu);
                nacc += len;
                nbd -= len;
                bits += len;
                if (nacc >= 16) {  // a code has at most 15 bits: one word at most
                    nacc -= 16;
                    mux[q0] = static_cast<uint16_t>(acc >> nacc);
                    acc &= (1ull << nacc) - 1;
                    q0 = q1;
                    --npend;
                }
            }
        }
#pragma unroll
        for (uint32_t q = 0; q < PF; ++q)
            cur[q] = nxt[q];
    }
    // the last partial word (zero padded), and a word of zeros when the
    // decoder's rule reads one beyond the bits
    if (live && npend > 0) {
        mux[q0] = static_cast<uint16_t>(nacc ? acc << (16 - nacc) : 0u);
        if (npend > 1)
            mux[q1] = 0;
    }
    if (ballot(bad != 0) && lane == 0)
        atomicMin(status, RANS_ENOSYM);
    *x_out = live ? bits : 0u;
    *nd_out = wpos;
}

// Places encoded chunk `chunk` (NL final states in x, nd digits starting at
// src, a 16-byte aligned address with at least 32 readable bytes past the
// digits) into the container.  Its offset is the sum of the
// padded lengths of all lower chunks, found in two lane-parallel levels:
// every chunk publishes its length; the lengths of the lower chunks of its
// own group of 64 are read one per lane and summed; the last chunk of each
// group publishes the group's total; the totals of the lower groups are
// read 64 at a time and summed.  A chunk only waits on lower chunks, which
// started earlier (chunk indices come from a ticket in start order), so the
// waits end; they are bounded anyway, and a timeout reports RANS_EINVAL and
// writes nothing.  p.lookback holds nch chunk words, then the group words,
// all zero before the kernel.
// Publishes chunk `chunk`'s aligned length (nd digits) for the look-back of
// the chunks above it.
template <int R, int NL>
__device__ __forceinline__ void publish_chunk(uint32_t chunk, uint32_t nd, const PlaceArgs& p)
{
    const uint64_t al = (uint64_t(4 * NL + nd * (R / 8)) + 15) & ~15ull;
    if ((threadIdx.x & 63) == 0)
        __hip_atomic_store(&p.lookback[chunk], kFlag | al, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The sum of the aligned lengths of the chunks below `chunk` in its group
// of 64 (awaited); the group's last chunk also publishes the group total.
template <int R, int NL>
__device__ __forceinline__ uint64_t chunk_local(uint32_t chunk, uint32_t nch, uint32_t nd, const PlaceArgs& p,
                                                bool& timeout)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t al = (uint64_t(4 * NL + nd * (R / 8)) + 15) & ~15ull;
    const uint32_t g = chunk >> 6, g0 = chunk & ~63u;
    const uint64_t local = wave_sum(g0 + lane < chunk ? await_word(&p.lookback[g0 + lane], timeout) : 0);
    if ((chunk & 63) == 63 && lane == 0)
        __hip_atomic_store(&p.lookback[nch + g], kFlag | (local + al), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return local;
}

// Places a chunk: publish its length, sum its predecessors' (its group's,
// then the earlier groups' totals), write its directory entry, states and
// digits.  pre: a wave that codes two chunks publishes both lengths and
// takes both group sums (local, timeout) before placing either, so that no
// chunk above them, in this group or a later one, waits on its copies.
template <int R, int NL>
__device__ __forceinline__ void place_chunk(uint32_t chunk, uint32_t nch, uint32_t x, uint32_t nd,
                                            const uint8_t* src, const PlaceArgs& p, int32_t* status,
                                            bool pre = false, uint64_t pre_local = 0, bool pre_timeout = false)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t pay = nd * (R / 8);
    const uint32_t len = 4 * NL + pay;
    const uint64_t al = (uint64_t(len) + 15) & ~15ull;
    uint64_t* grp = p.lookback + nch;
    bool timeout = pre_timeout;
    uint64_t local = pre_local;
    if (!pre) {
        publish_chunk<R, NL>(chunk, nd, p);
        local = chunk_local<R, NL>(chunk, nch, nd, p, timeout);
    }
    const uint32_t g = chunk >> 6;
    uint64_t before = 0;
    for (uint32_t b = 0; b < g; b += 64)
        before += wave_sum(b + lane < g ? await_word(&grp[b + lane], timeout) : 0);
    const uint64_t excl = uni64(before + local);
    timeout = ballot(timeout) != 0;
    const uint64_t base = (kHeaderBytes + uint64_t(kDirEntryBytes) * nch + 15) & ~15ull;
    const uint64_t off = base + excl;
    const bool fits = !timeout && off + al <= p.out_cap;
    if (fits) {
        uint8_t* dst = p.out + off;
        if (lane == 0) {
            uint32_t* de = reinterpret_cast<uint32_t*>(p.out + kHeaderBytes + uint64_t(kDirEntryBytes) * chunk);
            *reinterpret_cast<uint64_t*>(de) = off;
            de[2] = len;
            de[3] = 0;
        }
        if (NL == 64 || lane < NL)
            reinterpret_cast<uint32_t*>(dst)[lane] = x;
        const uint32_t mis = static_cast<uint32_t>(reinterpret_cast<uintptr_t>(src) & 15);
        // reads reach at most 31 bytes past the digits
        const uint4* S = reinterpret_cast<const uint4*>(src - mis);
        uint4* D = reinterpret_cast<uint4*>(dst + 4 * NL);
        const uint32_t pieces = static_cast<uint32_t>((al - 4 * NL) / 16);
        auto piece = [&](uint32_t q, const uint4& lo, const uint4& hi) {
            uint4 v = funnel16(lo, hi, mis);
            const uint32_t have = pay - 16 * q;  // > 0 for every piece
            if (have < 16) {
                const uint32_t keep[4] = {have >= 4 ? 4u : have, have >= 8 ? 4u : (have > 4 ? have - 4 : 0u),
                                          have >= 12 ? 4u : (have > 8 ? have - 8 : 0u),
                                          have > 12 ? have - 12 : 0u};
                auto m = [](uint32_t w, uint32_t nb) { return nb >= 4 ? w : (nb ? w & ((1u << (8 * nb)) - 1) : 0u); };
                v = make_uint4(m(v.x, keep[0]), m(v.y, keep[1]), m(v.z, keep[2]), m(v.w, keep[3]));
            }
            v4u t;  // the container is not read again here: a non-temporal store
            t.x = v.x;
            t.y = v.y;
            t.z = v.z;
            t.w = v.w;
            __builtin_nontemporal_store(t, gmem(reinterpret_cast<v4u*>(D + q)));
        };
        // KU rounds of loads in flight before their stores: one round at a
        // time would wait a full memory latency per KiB.  Two rounds keep
        // the copy's registers (four 16-byte loads per lane) under what the
        // coding loop holds, so the copy does not set the kernel's register
        // count: about 80, six waves per SIMD, where eight rounds took the
        // encoders to 117-127 registers and four waves per SIMD.
        constexpr uint32_t KU = 2;
        uint32_t q0 = lane;
        for (; q0 + 64 * (KU - 1) < pieces; q0 += 64 * KU) {
            uint4 lo[KU], hi[KU];
#pragma unroll
            for (uint32_t u = 0; u < KU; ++u) {
                lo[u] = gload16(S + q0 + 64 * u);
                hi[u] = gload16(S + q0 + 64 * u + 1);
            }
#pragma unroll
            for (uint32_t u = 0; u < KU; ++u)
                piece(q0 + 64 * u, lo[u], hi[u]);
        }
        for (uint32_t q = q0; q < pieces; q += 64)
            piece(q, gload16(S + q), gload16(S + q + 1));
    } else if (lane == 0) {
        atomicMin(status, timeout ? RANS_EINVAL : RANS_ENOSPC);
    }
    if (chunk + 1 == nch && lane == 0) {
        const uint64_t total = off + al;
        *p.total = total;
        if (p.total_out)
            *p.total_out = total;
        if (!timeout && total <= p.out_cap) {
            uint32_t* h = reinterpret_cast<uint32_t*>(p.out);
            for (int q = 0; q < 8; ++q)
                h[q] = reinterpret_cast<const uint32_t*>(p.hdr)[q];
        }
    }
}

}  // namespace c64
}  // namespace rans
