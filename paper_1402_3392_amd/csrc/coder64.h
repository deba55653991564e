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

constexpr uint32_t kWin = 512;       // stream window bytes
constexpr uint32_t kRing = 2 * kWin + 128;  // two windows + mirror of slot 0's head

// Output block per wave: 1 KiB, or 512 bytes next to the large fused table.
constexpr uint32_t obuf_bytes(int layout) { return layout == kFused ? 512 : 1024; }
constexpr uint32_t wave_lds_bytes(int layout) { return obuf_bytes(layout) + kRing; }

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

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// 8-byte variant of async_load.
__device__ __forceinline__ u32x2 async_load2(const uint8_t* p)
{
    u32x2 v;
    asm volatile("global_load_dwordx2 %0, %1, off" : "=v"(v) : "v"(p) : "memory");
    return v;
}

// Per lane: b where the lane's bit of mask m is set, a elsewhere (one
// v_cndmask on the ballot mask, no exec-mask branch).
__device__ __forceinline__ uint32_t select_mask(uint64_t m, uint32_t a, uint32_t b)
{
    uint32_t r;
    asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(m));
    return r;
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
    constexpr uint32_t OB = obuf_bytes(LAYOUT);
    uint8_t* obuf = wave_lds;        // output block
    uint8_t* ring = wave_lds + OB;   // two 512-byte windows + 128-byte mirror
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

    // Window w = payload bytes [w*512, w*512+512); lane fetches 8 of them.
    // Addresses past the container are clamped to its last whole 8 bytes, so
    // every load is issued (the wait counts rely on that) and stays inside.
    const uint64_t room = (in_len - 8) & ~7ull;  // in_len >= 32 here
    const uint64_t pay_off = off + 256 + 8 * lane;
    auto waddr = [&](uint32_t w) -> const uint8_t* {
        const uint64_t o = pay_off + uint64_t(w) * kWin;
        return in + (o <= room ? o : room);
    };
    // window w lives in ring slot w & 1; slot 0's first 128 bytes are mirrored
    // after slot 1, so a step's reads (< 128 bytes past any position) need no
    // wrap-around
    auto put_window = [&](uint32_t w, const u32x2& v) {
        *reinterpret_cast<u32x2*>(ring + (w & 1) * kWin + 8 * lane) = v;
        if ((w & 1) == 0 && lane < 16)
            *reinterpret_cast<u32x2*>(ring + 2 * kWin + 8 * lane) = v;
    };
    uint32_t x = async_load(in + off + 4 * lane);  // coder `lane`'s initial state
    u32x2 p0 = async_load2(waddr(0));
    u32x2 p1 = async_load2(waddr(1));
    u32x2 p2 = async_load2(waddr(2));
    u32x2 p3 = async_load2(waddr(3));
    wait_vm<2>();
    put_window(0, p0);
    put_window(1, p1);
    p0 = async_load2(waddr(4));
    p1 = async_load2(waddr(5));
    // ring holds windows kw, kw+1; p[(kw+2)%4 ..] hold kw+2 .. kw+5 in flight

    constexpr uint32_t WD = kWin / (R / 8);    // digits per window
    constexpr uint32_t SPB = OB / (64 * W);    // steps per output block
    constexpr uint32_t PIECE = OB / 64;         // bytes each lane moves per block
    using Piece = typename std::conditional<PIECE == 16, uint4, uint2>::type;
    const uint32_t full = nsym / 64;           // steps with all lanes active
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
    // Refill: every lane reads the ring at its would-be offset (the prefix
    // count of refilling lanes below it) and a select on the ballot keeps
    // the word in the lanes that need it.  The step is skipped as a whole
    // when no lane refills.
    auto refill = [&](bool act) {
        const bool n1 = act && x < L;
        const uint64_t m1 = ballot(n1);
        if (R == 16) {
            if (m1) {
                const uint32_t at = 2 * (pos & (2 * WD - 1));
                const uint32_t v = *reinterpret_cast<const uint16_t*>(ring + at + 2 * mbcnt(m1, 0));
                x = select_mask(m1, x, (x << 16) | v);
                pos += __popcll(m1);
            }
        } else {
            const bool n2 = act && x < (L >> 8);
            const uint64_t m2 = ballot(n2);
            if (m1) {
                const uint8_t* r = ring + (pos & (2 * WD - 1)) + mbcnt(m2, mbcnt(m1, 0));
                const uint32_t x1 = (x << 8) | r[0];
                const uint32_t x2 = (x1 << 8) | r[1];
                x = select_mask(m1, x, select_mask(m2, x1, x2));
                pos += __popcll(m1) + __popcll(m2);
            }
        }
    };
    auto flush = [&](uint32_t tb) {  // output block starting at step tb
        const Piece v = *reinterpret_cast<const Piece*>(obuf + PIECE * lane);
        *reinterpret_cast<Piece*>(reinterpret_cast<uint8_t*>(out + uint64_t(tb) * 64) + PIECE * lane) = v;
    };
    auto step1 = [&](OutT* dst) {
        uint32_t s;
        decode_one(s);
        refill(true);
        *dst = static_cast<OutT>(s);
    };
    // four full steps; t is a multiple of 4 here, so the output offsets are
    // immediates and a block ends exactly at a multiple of four
    auto step4 = [&]() {
        OutT* o4 = ob + (t & (SPB - 1)) * 64;
        step1(o4);
        step1(o4 + 64);
        step1(o4 + 128);
        step1(o4 + 192);
        t += 4;
        if ((t & (SPB - 1)) == 0)
            flush(t - SPB);
    };
    auto step_single = [&]() {
        step1(ob + (t & (SPB - 1)) * 64);
        ++t;
        if ((t & (SPB - 1)) == 0)
            flush(t - SPB);
    };
    // last, partial step: only lanes below nsym % 64 take part
    auto partial_step = [&]() {
        const bool act = lane < nsym - t * 64;
        uint32_t s = 0;
        if (act)
            decode_one(s);
        refill(act);
        ob[(t & (SPB - 1)) * 64] = static_cast<OutT>(s);
        ++t;
    };

    // Four steps read fewer than WD digits, so with pos < wend (= (kw+1)*WD)
    // they stay inside the resident windows kw, kw+1: the window test runs
    // once per four steps.  When fewer than four full steps remain, one shift
    // (if pos has entered window kw+1) keeps the rest inside the ring too.
    bool done = false;
#define RANS_SHIFT(PREG)                                                   \
    do {                                                                   \
        wait_vm<3>();                                                      \
        put_window(kw + 2, PREG);                                          \
        PREG = async_load2(waddr(kw + 6));                                 \
        ++kw;                                                              \
        wend += WD;                                                        \
    } while (0)
#define RANS_PHASE(PREG)                                                   \
    if (!done) {                                                           \
        while (t + 4 <= full && pos < wend)                                \
            step4();                                                       \
        if (t + 4 <= full) {                                               \
            RANS_SHIFT(PREG);                                              \
        } else {                                                           \
            if (pos >= wend)                                               \
                RANS_SHIFT(PREG);                                          \
            while (t < full)                                               \
                step_single();                                             \
            if (t < steps)                                                 \
                partial_step();                                            \
            done = true;                                                   \
        }                                                                  \
    }
    while (!done) {
        RANS_PHASE(p2)
        RANS_PHASE(p3)
        RANS_PHASE(p0)
        RANS_PHASE(p1)
    }
#undef RANS_PHASE
#undef RANS_SHIFT
    // Blocks that ended inside the full steps were flushed; the rest,
    // [tb, steps), holds the ragged end: whole lane pieces, then the one
    // lane that straddles the end byte by byte.
    const uint32_t tb = (full / SPB) * SPB;
    if (tb < steps) {
        const uint32_t nbytes = (nsym - tb * 64) * W;  // valid bytes of this block
        uint8_t* dst = reinterpret_cast<uint8_t*>(out + uint64_t(tb) * 64);
        if (PIECE * lane + PIECE <= nbytes) {
            *reinterpret_cast<Piece*>(dst + PIECE * lane) = *reinterpret_cast<const Piece*>(obuf + PIECE * lane);
        } else if (PIECE * lane < nbytes) {
            for (uint32_t b = PIECE * lane; b < nbytes; ++b)
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
                                             int32_t* status, uint32_t* x_out = nullptr,
                                             uint32_t* nd_out = nullptr)
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
    if (states_out)
        states_out[lane] = x;
    if (ndig_out && lane == 0)
        *ndig_out = static_cast<uint32_t>(slot_bytes / (R / 8)) - wpos;
    if (x_out)
        *x_out = x;
    if (nd_out)
        *nd_out = static_cast<uint32_t>(slot_bytes / (R / 8)) - wpos;
    if (ballot(nosym) && lane == 0)
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

constexpr uint64_t kFlagAgg = 1ull << 62, kFlagInc = 2ull << 62, kValMask = (1ull << 62) - 1;

// Places encoded chunk `chunk` (64 final states in x, nd digits ending at
// slot + slot_bytes) into the container by decoupled look-back over the
// published lengths of its predecessors, which all started earlier (chunk
// indices are taken from a ticket in start order), so the walk ends.  The
// walk is bounded; a timeout reports RANS_EINVAL and writes nothing.
template <int R>
__device__ __forceinline__ void place_chunk(uint32_t chunk, uint32_t nch, uint32_t x, uint32_t nd,
                                            const uint8_t* slot, uint64_t slot_bytes,
                                            const PlaceArgs& p, int32_t* status)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t pay = nd * (R / 8);
    const uint32_t len = 256 + pay;
    const uint64_t al = (uint64_t(len) + 15) & ~15ull;
    uint64_t excl = 0;
    uint32_t timeout = 0;
    if (lane == 0) {
        if (chunk == 0) {
            __hip_atomic_store(&p.lookback[0], kFlagInc | al, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(&p.lookback[chunk], kFlagAgg | al, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
            uint64_t j = chunk - 1;
            uint32_t spins = 0;
            for (;;) {
                const uint64_t v =
                    __hip_atomic_load(&p.lookback[j], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                if ((v >> 62) == 2) {
                    excl += v & kValMask;
                    break;
                }
                if ((v >> 62) == 1) {
                    excl += v & kValMask;
                    --j;  // chunk 0 publishes an inclusive value, so j stays >= 0
                    continue;
                }
                if (++spins > (1u << 22)) {
                    timeout = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            __hip_atomic_store(&p.lookback[chunk], kFlagInc | (excl + al), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    excl = uni64(excl);  // lane 0 is the first active lane
    timeout = uni(timeout);
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
        reinterpret_cast<uint32_t*>(dst)[lane] = x;
        const uint8_t* src = slot + slot_bytes - pay;
        const uint32_t mis = static_cast<uint32_t>(reinterpret_cast<uintptr_t>(src) & 15);
        // reads reach at most 31 bytes past the slot: inside its junk area
        const uint4* S = reinterpret_cast<const uint4*>(src - mis);
        uint4* D = reinterpret_cast<uint4*>(dst + 256);
        const uint32_t pieces = static_cast<uint32_t>((al - 256) / 16);
        for (uint32_t q = lane; q < pieces; q += 64) {
            uint4 v = funnel16(S[q], S[q + 1], mis);
            const uint32_t have = pay - 16 * q;  // > 0 for every piece
            if (have < 16) {
                const uint32_t keep[4] = {have >= 4 ? 4u : have, have >= 8 ? 4u : (have > 4 ? have - 4 : 0u),
                                          have >= 12 ? 4u : (have > 8 ? have - 8 : 0u),
                                          have > 12 ? have - 12 : 0u};
                auto m = [](uint32_t w, uint32_t nb) { return nb >= 4 ? w : (nb ? w & ((1u << (8 * nb)) - 1) : 0u); };
                v = make_uint4(m(v.x, keep[0]), m(v.y, keep[1]), m(v.z, keep[2]), m(v.w, keep[3]));
            }
            D[q] = v;
        }
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
