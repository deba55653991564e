// Encoder that codes two chunks of N = 32 interleaved coders per wave:
// lanes 0-31 encode chunk c and lanes 32-63 chunk c + 1, so no lane idles
// (the one-chunk encoder leaves half of each wave idle with N = 32).  Each
// chunk ("segment") is Algorithm 1's encoder with rANS's C per coder, walking
// its chunk backwards (Section 2), its digits written in decoder order at
// positions from one ballot prefix over the wave (Section 6); each segment
// keeps its own digit count, its own 2 KiB LDS digit ring and its own slot.
#pragma once

#include "decode_seg.h"

namespace rans {
namespace c64 {

// Per-wave LDS of the two-segment encoder: the one-chunk encoder's 4 KiB
// ring split into two 2 KiB digit rings (each at an LDS address that is a
// multiple of 2 KiB), and its symbol area (a 512-byte block per segment).
constexpr uint32_t kSegRing = 2048;
// Digits leave a ring in 512-byte windows (16 bytes per lane of the
// segment), aligned to multiples of 512 in the slot.  After a flush fewer
// than 512 bytes of a segment stay pending and a 512-byte symbol block adds
// at most 1 KiB, so a flush completes at most two windows per segment, and
// the ring holds the less than 1.5 KiB pending.
constexpr uint32_t kSegWindow = 512;
constexpr uint32_t kSegFlushStores = 2;
static_assert(2 * kSegRing == kEncRing && kSlotAlign % kSegWindow == 0 &&
                  kSegRing % kSegWindow == 0 && kSlotPad >= kSegWindow,
              "two-segment encoder geometry");

// One encoder step of both segments.  wpos: each segment's lowest digit
// written so far (it grows downwards); amask: the lanes that code a symbol on
// this step (wave-uniform; every lane when FULL); vhi: all ones in the upper
// segment's lanes; segbase: the LDS address of the lane's segment ring (a
// multiple of kSegRing: a digit's ring address is its position's bits or-ed
// in).  As enc_step, with the prefix count taken over the whole wave and
// the upper segment's lanes moved to their own position by a per-lane
// offset (the count also covers the lower segment's emitting lanes, which
// the offset takes back out).  Idle lanes keep their state through selects
// on amask: the ballots are masked with it, so no per-lane predicate is
// formed and no exec-mask branch splits the unrolled block.  ONE: as in
// enc_step (a one-digit table: no lane emits a second digit).
template <int R, bool BF, bool FULL, bool ONE = false>
__device__ __forceinline__ void enc_step_seg(uint32_t& x, uint32_t* wpos, uint32_t& bad, const uint4& e,
                                             uint64_t amask, uint32_t vhi, uint32_t segbase, uint32_t junkv)
{
    constexpr uint32_t RB = kSegRing;
    const uint64_t am = FULL ? ~0ull : amask;
    bad |= FULL ? e.w : select_mask(am, 0u, e.w);
    if (R == 16) {
        uint64_t m;
        uint32_t xs;
        if (FULL) {
            m = gt_shift16(x, e.y, &xs);
        } else {
            m = ballot(x > e.y) & am;
            xs = select_mask(m, x, x >> 16);
        }
        const uint32_t lo = __popc(static_cast<uint32_t>(m)), hi = __popc(static_cast<uint32_t>(m >> 32));
        wpos[0] -= lo;
        wpos[1] -= hi;
        const uint32_t pos = mbcnt(m, and_sv(wpos[1] - wpos[0] - lo, vhi)) + wpos[0];
        ring_store<2>(m, ((pos << 1) & (RB - 1)) | segbase, junkv, x);
        x = xs;
    } else if (ONE) {
        const bool e1 = x > e.y;
        const uint64_t m1 = FULL ? ballot(e1) : ballot(e1) & am;
        const uint32_t lo = __popc(static_cast<uint32_t>(m1)), hi = __popc(static_cast<uint32_t>(m1 >> 32));
        wpos[0] -= lo;
        wpos[1] -= hi;
        const uint32_t i1 = mbcnt(m1, and_sv(wpos[1] - wpos[0] - lo, vhi)) + wpos[0];
        ring_store<1>(m1, (i1 & (RB - 1)) | segbase, junkv, x);
        x = FULL ? (e1 ? x >> 8 : x) : select_mask(m1, x, x >> 8);
    } else {
        // a lane that emits two digits also emits one: m2 is within m1
        const bool e1 = x > e.y, e2 = (x >> 8) > e.y;
        const uint64_t m1 = FULL ? ballot(e1) : ballot(e1) & am, m2 = FULL ? ballot(e2) : ballot(e2) & am;
        const uint32_t lo1 = __popc(static_cast<uint32_t>(m1)), hi1 = __popc(static_cast<uint32_t>(m1 >> 32));
        const uint32_t lo2 = __popc(static_cast<uint32_t>(m2)), hi2 = __popc(static_cast<uint32_t>(m2 >> 32));
        wpos[0] -= lo1 + lo2;
        wpos[1] -= hi1 + hi2;
        uint32_t i1, i2;
        if (BF) {
            // first digits of a segment, then its second digits
            i1 = mbcnt(m1, and_sv(wpos[1] - wpos[0] - lo1, vhi)) + wpos[0];
            i2 = mbcnt(m2, and_sv((wpos[1] + hi1) - (wpos[0] + lo1) - lo2, vhi)) + (wpos[0] + lo1);
        } else {
            i1 = mbcnt(m1, mbcnt(m2, and_sv(wpos[1] - wpos[0] - lo1 - lo2, vhi))) + wpos[0];
            i2 = i1 + 1;
        }
        const uint32_t d1 = FULL ? (e2 ? x >> 8 : x) : select_mask(m2, x, x >> 8);
        ring_store<1>(m1, (i1 & (RB - 1)) | segbase, junkv, d1);
        ring_store<1>(m2, (i2 & (RB - 1)) | segbase, junkv, x);
        x = FULL ? (e2 ? x >> 16 : (e1 ? x >> 8 : x)) : select_mask(m2, select_mask(m1, x, x >> 8), x >> 16);
    }
    const uint32_t q = __umulhi(e.x, x + (e.w >> 24)) >> ((e.z >> 16) & 31u);
    // computed on every lane and selected: C's result through a branch on a
    // per-lane condition would split the block
    const uint32_t xn = c_update(x, q, e.z, e.w);
    x = FULL ? xn : select_mask(am, x, xn);
}

// Encodes chunks chunk0 and chunk0 + 1 (the second only when it is below
// n_chunks) of syms_base (n symbols of W bytes, C per chunk) with 32 coders
// each; chunk chunk0 + s goes to the digit slot slots[s] (digits end at
// slot + slot_bytes, a multiple of 512; kSlotPad more bytes follow).  On
// return every lane holds its coder's final state in *x (lanes 0-31 chunk
// chunk0's coders, 32-63 the next chunk's) and nd[s] is segment s's digit
// count; slot1 is not touched when there is no second chunk.  l_enc: staged
// encoder entries as for encode_chunk (alphabet + 1
// entries; 256 with 8-bit symbols); ring, sbuf: this wave's digit ring and
// symbol block, as for encode_chunk.  Arguments wave-uniform.  ONE: as in
// enc_step_seg.
template <int R, int W, bool BF, bool ONE = false>
__device__ __forceinline__ void encode_seg(const void* syms_base, uint64_t n, uint32_t C, uint64_t chunk0,
                                           uint32_t n_chunks, uint32_t l, uint32_t alphabet,
                                           const uint4* l_enc, uint8_t* slot0,
                                           uint8_t* slot1, uint64_t slot_bytes, uint8_t* ring, uint8_t* sbuf,
                                           int32_t* status, uint32_t* x_out, uint32_t* nd)
{
    constexpr uint32_t NL = 32;
    using InT = typename std::conditional<W == 1, uint8_t, uint16_t>::type;
    constexpr uint32_t SPB = 512 / (W * NL);  // steps per block: 512 symbol bytes per segment
    constexpr uint32_t DB = R / 8, WD = kSegWindow / DB;
    const uint32_t lane = threadIdx.x & 63, seg = lane >> 5, jl = lane & 31;
    const uint32_t vhi = seg ? 0xFFFFFFFFu : 0u, segoff = seg * kSegRing;
    const uint8_t* dring = ring;
    const uint32_t segbase = lds_addr(ring) + segoff;
    const uint32_t junkv = lds_addr(sbuf) + kEncSymBlock + 2 * lane;
    const bool has1 = chunk0 + 1 < n_chunks;
    uint32_t nsym[2], steps[2], nblk[2];
    const InT* in[2];
#pragma unroll
    for (uint32_t s = 0; s < 2; ++s) {
        const uint64_t first = (chunk0 + s) * C;
        const bool ok = s == 0 || has1;
        nsym[s] = ok ? uni(static_cast<uint32_t>(n - first < C ? n - first : C)) : 0u;
        steps[s] = (nsym[s] + NL - 1) / NL;
        nblk[s] = nsym[s] / (NL * SPB);
        in[s] = static_cast<const InT*>(syms_base) + (ok ? first : chunk0 * C);
    }
    const uint32_t top = uni(static_cast<uint32_t>(slot_bytes / DB));
    uint32_t x = 1u << l;
    uint32_t wpos[2] = {top, top};  // lowest digit written so far, per segment
    uint32_t wtop[2] = {top, top};  // digits from wtop up are in the slot
    uint32_t bad = 0;
    // per lane: its segment's slot and symbols.  Without a second chunk the
    // upper lanes only ever store padding: into the first chunk's slot
    // padding (slot1 may lie past the caller's slots then).
    uint8_t* myslot = seg && has1 ? slot1 : slot0;
    const InT* myin = seg ? in[1] : in[0];
    const uint32_t mynsym = seg ? nsym[1] : nsym[0];

    // this lane's 16 bytes of its segment's ring window of digits [lo, lo + WD)
    auto ring_word = [&](uint32_t lo) {
        return *reinterpret_cast<const uint4*>(dring + segoff + ((lo * DB) & (kSegRing - 1)) + 16 * jl);
    };
    auto flush = [&]() {
        uint32_t wc[2], cnt[2];
#pragma unroll
        for (uint32_t s = 0; s < 2; ++s) {
            wc[s] = (wpos[s] + WD - 1) / WD * WD;  // lowest window boundary at or above wpos
            cnt[s] = (wtop[s] - wc[s]) / WD;        // complete windows not yet stored (<= 2)
        }
        const uint32_t mytop = seg ? wtop[1] : wtop[0], mycnt = seg ? cnt[1] : cnt[0];
        lane_fence();
#pragma unroll
        for (uint32_t j = 0; j < kSegFlushStores; ++j) {
            const uint32_t lo = mytop - (j + 1) * WD;
            uint8_t* dst = j < mycnt ? myslot + uint64_t(lo) * DB : myslot + slot_bytes;
            const uint4 v = ring_word(lo);
            gstore(reinterpret_cast<uint4*>(dst) + jl, v);
        }
        lane_fence();
        wtop[0] = wc[0];
        wtop[1] = wc[1];
    };

    // blocks b = steps [b SPB, (b + 1) SPB), from the top down; a block is
    // whole for a segment below its nblk, empty at or above its steps; the
    // (at most two) blocks that are neither run step by step
    const uint32_t T = steps[0] > steps[1] ? steps[0] : steps[1];
    const uint32_t nb = (T + SPB - 1) / SPB;
    const bool any_full = nblk[0] + nblk[1] > 0;
    // a lane's 16-byte piece of block b of its segment, clamped into a
    // segment with whole blocks (the values of a block not whole are unused)
    const uint32_t mynblk = seg ? nblk[1] : nblk[0];
    const uint4* myblk = reinterpret_cast<const uint4*>(mynblk ? myin : (nblk[0] ? in[0] : in[1])) + jl;
    const uint32_t clampb = (mynblk ? mynblk : (nblk[0] ? nblk[0] : nblk[1])) - 1;
    auto load_blk = [&](int64_t b) {
        uint32_t bb = b < 0 ? 0u : static_cast<uint32_t>(b);
        bb = bb > clampb ? clampb : bb;
        const v4u v = __builtin_nontemporal_load(gmem(reinterpret_cast<const v4u*>(myblk + bb * 32)));
        return make_uint4(v.x, v.y, v.z, v.w);
    };
    const InT* sb = reinterpret_cast<const InT*>(sbuf + 512 * seg) + jl;
    constexpr int PF = 3;
    // a block's symbols go to LDS once every read of the previous block's
    // has been issued (the reads come first in each block)
    auto stage_blk = [&](const uint4& v) {
        lane_fence();
        *reinterpret_cast<uint4*>(sbuf + 16 * lane) = v;
        lane_fence();
    };
    auto run_blk = [&](uint64_t amask, auto full) {
        uint32_t sy[SPB];
#pragma unroll
        for (int q = 0; q < int(SPB); ++q) {
            const uint32_t v0 = static_cast<uint32_t>(sb[q * NL]);
            sy[q] = W == 1 ? v0 : min(v0, alphabet);  // 8-bit symbols index 256 staged entries
        }
        lane_fence();  // the symbols are in registers before the ring writes
        auto entry = [&](int q) { return l_enc[sy[q]]; };
        uint4 ent[SPB];
#pragma unroll
        for (int q = int(SPB) - 1; q >= int(SPB) - PF && q >= 0; --q)
            ent[q] = entry(q);
#pragma unroll
        for (int q = int(SPB) - 1; q >= 0; --q) {
            if (q - PF >= 0)
                ent[q - PF] = entry(q - PF);
            enc_step_seg<R, BF, decltype(full)::value, ONE>(x, wpos, bad, ent[q], amask, vhi, segbase, junkv);
        }
    };
    int64_t b = int64_t(nb) - 1;
    if (any_full)
        stage_blk(load_blk(b));
    for (; b >= 0; --b) {
        const uint32_t ub = static_cast<uint32_t>(b);
        // the next block's symbols load while this one is coded; held in
        // registers defined and consumed within the iteration, so no copy
        // at the back edge has to wait for them
        uint4 nv = make_uint4(0, 0, 0, 0);
        if (any_full && b > 0)
            nv = load_blk(b - 1);
        const bool clean0 = ub < nblk[0] || ub * SPB >= steps[0];
        const bool clean1 = ub < nblk[1] || ub * SPB >= steps[1];
        if (clean0 && clean1) {
            // each segment's lanes take part when the block is whole for it
            const uint64_t amask = (ub < nblk[0] ? 0xFFFFFFFFull : 0ull) | (ub < nblk[1] ? ~0xFFFFFFFFull : 0ull);
            if (amask == ~0ull)
                run_blk(amask, std::true_type());
            else
                run_blk(amask, std::false_type());
        } else {
            for (uint32_t t = (ub + 1) * SPB; t-- > ub * SPB;) {
                const uint32_t i = t * NL + jl;
                const bool act = i < mynsym;
                const uint32_t s = act ? static_cast<uint32_t>(gmem(myin)[i]) : 0u;
                enc_step_seg<R, BF, false, ONE>(x, wpos, bad, l_enc[W == 1 ? s : min(s, alphabet)], ballot(act),
                                                vhi, segbase, junkv);
            }
        }
        flush();
        if (any_full && b > 0)
            stage_blk(nv);
    }
    // the window holding each stream's first digits
    {
        const uint32_t mypos = seg ? wpos[1] : wpos[0], mytop = seg ? wtop[1] : wtop[0];
        lane_fence();
        const uint4 v = ring_word(mytop - WD);
        if (mypos < mytop)
            gstore(reinterpret_cast<uint4*>(myslot + uint64_t(mytop - WD) * DB) + jl, v);
    }
    *x_out = x;
    nd[0] = top - wpos[0];
    nd[1] = top - wpos[1];
    if (ballot((bad >> 23) & 1) && lane == 0)
        atomicMin(status, RANS_ENOSYM);
}

}  // namespace c64
}  // namespace rans
