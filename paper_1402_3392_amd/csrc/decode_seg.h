// Decoder that codes 64 / NL chunks per wave: with N = 32 interleaved coders
// per chunk, lanes 0-31 decode chunk c and lanes 32-63 chunk c + 1 (with
// N = 64, one chunk as before), so no lane idles.  Each chunk ("segment")
// keeps its own stream position and its own LDS ring of 256-byte windows,
// filled by direct global-to-LDS loads issued ahead of its read position;
// the segments step in lockstep, one rANS step (Section 2, Algorithm 1's
// decoder) per lane, and the refilling coders of a segment take consecutive
// digits in coder order from a ballot plus a prefix count (Section 6).
//
// Waits are exact: every vector-memory operation the wave issues (window and
// state loads, output stores) is numbered, each window remembers the number
// it was issued under, and entering a window waits until every operation up
// to the newest window the next steps may read has completed -- loads and
// stores complete in issue order, so that is "at most (issued - number)
// operations pending".
#pragma once

#include "coder64.h"

namespace rans {
namespace c64 {

constexpr uint32_t seg_count(int NL) { return 64 / NL; }

// LDS bytes per wave: the output block, then one ring of S windows plus the
// copy of slot 0 per segment.
constexpr uint32_t seg_wave_lds_bytes(int layout, int NL)
{
    return obuf_bytes(layout) + seg_count(NL) * (ring_slots(layout) + 1) * kWin;
}

// s & v for a wave-uniform s: one v_and_b32 reading the SGPR (the compiler
// otherwise turns a lane mask into a move plus a select).
__device__ __forceinline__ uint32_t and_sv(uint32_t s, uint32_t v)
{
    uint32_t r;
    asm("v_and_b32 %0, %1, %2" : "=v"(r) : "s"(uni(s)), "v"(v));
    return r;
}

// Waits until at most n (wave-uniform) vector-memory operations of this wave
// are pending; n above 31 waits as for 31 (longer, never too short).
// s_waitcnt takes its count as an immediate, so this jumps into a table of
// 32 waits (8 bytes each: the wait and a branch past the table) at
// pc + 16 + 8 n, pc being the address after s_getpc_b64 (the four
// instructions between it and the table are 4 bytes each).  The scratch
// SGPRs are named and clobbered.
__device__ __forceinline__ void wait_vm_atmost(uint32_t n)
{
    asm volatile(
        "s_min_u32 s30, %0, 31\n\t"
        "s_getpc_b64 s[28:29]\n\t"
        "s_lshl3_add_u32 s30, s30, 16\n\t"
        "s_add_u32 s28, s28, s30\n\t"
        "s_addc_u32 s29, s29, 0\n\t"
        "s_setpc_b64 s[28:29]\n\t"
        "s_waitcnt vmcnt(0)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(1)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(2)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(3)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(4)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(5)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(6)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(7)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(8)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(9)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(10)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(11)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(12)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(13)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(14)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(15)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(16)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(17)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(18)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(19)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(20)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(21)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(22)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(23)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(24)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(25)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(26)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(27)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(28)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(29)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(30)\n\ts_branch .Lwv%=\n\t"
        "s_waitcnt vmcnt(31)\n\ts_branch .Lwv%=\n\t"
        ".Lwv%=:"
        :
        : "s"(uni(n))
        : "memory", "scc", "s28", "s29", "s30");
}

// Decodes chunks chunk0 .. chunk0 + 64/NL - 1 (those below n_chunks) of the
// container `in`; arguments as decode_chunk's (every one wave-uniform).
// wave_lds: seg_wave_lds_bytes(LAYOUT, NL) bytes.  When it returns, every
// memory operation it issued has completed.
template <int R, int W, int SW, int LAYOUT, int NL, bool BF, bool ONE = false>
__device__ __forceinline__ void decode_seg(const uint8_t* in, uint64_t in_len, uint32_t n_chunks,
                                           uint64_t chunk0, uint32_t C, uint64_t n, void* out_base,
                                           uint32_t k_, uint32_t l, const void* l_sym_v,
                                           const uint32_t* l_ent, uint8_t* wave_lds, int32_t* status)
{
    constexpr uint32_t SEG = seg_count(NL);
    static_assert(SEG == 1 || SEG == 2, "one or two segments per wave");
    using SymT = typename std::conditional<SW == 1, uint8_t, uint16_t>::type;
    using OutT = typename std::conditional<W == 1, uint8_t, uint16_t>::type;
    constexpr uint32_t OW = sizeof(OutT);
    const SymT* l_sym = static_cast<const SymT*>(l_sym_v);
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t seg = SEG == 1 ? 0u : lane / NL, jl = lane % NL;
    constexpr uint32_t OB = obuf_bytes(LAYOUT), OBS = OB / SEG;  // output block, per segment
    constexpr uint32_t S = ring_slots(LAYOUT), TB = test_steps(LAYOUT);
    constexpr uint32_t DB = R / 8;                    // bytes per digit
    constexpr uint32_t MAXB = 2 * NL;                 // digit bytes a segment reads per step, at most
    constexpr uint32_t RES = 1 + (TB * MAXB + kWin - 1) / kWin;  // windows a test block may read
    constexpr uint32_t RING = (S + 1) * kWin;         // bytes per segment ring (with the copy)
    constexpr uint32_t DMASK = S * kWin / DB - 1;     // ring size in digits, minus 1
    constexpr uint32_t WD = kWin / DB;                // digits per window
    constexpr uint32_t SPB = OBS / (NL * OW);         // steps per output block
    constexpr uint32_t PIECE = OB / 64;               // bytes each lane moves per block
    using Piece = typename std::conditional<PIECE == 16, uint4, uint2>::type;
    static_assert(SPB % TB == 0 && RES < S && OBS == NL * PIECE, "segment geometry");

    uint8_t* obuf = wave_lds;
    const uint32_t lds_ob = lds_addr(obuf), lds_ring0 = lds_ob + OB, lane4 = 4 * lane;
    const uint32_t L = 1u << l, k = k_, mask = (1u << k) - 1;
    const uint64_t room = (in_len - 4) & ~3ull;  // last whole word (in_len >= 176 below)
    const uint64_t data0 = (kHeaderBytes + uint64_t(kDirEntryBytes) * n_chunks + 15) & ~15ull;

    // per segment (scalars): chunk geometry and stream state
    uint64_t pay[SEG];
    uint32_t nsym[SEG], nwin[SEG], wfast[SEG], ndig[SEG], pos[SEG], kw[SEG], wend[SEG];
    uint32_t exists = 0;  // bit s: segment s has a chunk that passed the checks
#pragma unroll
    for (uint32_t s = 0; s < SEG; ++s) {
        const uint64_t c = chunk0 + s;
        pay[s] = 0;
        nsym[s] = nwin[s] = wfast[s] = ndig[s] = pos[s] = kw[s] = 0;
        wend[s] = WD;
        if (c >= n_chunks)
            continue;
        const uint8_t* de = in + kHeaderBytes + kDirEntryBytes * c;
        const uint64_t off = uni64(*reinterpret_cast<const uint64_t*>(de));
        const uint32_t len = uni(*reinterpret_cast<const uint32_t*>(de + 8));
        if ((off & 15) || off < data0 || off > in_len || len > in_len - off || len < 4 * NL ||
            ((len - 4 * NL) % DB) != 0) {
            if (lane == 0)
                atomicMin(status, RANS_ECORRUPT);
            continue;
        }
        const uint64_t first = c * C;
        nsym[s] = uni(static_cast<uint32_t>(n - first < C ? n - first : C));
        const uint32_t plen = len - 4 * NL;
        pay[s] = off + 4 * NL;
        nwin[s] = (plen + kWin - 1) / kWin;
        ndig[s] = plen / DB;
        wfast[s] = uni(room + 4 >= pay[s] + kWin ? static_cast<uint32_t>((room + 4 - pay[s] - kWin) / kWin) + 1
                                                 : 0u);
        exists |= 1u << s;
    }
    if (exists == 0)
        return;

    // vector-memory operations issued so far, and the number each ring slot's
    // window was issued under (lane s * S + slot of wseq)
    uint32_t nops = 0, wseq = 0;
    auto fetch = [&](uint64_t src, uint32_t dst) {  // 256 container bytes from src
        uint32_t vo = lane4;
        if (src + kWin > room + 4) {
            if (src > room)
                src = room;
            vo = min(lane4, static_cast<uint32_t>(room - src));
        }
        dma256(in + src, vo, dst);
    };
    auto issue = [&](uint32_t s, uint32_t w) {
        const uint64_t src = pay[s] + uint64_t(w) * kWin;
        const uint32_t ring = lds_ring0 + s * RING;
        const uint32_t slot = w % S;
        if (slot == 0) {  // the copy goes first, so it lands no later than the window
            if (w < wfast[s])
                dma256(in + src, lane4, ring + S * kWin);
            else
                fetch(src, ring + S * kWin);
            ++nops;
        }
        if (w < wfast[s])
            dma256(in + src, lane4, ring + slot * kWin);
        else
            fetch(src, ring + slot * kWin);
        ++nops;
        wseq = lane == s * S + slot ? nops : wseq;
    };
    // windows up to w of segment s have landed
    auto need = [&](uint32_t s, uint32_t w) {
        const uint32_t q = uni(__builtin_amdgcn_readlane(wseq, s * S + w % S));
        wait_vm_atmost(nops - q);
    };

    // the coders' initial states: lane i of segment s reads word i - s NL of
    // its chunk's stream into obuf + 4 i (the load runs on that segment's
    // lanes only)
    uint32_t state_seq = 0;
#pragma unroll
    for (uint32_t s = 0; s < SEG; ++s) {
        if (!(exists >> s & 1))
            continue;
        if (seg == s)
            dma256(in + (pay[s] - 4 * NL) - 4 * NL * s, lane4, lds_ob);
        state_seq = ++nops;
    }
    // the first windows of every segment, interleaved so that the ones read
    // first are issued first
#pragma unroll
    for (uint32_t w = 0; w < S; ++w)
#pragma unroll
        for (uint32_t s = 0; s < SEG; ++s)
            if (w < nwin[s])
                issue(s, w);
    {
        uint32_t q = state_seq;
#pragma unroll
        for (uint32_t s = 0; s < SEG; ++s)
            if (nwin[s]) {
                const uint32_t w = (nwin[s] < RES ? nwin[s] : RES) - 1;
                const uint32_t qs = uni(__builtin_amdgcn_readlane(wseq, s * S + w));
                q = qs > q ? qs : q;
            }
        wait_vm_atmost(nops - q);
    }
    // with one segment, a wave only decodes when its chunk is present
    const bool live = SEG == 1 ? true : ((exists >> seg) & 1) != 0;
    const bool all_live = exists == (1u << SEG) - 1;
    uint32_t x = reinterpret_cast<const uint32_t*>(obuf)[lane];
    lane_fence();  // the output block is reused for symbols
    if (!live)
        x = L;  // coders of an absent chunk stay at L and never refill

    // per lane: where its symbols go in the output block and in memory
    OutT* ob = reinterpret_cast<OutT*>(obuf + seg * OBS) + jl;
    uint64_t first_lane = 0;
#pragma unroll
    for (uint32_t s = 0; s < SEG; ++s)
        if (seg == s)
            first_lane = (chunk0 + s) * C;
    uint8_t* out_lane = reinterpret_cast<uint8_t*>(static_cast<OutT*>(out_base) + first_lane) + PIECE * jl;
    const uint8_t* piece_lds = obuf + PIECE * lane;
    // lanes of the upper segment: all ones (the per-lane position offset)
    const uint32_t vhi = SEG == 2 && lane >= NL ? 0xFFFFFFFFu : 0u;
    constexpr uint32_t RBD = RING / DB;  // segment 1's ring, in digits after segment 0's

    auto decode_one = [&](uint32_t& s) {
        const uint32_t slot = x & mask;
        if (LAYOUT == kFused) {
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
    // ring-relative digit index of segment 0's read position, and the offset
    // that moves the upper segment's lanes to their own ring and position
    // (the prefix count over the whole wave also counts the lower segment's
    // reading lanes, which the offset takes back out)
    auto pos_off = [&](uint32_t lower) -> uint32_t {
        return SEG == 2 ? and_sv(RBD + (pos[SEG - 1] & DMASK) - (pos[0] & DMASK) - lower, vhi) : 0u;
    };
    auto refill = [&](bool act, auto dense) {
        const bool n1 = act && x < L;
        const uint64_t m1 = ballot(n1);
        const uint32_t lo1 = __popc(static_cast<uint32_t>(m1)), hi1 = __popc(static_cast<uint32_t>(m1 >> 32));
        if (R == 16) {
            if (dense || m1) {
                const uint16_t* rp = reinterpret_cast<const uint16_t*>(wave_lds + OB) + (pos[0] & DMASK);
                const uint32_t v = rp[mbcnt(m1, pos_off(lo1))];
                x = select_mask(m1, x, (x << 16) | v);
                if (SEG == 1) {
                    pos[0] += lo1 + hi1;
                } else {
                    pos[0] += lo1;
                    pos[SEG - 1] += hi1;
                }
            }
        } else if (ONE) {
            // a one-digit table: one byte per refilling lane
            if (dense || m1) {
                const uint8_t* r = wave_lds + OB + (pos[0] & DMASK);
                x = select_mask(m1, x, (x << 8) | r[mbcnt(m1, pos_off(lo1))]);
                if (SEG == 1) {
                    pos[0] += lo1 + hi1;
                } else {
                    pos[0] += lo1;
                    pos[SEG - 1] += hi1;
                }
            }
        } else {
            const bool n2 = act && x < (L >> 8);
            const uint64_t m2 = ballot(n2);
            const uint32_t lo2 = __popc(static_cast<uint32_t>(m2)), hi2 = __popc(static_cast<uint32_t>(m2 >> 32));
            if (dense || m1) {
                const uint8_t* r = wave_lds + OB + (pos[0] & DMASK);
                uint32_t x1, x2;
                if (BF) {
                    // first digits of a segment, then its second digits
                    const uint32_t o2 =
                        SEG == 2 ? and_sv(RBD + (pos[SEG - 1] & DMASK) + hi1 - (pos[0] & DMASK) - lo1 - lo2, vhi)
                                 : 0u;
                    x1 = (x << 8) | r[mbcnt(m1, pos_off(lo1))];
                    x2 = (x1 << 8) | (r + (SEG == 1 ? lo1 + hi1 : lo1))[mbcnt(m2, o2)];
                } else {
                    const uint8_t* q = r + (mbcnt(m1, pos_off(lo1 + lo2)) + mbcnt(m2, 0));
                    x1 = (x << 8) | q[0];
                    x2 = (x1 << 8) | q[1];
                }
                x = select_mask(m1, x, select_mask(m2, x1, x2));
                if (SEG == 1) {
                    pos[0] += lo1 + hi1 + lo2 + hi2;
                } else {
                    pos[0] += lo1 + lo2;
                    pos[SEG - 1] += hi1 + hi2;
                }
            }
        }
    };
    // A full step of every lane.  Lanes of an absent segment keep x = L
    // (so they never refill) and write their symbols into their segment's
    // part of the output block, which is never stored: no branch per step.
    auto step_full = [&](OutT* dst, auto dense, auto all) {
        uint32_t s = 0;
        const uint32_t x0 = x;
        decode_one(s);
        if (!all && !live)
            x = x0;
        refill(true, dense);
        *dst = static_cast<OutT>(s);
    };
    auto step1 = [&](OutT* dst, bool act) {  // tail step: only lanes with a symbol left
        uint32_t s = 0;
        if (act)
            decode_one(s);
        refill(act, std::false_type{});
        if (act)
            *dst = static_cast<OutT>(s);
    };
    auto flush = [&](uint32_t tb, auto all) {  // a whole output block of every segment
        lane_fence();
        const Piece v = *reinterpret_cast<const Piece*>(piece_lds);
        lane_fence();
        if (all || live)
            gstore(out_lane + uint64_t(tb) * NL * OW, v);
        ++nops;  // one store instruction (at least one segment is live)
    };
    // a test block of TB steps starting below wend reads at most TB MAXB
    // bytes per segment: windows kw .. kw + RES - 1 suffice
    auto advance = [&]() {
#pragma unroll
        for (uint32_t s = 0; s < SEG; ++s) {
            while (pos[s] >= wend[s]) {
                ++kw[s];
                wend[s] += WD;
                if (kw[s] + S - 1 < nwin[s])
                    issue(s, kw[s] + S - 1);
                const uint32_t w = kw[s] + RES - 1 < nwin[s] ? kw[s] + RES - 1 : nwin[s] - 1;
                if (kw[s] < nwin[s])
                    need(s, w);
            }
        }
    };

    uint32_t full = ~0u, steps = 0;
#pragma unroll
    for (uint32_t s = 0; s < SEG; ++s)
        if (exists >> s & 1) {
            full = min(full, nsym[s] / NL);
            steps = max(steps, (nsym[s] + NL - 1) / NL);
        }
    uint32_t t = 0;
    // whole output blocks with every present segment full: offsets are
    // immediates, one flush per block
    constexpr uint32_t NB = SPB / TB;
    auto blocks = [&](auto dense, auto all) {
        while (t + SPB <= full) {
#pragma unroll
            for (uint32_t b = 0; b < NB; ++b) {
                advance();
#pragma unroll
                for (uint32_t i = 0; i < TB; ++i)
                    step_full(ob + (b * TB + i) * NL, dense, all);
            }
            t += SPB;
            flush(t - SPB, all);
        }
    };
    uint64_t dig = 0, syms = 0;
#pragma unroll
    for (uint32_t s = 0; s < SEG; ++s) {
        dig += ndig[s];
        syms += nsym[s];
    }
    // dense: at least one refill per 16 coder steps, so a step without any
    // refill is rare and the refill runs unconditionally
    const bool dense = dig * 16 >= syms * (R == 8 ? 2 : 1);
    if (SEG == 1 || all_live) {
        if (dense)
            blocks(std::true_type{}, std::true_type{});
        else
            blocks(std::false_type{}, std::true_type{});
    } else {
        if (dense)
            blocks(std::true_type{}, std::false_type{});
        else
            blocks(std::false_type{}, std::false_type{});
    }

    // The rest, step by step: a segment may run out before the other (the
    // last chunk of a container is short).  A block whose pieces are not all
    // whole is written byte by byte after draining every pending operation.
    auto tail_flush = [&](uint32_t tb) {
        lane_fence();
        uint32_t mine = 0;  // valid bytes of this lane's piece
#pragma unroll
        for (uint32_t s = 0; s < SEG; ++s)
            if (seg == s) {
                const int64_t v = int64_t(nsym[s]) * OW - (int64_t(tb) * NL * OW + int64_t(PIECE) * jl);
                mine = v <= 0 ? 0u : (v >= PIECE ? PIECE : static_cast<uint32_t>(v));
            }
        if (!live)
            mine = 0;
        uint8_t* dst = out_lane + uint64_t(tb) * NL * OW;
        if (ballot(mine == PIECE)) {
            if (mine == PIECE)
                gstore(dst, *reinterpret_cast<const Piece*>(piece_lds));
            ++nops;
        }
        if (ballot(mine != 0 && mine != PIECE)) {
            wait_vm<0>();
            for (uint32_t b = 0; b < mine && mine != PIECE; ++b)
                dst[b] = piece_lds[b];
            wait_vm<0>();  // the byte stores are not counted: nothing stays pending
        }
        lane_fence();
    };
    while (t < steps) {
        advance();
        bool act = false;
#pragma unroll
        for (uint32_t s = 0; s < SEG; ++s)
            if (seg == s)
                act = live && t * NL + jl < nsym[s];
        step1(ob + (t % SPB) * NL, act);
        ++t;
        if (t % SPB == 0)
            tail_flush(t - SPB);
    }
    if (t % SPB != 0)
        tail_flush(t - t % SPB);
    wait_vm<0>();  // windows fetched ahead land before wave_lds is reused

    // end check of every present segment: all coders back at L, its stream
    // exactly consumed (Section 3: the decoder retraces the encoder's states)
    const uint64_t badx = ballot(live && x != L);
#pragma unroll
    for (uint32_t s = 0; s < SEG; ++s) {
        if (!(exists >> s & 1))
            continue;
        const uint64_t segbits = SEG == 1 ? ~0ull : (0xFFFFFFFFull << (32 * s));
        if (((badx & segbits) || pos[s] != ndig[s]) && lane == 0)
            atomicMin(status, RANS_ECORRUPT);
    }
}

}  // namespace c64
}  // namespace rans
