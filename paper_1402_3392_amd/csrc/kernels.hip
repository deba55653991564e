// librans HIP kernels for gfx950 (wave64).
//
// One coder state per lane.  A chunk of the container is one interleaved
// stream of N coders (Sections 3-4 of the paper): symbol i of the chunk
// belongs to coder i mod N, which is lane (i mod N) of a wave segment of N
// lanes; a wave holds 64/N segments, i.e. 64/N chunks.  Within a step the N
// lanes decode (or encode) one symbol each; the lanes that must read (write)
// a digit find their stream offset from a ballot of "I do I/O" and a prefix
// count of the lanes below them (Section 6), and the segment's stream
// position advances by the ballot's population count.
#include <hip/hip_runtime.h>

#include "rans_internal.h"

namespace rans {
namespace {

constexpr int kMaxThreads = 1024;

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ uint32_t popc(uint64_t m) { return __popcll(m); }

// Number of set bits of m in lanes below this one.
__device__ __forceinline__ uint32_t prefix(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}

__device__ __forceinline__ uint64_t align16(uint64_t v) { return (v + 15) & ~uint64_t(15); }

__device__ __forceinline__ uint32_t ld_u32(const uint8_t* p)
{
    return *reinterpret_cast<const uint32_t*>(p);
}

// Copies `bytes` (a multiple of 16) from global memory into LDS.
__device__ __forceinline__ void stage(uint8_t* lds, const void* src, uint32_t bytes)
{
    const uint4* s = static_cast<const uint4*>(src);
    uint4* d = reinterpret_cast<uint4*>(lds);
    for (uint32_t i = threadIdx.x; i < bytes / 16; i += blockDim.x)
        d[i] = s[i];
}

// Lane geometry of one wave: segment of N lanes = one chunk.
struct Lanes {
    uint32_t lane, j;   // wave lane, coder index within the segment
    uint64_t segmask;   // lanes of my segment
    uint64_t below;     // lanes of my segment below me
    uint64_t chunk;     // chunk handled by my segment
};

template <bool FULL>
__device__ __forceinline__ Lanes lane_geometry(uint32_t log2N)
{
    Lanes g;
    g.lane = threadIdx.x & 63;
    const uint32_t wave = threadIdx.x >> 6, wpb = blockDim.x >> 6;
    const uint32_t lg = FULL ? 6 : log2N;
    const uint32_t seg = FULL ? 0 : g.lane >> lg;
    g.j = FULL ? g.lane : (g.lane & ((1u << lg) - 1));
    g.segmask = FULL || lg == 6 ? ~0ull : (((1ull << (1u << lg)) - 1) << (seg << lg));
    g.below = g.segmask & ((1ull << g.lane) - 1);
    g.chunk = (static_cast<uint64_t>(blockIdx.x) * wpb + wave) * (64u >> lg) + seg;
    return g;
}

// ---------------------------------------------------------------- decode --
//
// Per step and lane (Algorithm 1, Decode, with rANS's D):
//   slot = x mod M;  s = symbol of slot;  x = f_s * floor(x/M) + slot - cum_s
//   then while x < L: x = b*x + next digit.
// With b = 2^16 >= M at most one digit is read (Section 5); with b = 2^8 and
// L = 2^l, l >= 16, at most two, and the count is known before reading:
// d = [x < L] + [x < L/256] since L is a multiple of 256.  Depth-first
// order (Section 5) lays the digits of one step out coder by coder, each
// coder's more significant digit first, so coder j's digits sit at
//   pos + #{lanes below j with d >= 1} + #{lanes below j with d >= 2} (+1);
// breadth-first order puts every coder's first digit before any second one:
//   pos + #{lanes below j with d >= 1}  and
//   pos + #{lanes with d >= 1} + #{lanes below j with d >= 2}.
// Escape coding (a.esc; 16-bit symbols, depth-first): a lane that decodes the
// escape E = alphabet - 1 then reads 16/R raw digits right after its own
// renormalisation digits; they hold its output value.

template <int R, int W, int SW, int LAYOUT, bool FULL>
__global__ void __launch_bounds__(kMaxThreads) k_decode(const DecodeArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    stage(lds, a.tab0, a.tab0_bytes);
    stage(lds + a.tab0_bytes, a.tab1, a.tab1_bytes);
    __syncthreads();

    using SymT = typename std::conditional<SW == 1, uint8_t, uint16_t>::type;
    using OutT = typename std::conditional<W == 1, uint8_t, uint16_t>::type;
    const uint32_t* l_dec = reinterpret_cast<const uint32_t*>(lds);
    const SymT* l_sym = reinterpret_cast<const SymT*>(lds + (LAYOUT == kPacked ? a.tab0_bytes : 0));
    const uint32_t* l_fc = reinterpret_cast<const uint32_t*>(lds + a.tab0_bytes);

    const Lanes g = lane_geometry<FULL>(a.log2N);
    const uint32_t N = FULL ? 64u : (1u << a.log2N);
    const uint32_t L = 1u << a.l, k = a.k, mask = (1u << k) - 1;

    bool ok = g.chunk < a.n_chunks;
    uint64_t off = 0;
    uint32_t len = 0, nsym = 0;
    if (ok) {
        const uint8_t* de = a.in + kHeaderBytes + kDirEntryBytes * g.chunk;
        off = *reinterpret_cast<const uint64_t*>(de);
        len = ld_u32(de + 8);
        const uint64_t first = g.chunk * a.C;
        nsym = static_cast<uint32_t>(a.n - first < a.C ? a.n - first : a.C);
        const uint64_t data0 = align16(kHeaderBytes + uint64_t(kDirEntryBytes) * a.n_chunks);
        const bool bad = (off & 15) || off < data0 || off > a.in_len || len > a.in_len - off ||
                         len < 4 * N || ((len - 4 * N) % (R / 8)) != 0;
        if (bad) {
            if (g.j == 0)
                atomicMin(a.status, RANS_ECORRUPT);
            ok = false;
            nsym = 0;
        }
    }
    const uint8_t* dig = a.in + off + 4 * N;
    const uint32_t ndig = ok ? (len - 4 * N) / (R / 8) : 0;
    uint32_t x = ok ? ld_u32(a.in + off + 4 * g.j) : L;
    uint32_t pos = 0;
    bool bad = false;
    OutT* out = static_cast<OutT*>(a.out) + g.chunk * a.C;

    for (uint32_t t = 0;; ++t) {
        const uint64_t i = uint64_t(t) * N + g.j;
        const bool act = i < nsym;
        if (!ballot(act))
            break;
        uint32_t s = 0;
        if (act) {
            const uint32_t slot = x & mask;
            if (LAYOUT == kFused) {
                const uint2 e = reinterpret_cast<const uint2*>(lds)[slot];
                s = e.y >> 24;
                x = __umul24(e.y, x >> k) + e.x;
            } else if (LAYOUT == kPacked) {
                const uint32_t e = l_dec[slot];
                s = l_sym[slot];
                x = __umul24(e >> 16, x >> k) + (e & 0xFFFFu);
            } else {
                s = l_sym[slot];
                const uint32_t fc = l_fc[s];
                x = __umul24(fc & 0xFFFFu, x >> k) + slot - (fc >> 16);
            }
        }
        const bool n1 = act && x < L;
        const bool n2 = R == 8 && act && x < (L >> 8);
        const bool ne = act && a.esc && s == a.alphabet - 1;
        const uint64_t m1 = ballot(n1);
        const uint64_t m2 = R == 8 ? ballot(n2) : 0ull;
        const uint64_t me = ballot(ne);
        const uint32_t b1 = FULL ? prefix(m1) : popc(m1 & g.below);
        const uint32_t b2 = FULL ? prefix(m2) : popc(m2 & g.below);
        const uint32_t be = FULL ? prefix(me) : popc(me & g.below);
        const uint32_t t1 = FULL ? popc(m1) : popc(m1 & g.segmask);
        const uint32_t t2 = FULL ? popc(m2) : popc(m2 & g.segmask);
        const uint32_t te = FULL ? popc(me) : popc(me & g.segmask);
        constexpr uint32_t RW = 16 / R;  // raw digits of an escaped value
        const uint32_t o = a.bf ? b1 : b1 + b2 + RW * be;
        if (n1) {
            uint32_t idx = pos + o;
            uint32_t d = 0;
            if (idx < ndig)
                d = R == 16 ? reinterpret_cast<const uint16_t*>(dig)[idx] : dig[idx];
            else
                bad = true;
            x = (x << R) | d;
            if (R == 8 && n2) {
                idx = a.bf ? pos + t1 + b2 : idx + 1;
                d = 0;
                if (idx < ndig)
                    d = dig[idx];
                else
                    bad = true;
                x = (x << 8) | d;
            }
        }
        if (ne) {
            uint32_t idx = pos + o + (n1 ? 1u : 0u) + (n2 ? 1u : 0u), v = 0;
            for (uint32_t q = 0; q < RW; ++q, ++idx) {
                uint32_t d = 0;
                if (idx < ndig)
                    d = R == 16 ? reinterpret_cast<const uint16_t*>(dig)[idx] : dig[idx];
                else
                    bad = true;
                v = (v << R) | d;
            }
            s = v;
        }
        pos += t1 + t2 + RW * te;
        if (act)
            out[i] = static_cast<OutT>(s);
    }
    // The decoder retraces the encoder's states backwards, so every coder
    // must be back at the start state L with the stream exactly consumed.
    if (ok && (x != L || pos != ndig))
        bad = true;
    const uint64_t badm = ballot(bad);
    if (badm && g.lane == static_cast<uint32_t>(__builtin_ctzll(badm)))
        atomicMin(a.status, RANS_ECORRUPT);
}

// ---------------------------------------------------------------- encode --
//
// Per step, walking the chunk backwards (Section 2), lane j with symbol s
// (Algorithm 1, Encode, with rANS's C):
//   while C(s,x) >= bL: emit x mod b; x = floor(x/b)
//   x = C(s,x) = M*floor(x/f) + (x mod f) + cum = x + q*(M - f) + cum, q = floor(x/f)
// C(s,x) >= bL  <=>  x >= f * 2^(l+r-k)  <=>  (x >> (l+r-k)) >= f.
// The digits of the step are prepended as one block laid out like the
// decoder reads it: coders ascending, each coder's high digit first, in
// depth-first or breadth-first order (as the decoder above describes).
// Escape coding (a.esc): a value the table lacks (v >= E = alphabet - 1 or
// f_v = 0) is coded as E, and the lane also emits 16/R raw digits holding
// v, after its renormalisation digits in decoder order.

template <int R, int W, bool FULL>
__global__ void __launch_bounds__(kMaxThreads) k_encode(const EncodeArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    stage(lds, a.enc, a.enc_bytes);
    __syncthreads();
    const uint4* l_enc = reinterpret_cast<const uint4*>(lds);

    using InT = typename std::conditional<W == 1, uint8_t, uint16_t>::type;
    const Lanes g = lane_geometry<FULL>(a.log2N);
    const uint32_t N = FULL ? 64u : (1u << a.log2N);
    const uint32_t L = 1u << a.l, sh = a.l + R - a.k;

    const bool ok = g.chunk < a.n_chunks;
    uint32_t nsym = 0;
    if (ok) {
        const uint64_t first = g.chunk * a.C;
        nsym = static_cast<uint32_t>(a.n - first < a.C ? a.n - first : a.C);
    }
    const uint32_t cap = static_cast<uint32_t>(a.slot_bytes / (R / 8));  // digits per slot
    uint8_t* slot = a.slots + (ok ? g.chunk : 0) * a.slot_stride;
    const InT* in = static_cast<const InT*>(a.syms) + (ok ? g.chunk * a.C : 0);

    uint32_t steps = (nsym + N - 1) / N;
    if (!FULL) {
        for (int d = 32; d >= 1; d >>= 1)
            steps = max(steps, static_cast<uint32_t>(__shfl_xor(static_cast<int>(steps), d)));
    }
    uint32_t x = L, wpos = cap;
    bool nosym = false, overflow = false;

    for (uint32_t t = steps; t-- > 0;) {
        const uint64_t i = uint64_t(t) * N + g.j;
        bool act = i < nsym;
        const uint32_t v = act ? static_cast<uint32_t>(in[i]) : 0u;
        uint32_t s = min(v, a.alphabet);  // entry `alphabet` has f = 0
        uint4 e = l_enc[s];
        const bool esc = act && a.esc && (v >= a.alphabet - 1 || (e.y & 0xFFFFu) == 0);
        if (esc)
            e = l_enc[a.alphabet - 1];
        const uint32_t f = e.y & 0xFFFFu, cum = e.y >> 16;
        if (act && f == 0) {
            nosym = true;
            act = false;
        }
        const bool e1 = act && (x >> sh) >= f;
        const bool e2 = R == 8 && act && (x >> (sh + 8)) >= f;
        const uint64_t m1 = ballot(e1);
        const uint64_t m2 = R == 8 ? ballot(e2) : 0ull;
        const bool emit_raw = esc && act;
        const uint64_t me = ballot(emit_raw);
        const uint32_t b1 = FULL ? prefix(m1) : popc(m1 & g.below);
        const uint32_t b2 = FULL ? prefix(m2) : popc(m2 & g.below);
        const uint32_t be = FULL ? prefix(me) : popc(me & g.below);
        const uint32_t t1 = FULL ? popc(m1) : popc(m1 & g.segmask);
        const uint32_t t2 = FULL ? popc(m2) : popc(m2 & g.segmask);
        const uint32_t te = FULL ? popc(me) : popc(me & g.segmask);
        constexpr uint32_t RW = 16 / R;  // raw digits of an escaped value
        wpos -= t1 + t2 + RW * te;
        if (emit_raw) {
            uint32_t idx = wpos + b1 + b2 + RW * be + (e1 ? 1u : 0u) + (e2 ? 1u : 0u);
            for (uint32_t q = 0; q < RW; ++q, ++idx) {
                const uint32_t d = (v >> (R * (RW - 1 - q))) & ((1u << R) - 1);
                if (idx < cap) {
                    if (R == 16)
                        reinterpret_cast<uint16_t*>(slot)[idx] = static_cast<uint16_t>(d);
                    else
                        slot[idx] = static_cast<uint8_t>(d);
                } else {
                    overflow = true;
                }
            }
        }
        if (e1) {
            const uint32_t idx = wpos + (a.bf ? b1 : b1 + b2 + RW * be);
            if (R == 16) {
                if (idx < cap)
                    reinterpret_cast<uint16_t*>(slot)[idx] = static_cast<uint16_t>(x);
                else
                    overflow = true;
                x >>= 16;
            } else if (e2) {
                const uint32_t idx2 = a.bf ? wpos + t1 + b2 : idx + 1;
                if (idx < cap && idx2 < cap) {
                    slot[idx] = static_cast<uint8_t>(x >> 8);
                    slot[idx2] = static_cast<uint8_t>(x);
                } else {
                    overflow = true;
                }
                x >>= 16;
            } else {
                if (idx < cap)
                    slot[idx] = static_cast<uint8_t>(x);
                else
                    overflow = true;
                x >>= 8;
            }
        }
        if (act) {
            const uint32_t q = __umulhi(e.x, x + (e.z & 0xFFu)) >> (e.z >> 8);
            x = x + __umul24(q, e.w) + cum;
        }
    }
    if (ok) {
        a.states[g.chunk * N + g.j] = x;
        if (g.j == 0)
            a.ndig[g.chunk] = cap - wpos;
    }
    const uint64_t nm = ballot(nosym), om = ballot(overflow);
    if ((nm | om) && g.lane == static_cast<uint32_t>(__builtin_ctzll(nm | om)))
        atomicMin(a.status, nm ? RANS_ENOSYM : RANS_EINVAL);
}

// Exclusive scan of the 16-byte aligned chunk lengths into directory
// offsets; writes the header and directory when the container fits.
__global__ void __launch_bounds__(kMaxThreads) k_scan(const ScanArgs a)
{
    __shared__ uint64_t part[kMaxThreads];
    const uint32_t T = blockDim.x, tid = threadIdx.x;
    const uint32_t per = (a.n_chunks + T - 1) / T;
    const uint32_t lo = min(a.n_chunks, tid * per), hi = min(a.n_chunks, lo + per);
    uint64_t sum = 0;
    for (uint32_t c = lo; c < hi; ++c)
        sum += align16(4ull * a.N + uint64_t(a.ndig[c]) * a.digit_bytes);
    part[tid] = sum;
    __syncthreads();
    for (uint32_t o = 1; o < T; o <<= 1) {
        const uint64_t v = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    const uint64_t base = align16(kHeaderBytes + uint64_t(kDirEntryBytes) * a.n_chunks);
    const uint64_t total = a.n_chunks ? base + part[T - 1] : kHeaderBytes;
    const bool fits = total <= a.out_cap;
    uint64_t off = base + (tid ? part[tid - 1] : 0);
    for (uint32_t c = lo; c < hi; ++c) {
        const uint32_t len = 4 * a.N + a.ndig[c] * a.digit_bytes;
        a.chunk_off[c] = off;
        if (fits) {
            uint8_t* de = a.out + kHeaderBytes + uint64_t(kDirEntryBytes) * c;
            *reinterpret_cast<uint64_t*>(de) = off;
            reinterpret_cast<uint32_t*>(de)[2] = len;
            reinterpret_cast<uint32_t*>(de)[3] = 0;
        }
        off += align16(len);
    }
    if (tid == 0) {
        *a.total = total;
        if (a.total_out)
            *a.total_out = total;
        if (fits) {
            uint32_t* h = reinterpret_cast<uint32_t*>(a.out);
            for (int q = 0; q < 8; ++q)
                h[q] = reinterpret_cast<const uint32_t*>(a.hdr)[q];
        } else {
            atomicMin(a.status, RANS_ENOSPC);
        }
    }
}

// Moves each chunk (states + digits from the end of its slot) to its
// directory offset, zero-filling up to the next 16-byte boundary.
__global__ void __launch_bounds__(256) k_compact(const CompactArgs a)
{
    if (*a.total > a.out_cap)
        return;
    for (uint32_t c = blockIdx.x; c < a.n_chunks; c += gridDim.x) {
        const uint64_t off = a.chunk_off[c];
        const uint32_t pay = a.ndig[c] * a.digit_bytes;
        const uint32_t words = static_cast<uint32_t>(align16(4ull * a.N + pay) / 4);
        const uint8_t* slot_end = a.slots + uint64_t(c) * a.slot_stride + a.slot_bytes;
        const uint8_t* src = slot_end - pay;
        uint32_t* dst = reinterpret_cast<uint32_t*>(a.out + off);
        for (uint32_t q = threadIdx.x; q < words; q += blockDim.x) {
            uint32_t v = 0;
            if (q < a.N) {
                v = a.states[uint64_t(c) * a.N + q];
            } else {
                const uint32_t p = (q - a.N) * 4;
                if (p < pay) {
                    const uintptr_t ad = reinterpret_cast<uintptr_t>(src + p);
                    const uintptr_t al = ad & ~uintptr_t(3);
                    const uint32_t lo = *reinterpret_cast<const uint32_t*>(al);
                    const uint32_t hi = al + 4 < reinterpret_cast<uintptr_t>(slot_end)
                                            ? *reinterpret_cast<const uint32_t*>(al + 4)
                                            : 0u;
                    v = static_cast<uint32_t>(((uint64_t(hi) << 32) | lo) >> ((ad & 3) * 8));
                    const uint32_t rem = pay - p;
                    if (rem < 4)
                        v &= (1u << (8 * rem)) - 1;
                }
            }
            dst[q] = v;
        }
    }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t value, uint32_t count)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        p[i] = value;
}

template <typename K>
hipError_t set_lds(K kernel, uint32_t bytes)
{
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
}

// Waves per block: enough blocks to cover the chunks, up to 16 waves each.
uint32_t waves_for(uint64_t n_chunks, uint32_t segs)
{
    const uint64_t waves = (n_chunks + segs - 1) / segs;
    return static_cast<uint32_t>(waves < 16 ? (waves ? waves : 1) : 16);
}

template <int R, int W, int SW, int LAYOUT, bool FULL>
hipError_t run_decode(const DecodeArgs& a, hipStream_t st)
{
    const uint32_t segs = 64u >> a.log2N;
    const uint32_t wpb = waves_for(a.n_chunks, segs);
    const uint64_t chunks_per_block = uint64_t(wpb) * segs;
    const uint32_t blocks = static_cast<uint32_t>((a.n_chunks + chunks_per_block - 1) / chunks_per_block);
    const uint32_t lds = a.tab0_bytes + a.tab1_bytes;
    auto kern = k_decode<R, W, SW, LAYOUT, FULL>;
    hipError_t e = set_lds(kern, lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * wpb), lds, st, a);
    return hipGetLastError();
}

template <int R, int W, int SW, int LAYOUT>
hipError_t run_decode_n(const DecodeArgs& a, hipStream_t st)
{
    return a.log2N == 6 ? run_decode<R, W, SW, LAYOUT, true>(a, st)
                        : run_decode<R, W, SW, LAYOUT, false>(a, st);
}

template <int R, int W, int SW>
hipError_t run_decode_l(const DecodeArgs& a, Layout layout, hipStream_t st)
{
    if (SW == 1 && layout == kFused)
        return run_decode_n<R, W, 1, kFused>(a, st);
    return layout == kPacked ? run_decode_n<R, W, SW, kPacked>(a, st)
                             : run_decode_n<R, W, SW, kTwoLevel>(a, st);
}

template <int R>
hipError_t run_decode_w(const DecodeArgs& a, int W, Layout layout, hipStream_t st)
{
    if (W == 1)
        return run_decode_l<R, 1, 1>(a, layout, st);
    if (a.alphabet <= 256)
        return run_decode_l<R, 2, 1>(a, layout, st);
    return run_decode_l<R, 2, 2>(a, layout, st);
}

template <int R, int W, bool FULL>
hipError_t run_encode(const EncodeArgs& a, hipStream_t st)
{
    const uint32_t segs = 64u >> a.log2N;
    const uint32_t wpb = waves_for(a.n_chunks, segs);
    const uint64_t chunks_per_block = uint64_t(wpb) * segs;
    const uint32_t blocks = static_cast<uint32_t>((a.n_chunks + chunks_per_block - 1) / chunks_per_block);
    auto kern = k_encode<R, W, FULL>;
    hipError_t e = set_lds(kern, a.enc_bytes);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * wpb), a.enc_bytes, st, a);
    return hipGetLastError();
}

template <int R, int W>
hipError_t run_encode_n(const EncodeArgs& a, hipStream_t st)
{
    return a.log2N == 6 ? run_encode<R, W, true>(a, st) : run_encode<R, W, false>(a, st);
}

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, uint32_t count, hipStream_t stream)
{
    const uint32_t blocks = count ? (count + 255) / 256 : 1;
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks < 1024 ? blocks : 1024), dim3(256), 0, stream, p,
                       value, count);
    return hipGetLastError();
}

hipError_t launch_decode(const DecodeArgs& a, int R, int W, Layout layout, hipStream_t stream)
{
    if (a.n_chunks == 0)
        return hipSuccess;
    return R == 16 ? run_decode_w<16>(a, W, layout, stream) : run_decode_w<8>(a, W, layout, stream);
}

hipError_t launch_encode(const EncodeArgs& a, int R, int W, hipStream_t stream)
{
    if (a.n_chunks == 0)
        return hipSuccess;
    if (R == 16)
        return W == 1 ? run_encode_n<16, 1>(a, stream) : run_encode_n<16, 2>(a, stream);
    return W == 1 ? run_encode_n<8, 1>(a, stream) : run_encode_n<8, 2>(a, stream);
}

hipError_t launch_scan(const ScanArgs& a, hipStream_t stream)
{
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kMaxThreads), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_compact(const CompactArgs& a, hipStream_t stream)
{
    if (a.n_chunks == 0)
        return hipSuccess;
    const uint32_t blocks = a.n_chunks < 65535 ? a.n_chunks : 65535;
    hipLaunchKernelGGL(k_compact, dim3(blocks), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace rans
