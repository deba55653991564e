// Batched encode/decode of many independent streams (each with its own
// table) in one pass: a single-block preparation kernel completes each job's
// description on the device (a decode job's chunk count lives in its
// container header), turns chunk counts into work items of G chunks and maps
// items to jobs; a persistent grid then pulls work items from an atomic
// counter.  A block restages its LDS table whenever the next work item
// belongs to another job; each of its G waves codes one chunk with the same
// N = 32 or 64 chunk coder as the single-buffer kernels.  An encoded chunk
// places itself in its job's container at once, by the same look-back over
// the job's lower chunks as the single-buffer encoder; encode work items are
// therefore taken strictly in start order (a ticket from the counter), so
// every chunk a wave waits on belongs to a block that is already running,
// and the copy overlaps the coding of other items.  Every block leaves when
// the counter passes the last item.
#include "encode_seg.h"

namespace rans {
namespace {


// Completes job j's description: chunk size, symbol count and chunk count
// (a decode job's come from its container header, which is checked).
__device__ void plan_job(const BatchArgs& a, uint32_t j, bool decode)
{
    BatchJob& jb = a.jobs[j];
    int32_t st = RANS_OK;
    uint64_t n = 0;
    uint32_t C = 0, nch = 0;
    if (decode) {
        if (jb.in_len < kHeaderBytes) {
            st = RANS_ECORRUPT;
        } else {
            const uint4* h4 = reinterpret_cast<const uint4*>(jb.in);
            const uint4 h0 = h4[0], h1 = h4[1];
            const uint32_t magic = h0.x;
            const uint32_t b4 = h0.y;  // version, k, r, l
            const uint32_t b8 = h0.z;  // w, digit order, N (u16)
            C = h0.w;
            n = uint64_t(h1.x) | (uint64_t(h1.y) << 32);
            nch = h1.z;
            const bool hdr_ok = magic == kMagic && (b4 & 0xFF) == 1 && ((b8 >> 8) & 0xFF) <= 1;
            // every chunk takes a directory entry and at least 4N bytes of
            // states: a container that claims more chunks is malformed (and
            // the host sized the work-item map by this bound)
            if (!hdr_ok || (n == 0 ? nch != 0 : (C == 0 || nch != (n + C - 1) / C)) ||
                kHeaderBytes + (uint64_t(kDirEntryBytes) + 4ull * a.N) * nch > jb.in_len) {
                st = RANS_ECORRUPT;
            } else if (((b4 >> 8) & 0xFF) != a.k || ((b4 >> 16) & 0xFF) != a.r ||
                       (b4 >> 24) != a.l || (b8 & 0xFF) != a.w || (b8 >> 16) != a.N ||
                       ((b8 >> 8) & 0xFF) != a.bf) {
                st = RANS_EINVAL;
            } else if (n * a.w > jb.out_cap) {
                st = RANS_ENOSPC;
            } else if ((uint64_t(C) * a.w) % 16 != 0) {
                st = RANS_EINVAL;  // chunks must start 16-byte aligned in the output
            }
        }
        if (st != RANS_OK) {
            n = 0;
            nch = 0;
        }
        *jb.d_out_len = n;
    } else {
        n = jb.in_len / a.w;
        C = a.C ? a.C : static_cast<uint32_t>(n);
        nch = n ? static_cast<uint32_t>((n + C - 1) / C) : 0;
    }
    *jb.d_status = st;
    jb.n = n;
    jb.C = C;
    jb.nch = nch;
}

// Single block, one launch before the persistent kernel: plans every job,
// scans work items and chunks over the jobs, fills the item -> job (and, to
// encode, chunk -> job) maps and zeroes the work-queue counter.  A job's map
// entries are written by the thread that planned it, or by the whole block
// when the job has many of them.
constexpr uint32_t kPrepThreads = 1024;
constexpr uint32_t kBigJobs = 256;
constexpr uint32_t kSmallEntries = 32;

// Header words of an encode job's container.
__device__ __forceinline__ void job_header(const BatchArgs& a, const BatchJob& jb, uint32_t nch, uint32_t* h)
{
    h[0] = kMagic;
    h[1] = 1u | (a.k << 8) | (a.r << 16) | (a.l << 24);
    h[2] = a.w | (a.bf << 8) | (a.N << 16);
    h[3] = jb.C;
    h[4] = static_cast<uint32_t>(jb.n);
    h[5] = static_cast<uint32_t>(jb.n >> 32);
    h[6] = nch;
    h[7] = 0;
}

__global__ void __launch_bounds__(kPrepThreads) k_batch_prepare(BatchArgs a, bool decode)
{
    __shared__ uint32_t part_i[kPrepThreads];
    // jobs whose map entries (and, to encode, placement words) the whole
    // block writes: job, item base, items (kept here so the block's loop over
    // them reads no global memory)
    __shared__ uint32_t big[kBigJobs][3];
    __shared__ uint32_t nbig;
    const uint32_t T = blockDim.x, tid = threadIdx.x;
    if (tid == 0) {
        // decode: items below grid are taken by block index; encode: every
        // item by ticket, in start order
        a.counter[0] = decode ? a.grid : 0u;
        nbig = 0;
    }
    // contiguous job ranges per thread, so the scan below is ordered
    const uint32_t per = (a.njobs + T - 1) / T;
    const uint32_t lo = min(a.njobs, tid * per), hi = min(a.njobs, lo + per);
    uint32_t si = 0;
    for (uint32_t j = lo; j < hi; ++j) {
        plan_job(a, j, decode);
        si += (a.jobs[j].nch + a.cpi - 1) / a.cpi;
    }
    part_i[tid] = si;
    __syncthreads();
    for (uint32_t o = 1; o < T; o <<= 1) {
        const uint32_t vi = tid >= o ? part_i[tid - o] : 0;
        __syncthreads();
        part_i[tid] += vi;
        __syncthreads();
    }
    uint32_t bi = tid ? part_i[tid - 1] : 0;
    for (uint32_t j = lo; j < hi; ++j) {
        BatchJob& jb = a.jobs[j];
        // a job whose work items would run past the map the host sized fails
        // as a whole instead of being coded in part: its items keep their
        // place in the scan, but with no chunks every wave that takes one
        // skips it
        const uint32_t nch_j = jb.nch, items = (nch_j + a.cpi - 1) / a.cpi;
        const bool over = uint64_t(bi) + items > a.max_items;
        if (over) {
            *jb.d_status = RANS_EINVAL;
            *jb.d_out_len = 0;
            jb.nch = 0;
        }
        jb.item_base = bi;
        const uint32_t words = decode || over ? 0u : nch_j + (nch_j + 63) / 64;
        if (items <= kSmallEntries && words <= 64) {
            // the host sized the map from the jobs' lengths; never exceed it
            for (uint32_t i = 0; i < items; ++i)
                if (bi + i < a.max_items)
                    a.item_job[bi + i] = j;
            for (uint32_t i = 0; i < words; ++i)  // the placement words start at zero
                jb.lookback[i] = 0;
        } else {
            const uint32_t slot = atomicAdd(&nbig, 1u);
            if (slot < kBigJobs) {
                big[slot][0] = j;
                big[slot][1] = bi;
                big[slot][2] = items;
            } else {
                for (uint32_t i = 0; i < items; ++i)
                    if (bi + i < a.max_items)
                        a.item_job[bi + i] = j;
                for (uint32_t i = 0; i < words; ++i)
                    jb.lookback[i] = 0;
            }
        }
        if (!decode && !over && nch_j == 0) {  // no chunk will place it: the header-only container
            *jb.d_out_len = kHeaderBytes;
            if (jb.out_cap >= kHeaderBytes) {
                uint32_t h[8];
                job_header(a, jb, 0, h);
                for (int q = 0; q < 8; ++q)
                    reinterpret_cast<uint32_t*>(jb.out)[q] = h[q];
            } else {
                *jb.d_status = RANS_ENOSPC;
            }
        }
        bi += items;
    }
    if (tid == T - 1)
        a.totals[0] = min(part_i[T - 1], a.max_items);
    __syncthreads();
    const uint32_t nb = min(nbig, kBigJobs);
    for (uint32_t b = 0; b < nb; ++b) {
        const uint32_t j = big[b][0], ib = big[b][1], items = big[b][2];
        for (uint32_t i = tid; i < items; i += T)
            if (ib + i < a.max_items)
                a.item_job[ib + i] = j;
        const BatchJob& jb = a.jobs[j];
        if (!decode && jb.nch) {
            const uint32_t words = jb.nch + (jb.nch + 63) / 64;
            for (uint32_t i = tid; i < words; i += T)
                jb.lookback[i] = 0;
        }
    }
}

// Fetches the block's next work item; returns its job or -1 when the queue
// is exhausted (the same value for every thread of the block).  A block's
// first item is its own index; later ones come from the atomic counter,
// which starts at the grid size.
__device__ __forceinline__ int next_item(const BatchArgs& a, uint32_t* s_slot, uint32_t* item, bool first)
{
    __syncthreads();  // everyone is done with the previous item
    if (threadIdx.x == 0) {
        const uint32_t it = first ? blockIdx.x : atomicAdd(a.counter, 1u);
        s_slot[0] = it;
        const uint32_t j = it < a.totals[0] ? a.item_job[it] : 0xFFFFFFFFu;
        s_slot[1] = j < a.njobs ? j : 0xFFFFFFFFu;
    }
    __syncthreads();
    *item = s_slot[0];
    return static_cast<int>(s_slot[1]);
}

template <int R, int W, int SW, int LAYOUT, int NL, bool BF>
__global__ void __launch_bounds__(1024) k_batch_decode64(const BatchArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ uint32_t s_slot[2];
    const uint32_t wave = c64::uni(threadIdx.x >> 6);
    // the waves' rings and output blocks first (low LDS addresses for the
    // direct-to-LDS loads), the job's tables after them
    constexpr uint32_t SEG = c64::seg_count(NL);  // chunks per wave
    uint8_t* wave_lds = lds + wave * c64::seg_wave_lds_bytes(LAYOUT, NL);
    uint8_t* tab = lds + a.G * c64::seg_wave_lds_bytes(LAYOUT, NL);
    int cur = -1;
    uint32_t item;
    for (bool first = true;; first = false) {
        const int j = next_item(a, s_slot, &item, first);
        if (j < 0)
            break;
        const BatchJob& jb = a.jobs[j];
        if (j != cur) {
            c64::stage2(tab, jb.tab_sym, jb.sym_bytes, jb.tab_ent, jb.ent_bytes);
            __syncthreads();
            cur = j;
        }
        const uint32_t nch = c64::uni(jb.nch);
        const uint32_t c = c64::uni(((item - jb.item_base) * a.G + wave) * SEG);
        if (c < nch) {
            const uint32_t sym_bytes = c64::uni(jb.sym_bytes);
            auto code = [&](auto one) {
                constexpr bool ONE = decltype(one)::value;
                if constexpr (SEG == 1)
                    c64::decode_chunk<R, W, SW, LAYOUT, NL, BF, 0, false, false, ONE>(
                        jb.in, jb.in_len, nch, c, c64::uni(jb.C), jb.n, jb.out, a.k, a.l, tab,
                        reinterpret_cast<const uint32_t*>(tab + sym_bytes), wave_lds, jb.d_status);
                else
                    c64::decode_seg<R, W, SW, LAYOUT, NL, BF, ONE>(jb.in, jb.in_len, nch, c, c64::uni(jb.C), jb.n,
                                                                   jb.out, a.k, a.l, tab,
                                                                   reinterpret_cast<const uint32_t*>(tab + sym_bytes),
                                                                   wave_lds, jb.d_status);
            };
            // byte digits and a one-digit table: the single-byte refill
            // (8-bit symbols only: a second inlined decoder cost the 16-bit
            // symbol kernels 3%, and their tables rarely qualify)
            if constexpr (R == 8 && W == 1) {
                if (c64::uni(jb.one))
                    code(std::true_type{});
                else
                    code(std::false_type{});
            } else {
                code(std::false_type{});
            }
        }
    }
}

// The placement arguments of job jb (nch chunks).
__device__ __forceinline__ PlaceArgs job_place_args(const BatchArgs& a, BatchJob& jb, uint32_t nch)
{
    PlaceArgs pa;
    pa.ticket = nullptr;
    pa.lookback = reinterpret_cast<uint64_t*>(c64::uni64(reinterpret_cast<uintptr_t>(jb.lookback)));
    pa.out = jb.out;
    pa.out_cap = jb.out_cap;
    pa.total = &jb.total;
    pa.total_out = jb.d_out_len;
    uint32_t h[8];
    job_header(a, jb, nch, h);
    for (int q = 0; q < 8; ++q)
        reinterpret_cast<uint32_t*>(pa.hdr)[q] = h[q];
    return pa;
}

template <int R, int W, int NL, bool BF>
__global__ void __launch_bounds__(1024) k_batch_encode64(const BatchArgs a)
{
    // LDS: the waves' digit rings from address 0 (the kernel has no static
    // LDS, so each ring's address is a multiple of its size), their symbol
    // areas, the job's encoder entries, the work-item slot
    extern __shared__ __align__(16) uint8_t lds[];
    const uint32_t wave = c64::uni(threadIdx.x >> 6);
    uint8_t* ring = lds + wave * c64::kEncRing;
    uint8_t* sbuf = lds + a.G * c64::kEncRing + wave * c64::kEncSymArea;
    uint8_t* tab = lds + a.G * c64::kEncWaveLds;
    uint32_t* s_slot = reinterpret_cast<uint32_t*>(tab + a.tab_lds);
    // chunks per wave: with N = 32, lanes 0-31 code chunk c, lanes 32-63 c + 1
    constexpr uint32_t PER = NL == 32 ? 2 : 1;
    int cur = -1;
    uint32_t item;
    for (;;) {
        const int j = next_item(a, s_slot, &item, false);  // tickets only: start order
        if (j < 0)
            break;
        BatchJob& jb = a.jobs[j];
        if (j != cur) {
            c64::stage_enc(tab, jb.enc, jb.enc_bytes, a.l + R - a.k, ~0u, W == 1 ? 256u : 0u);
            __syncthreads();
            cur = j;
        }
        const uint32_t nch = c64::uni(jb.nch);
        const uint32_t c = c64::uni(((item - jb.item_base) * a.G + wave) * PER);
        if (c >= nch)
            continue;
        // the job's own slots (the host sized them for its nch chunks); the
        // digits end at a slot's end, and the stride leaves room after it
        // for the copy's reads past them
        uint8_t* s0 = reinterpret_cast<uint8_t*>(c64::uni64(reinterpret_cast<uintptr_t>(jb.slots))) +
                      uint64_t(c) * a.slot_stride;
        uint32_t x = 0, nd[2] = {0, 0};
        auto code = [&](auto one) {
            constexpr bool ONE = decltype(one)::value;
            if constexpr (NL == 32)
                c64::encode_seg<R, W, BF, ONE>(jb.in, jb.n, c64::uni(jb.C), c, nch, a.l, jb.alphabet,
                                               reinterpret_cast<const uint4*>(tab), s0, s0 + a.slot_stride,
                                               a.slot_bytes, ring, sbuf, jb.d_status, &x, nd);
            else
                c64::encode_chunk<R, W, NL, BF, false, ONE>(jb.in, jb.n, c64::uni(jb.C), c, a.k, a.l, jb.alphabet,
                                                            reinterpret_cast<const uint4*>(tab), s0, a.slot_bytes,
                                                            ring, sbuf, nullptr, nullptr, jb.d_status, &x, &nd[0]);
        };
        // byte digits and a one-digit table: the single-digit step
        if constexpr (R == 8) {
            if (c64::uni(jb.one))
                code(std::true_type{});
            else
                code(std::false_type{});
        } else {
            code(std::false_type{});
        }
        const PlaceArgs pa = job_place_args(a, jb, nch);
        const uint32_t nd0 = c64::uni(nd[0]), nd1 = c64::uni(nd[1]);
        if constexpr (NL == 32) {
            // both lengths and group sums first: no chunk above them, in
            // this group or a later one, waits on this wave's copies
            const uint32_t x1 =
                static_cast<uint32_t>(__shfl(static_cast<int>(x), static_cast<int>((threadIdx.x & 63) | 32)));
            const bool two = c + 1 < nch;
            c64::publish_chunk<R, 32>(c, nd0, pa);
            if (two)
                c64::publish_chunk<R, 32>(c + 1, nd1, pa);
            bool t0 = false, t1 = false;
            const uint64_t l0 = c64::chunk_local<R, 32>(c, nch, nd0, pa, t0);
            const uint64_t l1 = two ? c64::chunk_local<R, 32>(c + 1, nch, nd1, pa, t1) : 0;
            c64::place_chunk<R, 32>(c, nch, x, nd0, s0 + a.slot_bytes - uint64_t(nd0) * (R / 8), pa, jb.d_status,
                                    true, l0, t0);
            if (two)
                c64::place_chunk<R, 32>(c + 1, nch, x1, nd1,
                                        s0 + a.slot_stride + a.slot_bytes - uint64_t(nd1) * (R / 8), pa,
                                        jb.d_status, true, l1, t1);
        } else {
            c64::place_chunk<R, NL>(c, nch, x, nd0, s0 + a.slot_bytes - uint64_t(nd0) * (R / 8), pa, jb.d_status);
        }
    }
}

template <typename K>
hipError_t set_lds(K kernel, uint32_t bytes)
{
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
}

template <int R, int W, int SW, int LAYOUT, int NL, bool BF>
hipError_t persistent_decode(const BatchArgs& a, uint32_t grid, hipStream_t st)
{
    const uint32_t lds = a.tab_lds + a.G * c64::seg_wave_lds_bytes(LAYOUT, NL);
    auto kern = k_batch_decode64<R, W, SW, LAYOUT, NL, BF>;
    hipError_t e = set_lds(kern, lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * a.G), lds, st, a);
    return hipGetLastError();
}

template <int R, int W, int SW, int LAYOUT, bool BF>
hipError_t persistent_decode_n(const BatchArgs& a, uint32_t grid, hipStream_t st)
{
    return a.N == 32 ? persistent_decode<R, W, SW, LAYOUT, 32, BF>(a, grid, st)
                     : persistent_decode<R, W, SW, LAYOUT, 64, BF>(a, grid, st);
}

template <int R, int W, int SW, bool BF>
hipError_t persistent_decode_l(const BatchArgs& a, Layout layout, uint32_t grid, hipStream_t st)
{
    if (SW == 1 && layout == kFused)
        return persistent_decode_n<R, W, 1, kFused, BF>(a, grid, st);
    return layout == kPacked ? persistent_decode_n<R, W, SW, kPacked, BF>(a, grid, st)
                             : persistent_decode_n<R, W, SW, kTwoLevel, BF>(a, grid, st);
}

template <int R, bool BF>
hipError_t persistent_decode_w(const BatchArgs& a, int W, int SW, Layout layout, uint32_t grid,
                               hipStream_t st)
{
    if (W == 1)
        return persistent_decode_l<R, 1, 1, BF>(a, layout, grid, st);
    if (SW == 1)
        return persistent_decode_l<R, 2, 1, BF>(a, layout, grid, st);
    return persistent_decode_l<R, 2, 2, BF>(a, layout, grid, st);
}

template <int R, int W, int NL, bool BF>
hipError_t persistent_encode(const BatchArgs& a, uint32_t grid, hipStream_t st)
{
    const uint32_t lds = a.G * c64::kEncWaveLds + a.tab_lds + 16;  // rings, blocks, table, item slot
    auto kern = k_batch_encode64<R, W, NL, BF>;
    hipError_t e = set_lds(kern, lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * a.G), lds, st, a);
    return hipGetLastError();
}

template <int R, bool BF>
hipError_t persistent_encode_w(const BatchArgs& a, int W, uint32_t grid, hipStream_t st)
{
    if (a.N == 32)
        return W == 1 ? persistent_encode<R, 1, 32, BF>(a, grid, st) : persistent_encode<R, 2, 32, BF>(a, grid, st);
    return W == 1 ? persistent_encode<R, 1, 64, BF>(a, grid, st) : persistent_encode<R, 2, 64, BF>(a, grid, st);
}

}  // namespace

hipError_t launch_batch(const BatchArgs& a, bool decode, int R, int W, int SW, Layout layout,
                        uint32_t grid, hipStream_t st)
{
    if (a.njobs == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_batch_prepare, dim3(1), dim3(kPrepThreads), 0, st, a, decode);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    // 16-bit digits: one digit per step at most (b >= M), both orders coincide
    if (decode) {
        if (R == 16)
            return persistent_decode_w<16, false>(a, W, SW, layout, grid, st);
        return a.bf ? persistent_decode_w<8, true>(a, W, SW, layout, grid, st)
                    : persistent_decode_w<8, false>(a, W, SW, layout, grid, st);
    }
    if (R == 16)
        e = persistent_encode_w<16, false>(a, W, grid, st);
    else if (a.bf)
        e = persistent_encode_w<8, true>(a, W, grid, st);
    else
        e = persistent_encode_w<8, false>(a, W, grid, st);
    return e;
}

}  // namespace rans
