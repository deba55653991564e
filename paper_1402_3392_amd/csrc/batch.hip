// Batched encode/decode of many independent streams (each with its own
// table) in one pass: a single-block preparation kernel completes each job's
// description on the device (a decode job's chunk count lives in its
// container header), turns chunk counts into work items of G chunks and maps
// items to jobs; a persistent grid then pulls work items from an atomic
// counter.  A block restages its LDS table
// whenever the next work item belongs to another job; each of its G waves
// codes one chunk with the same N = 32 or 64 chunk coder as the single-buffer
// kernels.  Encode jobs then get their container laid out per job (scan of
// chunk lengths, header, directory) and compacted.  No kernel waits on
// another block: every block leaves when the counter passes the last item.
#include "coder64.h"

namespace rans {
namespace {

__device__ __forceinline__ uint64_t align16(uint64_t v) { return (v + 15) & ~uint64_t(15); }

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

__global__ void __launch_bounds__(kPrepThreads) k_batch_prepare(BatchArgs a, bool decode)
{
    __shared__ uint32_t part_i[kPrepThreads], part_c[kPrepThreads];
    __shared__ uint32_t big[kBigJobs];
    __shared__ uint32_t nbig;
    const uint32_t T = blockDim.x, tid = threadIdx.x;
    if (tid == 0) {
        a.counter[0] = a.grid;  // items below grid are taken by block index
        nbig = 0;
    }
    // contiguous job ranges per thread, so the scan below is ordered
    const uint32_t per = (a.njobs + T - 1) / T;
    const uint32_t lo = min(a.njobs, tid * per), hi = min(a.njobs, lo + per);
    uint32_t si = 0, sc = 0;
    for (uint32_t j = lo; j < hi; ++j) {
        plan_job(a, j, decode);
        si += (a.jobs[j].nch + a.G - 1) / a.G;
        sc += a.jobs[j].nch;
    }
    part_i[tid] = si;
    part_c[tid] = sc;
    __syncthreads();
    for (uint32_t o = 1; o < T; o <<= 1) {
        const uint32_t vi = tid >= o ? part_i[tid - o] : 0, vc = tid >= o ? part_c[tid - o] : 0;
        __syncthreads();
        part_i[tid] += vi;
        part_c[tid] += vc;
        __syncthreads();
    }
    uint32_t bi = tid ? part_i[tid - 1] : 0, bc = tid ? part_c[tid - 1] : 0;
    for (uint32_t j = lo; j < hi; ++j) {
        BatchJob& jb = a.jobs[j];
        jb.item_base = bi;
        jb.chunk_base = bc;
        const uint32_t items = (jb.nch + a.G - 1) / a.G;
        if (items <= kSmallEntries && (decode || jb.nch <= kSmallEntries)) {
            // the host sized the maps from the jobs' lengths; never exceed them
            for (uint32_t i = 0; i < items; ++i)
                if (bi + i < a.max_items)
                    a.item_job[bi + i] = j;
            if (!decode)
                for (uint32_t c = 0; c < jb.nch; ++c)
                    if (bc + c < a.max_chunks)
                        a.chunk_job[bc + c] = j;
        } else {
            const uint32_t slot = atomicAdd(&nbig, 1u);
            if (slot < kBigJobs) {
                big[slot] = j;
            } else {
                for (uint32_t i = 0; i < items; ++i)
                    if (bi + i < a.max_items)
                        a.item_job[bi + i] = j;
                if (!decode)
                    for (uint32_t c = 0; c < jb.nch; ++c)
                        if (bc + c < a.max_chunks)
                            a.chunk_job[bc + c] = j;
            }
        }
        bi += items;
        bc += jb.nch;
    }
    if (tid == T - 1) {
        a.totals[0] = min(part_i[T - 1], a.max_items);
        a.totals[1] = min(part_c[T - 1], a.max_chunks);
    }
    __syncthreads();
    const uint32_t nb = min(nbig, kBigJobs);
    for (uint32_t b = 0; b < nb; ++b) {
        const uint32_t j = big[b];
        const BatchJob& jb = a.jobs[j];
        const uint32_t items = (jb.nch + a.G - 1) / a.G;
        for (uint32_t i = tid; i < items; i += T)
            if (jb.item_base + i < a.max_items)
                a.item_job[jb.item_base + i] = j;
        if (!decode)
            for (uint32_t c = tid; c < jb.nch; c += T)
                if (jb.chunk_base + c < a.max_chunks)
                    a.chunk_job[jb.chunk_base + c] = j;
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
    uint8_t* wave_lds = lds + wave * c64::wave_lds_bytes(LAYOUT);
    uint8_t* tab = lds + a.G * c64::wave_lds_bytes(LAYOUT);
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
        const uint32_t c = c64::uni((item - jb.item_base) * a.G + wave);
        if (c < nch) {
            const uint32_t sym_bytes = c64::uni(jb.sym_bytes);
            c64::decode_chunk<R, W, SW, LAYOUT, NL, BF>(jb.in, jb.in_len, nch, c, c64::uni(jb.C), jb.n, jb.out,
                                                a.k, a.l, tab,
                                                reinterpret_cast<const uint32_t*>(tab + sym_bytes),
                                                wave_lds, jb.d_status);
        }
    }
}

template <int R, int W, int NL, bool BF>
__global__ void __launch_bounds__(1024) k_batch_encode64(const BatchArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ uint32_t s_slot[2];
    const uint32_t wave = c64::uni(threadIdx.x >> 6);
    uint8_t* sbuf = lds + a.tab_lds + wave * c64::kEncWaveLds;
    int cur = -1;
    uint32_t item;
    for (bool first = true;; first = false) {
        const int j = next_item(a, s_slot, &item, first);
        if (j < 0)
            break;
        const BatchJob& jb = a.jobs[j];
        if (j != cur) {
            c64::stage_enc(lds, jb.enc, jb.enc_bytes, a.l + R - a.k);
            __syncthreads();
            cur = j;
        }
        const uint32_t nch = c64::uni(jb.nch);
        const uint32_t c = c64::uni((item - jb.item_base) * a.G + wave);
        if (c < nch) {
            const uint64_t g = c64::uni(jb.chunk_base) + uint64_t(c);
            c64::encode_chunk<R, W, NL, BF>(jb.in, jb.n, c64::uni(jb.C), c, a.k, a.l, jb.alphabet,
                                    reinterpret_cast<const uint4*>(lds), a.slots + g * a.slot_stride,
                                    a.slot_bytes, sbuf, a.states + g * 64, a.ndig + g, jb.d_status);
        }
    }
}

// Block per encode job: chunk offsets, directory, header, container length.
__global__ void __launch_bounds__(256) k_batch_cscan(BatchArgs a)
{
    __shared__ uint64_t part[256];
    const uint32_t j = blockIdx.x;
    if (j >= a.njobs)
        return;
    BatchJob& jb = a.jobs[j];
    const uint32_t T = blockDim.x, tid = threadIdx.x, nch = jb.nch, db = a.r / 8;
    const uint32_t per = (nch + T - 1) / T;
    const uint32_t lo = min(nch, tid * per), hi = min(nch, lo + per);
    uint64_t sum = 0;
    for (uint32_t c = lo; c < hi; ++c)
        sum += align16(4ull * a.N + uint64_t(a.ndig[jb.chunk_base + c]) * db);
    part[tid] = sum;
    __syncthreads();
    for (uint32_t o = 1; o < T; o <<= 1) {
        const uint64_t v = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    const uint64_t base = align16(kHeaderBytes + uint64_t(kDirEntryBytes) * nch);
    const uint64_t total = nch ? base + part[T - 1] : kHeaderBytes;
    const bool fits = total <= jb.out_cap;
    uint64_t off = base + (tid ? part[tid - 1] : 0);
    for (uint32_t c = lo; c < hi; ++c) {
        const uint32_t len = 4 * a.N + a.ndig[jb.chunk_base + c] * db;
        a.chunk_off[jb.chunk_base + c] = off;
        if (fits) {
            uint8_t* de = jb.out + kHeaderBytes + uint64_t(kDirEntryBytes) * c;
            *reinterpret_cast<uint64_t*>(de) = off;
            reinterpret_cast<uint32_t*>(de)[2] = len;
            reinterpret_cast<uint32_t*>(de)[3] = 0;
        }
        off += align16(len);
    }
    if (tid == 0) {
        jb.total = total;
        *jb.d_out_len = total;
        if (fits) {
            uint32_t* h = reinterpret_cast<uint32_t*>(jb.out);
            h[0] = kMagic;
            h[1] = 1u | (a.k << 8) | (a.r << 16) | (a.l << 24);
            h[2] = a.w | (a.bf << 8) | (a.N << 16);
            h[3] = jb.C;
            h[4] = static_cast<uint32_t>(jb.n);
            h[5] = static_cast<uint32_t>(jb.n >> 32);
            h[6] = nch;
            h[7] = 0;
        } else {
            atomicMin(jb.d_status, RANS_ENOSPC);
        }
    }
}

// Grid-stride over all chunks of the batch: move each chunk (states + digits
// from the end of its slot) to its directory offset, zero padding.
__global__ void __launch_bounds__(256) k_batch_compact(BatchArgs a)
{
    const uint32_t nchunks = a.totals[1];
    for (uint32_t g = blockIdx.x; g < nchunks; g += gridDim.x) {
        const BatchJob& jb = a.jobs[a.chunk_job[g]];
        if (jb.total > jb.out_cap)
            continue;
        const uint32_t db = a.r / 8, N = a.N;
        const uint64_t off = a.chunk_off[g];
        const uint32_t pay = a.ndig[g] * db;
        const uint32_t words = static_cast<uint32_t>(align16(4ull * N + pay) / 4);
        const uint8_t* slot_end = a.slots + uint64_t(g) * a.slot_stride + a.slot_bytes;
        const uint8_t* src = slot_end - pay;
        uint32_t* dst = reinterpret_cast<uint32_t*>(jb.out + off);
        for (uint32_t q = threadIdx.x; q < words; q += blockDim.x) {
            uint32_t v = 0;
            if (q < N) {
                v = a.states[uint64_t(g) * 64 + q];
            } else {
                const uint32_t p = (q - N) * 4;
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

template <typename K>
hipError_t set_lds(K kernel, uint32_t bytes)
{
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
}

template <int R, int W, int SW, int LAYOUT, int NL, bool BF>
hipError_t persistent_decode(const BatchArgs& a, uint32_t grid, hipStream_t st)
{
    const uint32_t lds = a.tab_lds + a.G * c64::wave_lds_bytes(LAYOUT);
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
    const uint32_t lds = a.tab_lds + a.G * c64::kEncWaveLds;
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
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_batch_cscan, dim3(a.njobs), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_batch_compact, dim3(4096), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace rans
