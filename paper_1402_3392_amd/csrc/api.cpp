// librans single-buffer entry points: parameter checks, container header,
// per-stream device workspace, kernel launches and status read-back.
#include <cstring>
#include <map>
#include <mutex>
#include <utility>

#include "rans_internal.h"
#include "timing.h"
#include "workspace.h"

namespace rans {

int max_lds_bytes()
{
    // per device, asked once (every launch needs it)
    static std::mutex mu;
    static std::map<int, int> known;
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return 65536;
    std::lock_guard<std::mutex> lk(mu);
    auto it = known.find(dev);
    if (it != known.end())
        return it->second;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 65536;
    known[dev] = v;
    return v;
}

int check_params(const rans_params* p)
{
    if (!p)
        return RANS_EINVAL;
    const uint32_t k = p->prob_bits, r = p->radix_bits, l = p->state_lbits, w = p->sym_bytes,
                   N = p->interleave;
    if (k < 8 || k > 15 || (r != 8 && r != 16) || l < k || l + r > 32 || (w != 1 && w != 2))
        return RANS_EINVAL;
    if (N < 1 || N > 64 || (N & (N - 1)) != 0 || p->digit_order > 1 || p->escape > 1)
        return RANS_EINVAL;
    // escape coding: 16-bit symbols, depth-first digit order
    if (p->escape && (w != 2 || p->digit_order != 0))
        return RANS_EINVAL;
    return RANS_OK;
}

uint32_t log2u(uint32_t v)
{
    uint32_t r = 0;
    while ((1u << r) < v)
        ++r;
    return r;
}

// Digits a symbol can emit at most: the state drops below f*b*L/M after at
// most ceil(k/r) divisions by b.
uint32_t max_digits(uint32_t k, uint32_t r) { return (k + r - 1) / r; }

// Raw digits an escaped 16-bit value adds (escape coding).
uint32_t raw_digits(uint32_t r) { return 16 / r; }

// Digit slot of one chunk: room for its largest stream, rounded to whole
// encoder windows (kSlotAlign bytes, aligned to the slot's end).
uint64_t slot_bytes_for(uint32_t C, uint32_t k, uint32_t r, bool esc)
{
    const uint64_t per = max_digits(k, r) + (esc ? raw_digits(r) : 0);
    return (uint64_t(C) * per * (r / 8) + kSlotAlign - 1) & ~(kSlotAlign - 1);
}

void make_header(uint8_t* h, const rans_params& p, uint32_t C, uint64_t n, uint32_t nch)
{
    std::memset(h, 0, 32);
    const uint32_t magic = kMagic;
    std::memcpy(h, &magic, 4);
    h[4] = 1;
    h[5] = p.prob_bits;
    h[6] = p.radix_bits;
    h[7] = p.state_lbits;
    h[8] = p.sym_bytes;
    h[9] = static_cast<uint8_t>(p.digit_order | (p.escape << 1));
    const uint16_t N = p.interleave;
    std::memcpy(h + 10, &N, 2);
    std::memcpy(h + 12, &C, 4);
    std::memcpy(h + 16, &n, 8);
    std::memcpy(h + 24, &nch, 4);
}

int parse_header(const uint8_t* h, uint64_t in_len, Header* out)
{
    uint32_t magic, C, nch;
    uint16_t N;
    uint64_t n;
    std::memcpy(&magic, h, 4);
    std::memcpy(&N, h + 10, 2);
    std::memcpy(&C, h + 12, 4);
    std::memcpy(&n, h + 16, 8);
    std::memcpy(&nch, h + 24, 4);
    if (magic != kMagic || h[4] != 1 || (h[9] > 3 && h[9] != 4))
        return RANS_ECORRUPT;
    rans_params p{};
    p.prob_bits = h[5];
    p.radix_bits = h[6];
    p.state_lbits = h[7];
    p.sym_bytes = h[8];
    p.interleave = N;
    const bool pfx = h[9] == 4;  // the prefix-code family: 16-bit words
    p.digit_order = pfx ? 0 : h[9] & 1;
    p.escape = pfx ? 0 : h[9] >> 1;
    p.chunk_syms = C;
    if (check_params(&p) != RANS_OK)
        return RANS_ECORRUPT;
    if (n == 0 ? nch != 0 : (C == 0 || nch != (n + C - 1) / C))
        return RANS_ECORRUPT;
    if (kHeaderBytes + uint64_t(kDirEntryBytes) * nch > in_len)
        return RANS_ECORRUPT;
    if (pfx && p.radix_bits != 16)
        return RANS_ECORRUPT;
    out->pfx = pfx;
    out->p = p;
    out->n = n;
    out->n_chunks = nch;
    return RANS_OK;
}

bool choose_layout(const DevTable& t, Layout* layout, uint32_t* lds, uint32_t extra, uint32_t seg_n)
{
    const uint64_t maxl = static_cast<uint64_t>(max_lds_bytes());
    // LDS per wave of the kernel that will run: the segment decoder for
    // symbol output (seg_n = N), else the one-chunk decoder
    auto per_wave = [seg_n](Layout lay) {
        return seg_n ? decode_seg_lds_per_wave(lay, seg_n) : decode64_lds_per_wave(lay);
    };
    const uint64_t packed = t.dec_bytes + t.sym_bytes + extra, two = t.sym_bytes + t.fc_bytes + extra;
    // One LDS read per symbol when the fused table leaves room for 16 waves'
    // rings; else the packed table (two independent reads) while it leaves
    // room for a second block; else the small two-level table with room for
    // at least one wave.  `extra`: LDS the kernel stages beside the table.
    if (t.fused && t.fused_bytes + extra + 16 * per_wave(kFused) <= maxl) {
        *layout = kFused;
        *lds = static_cast<uint32_t>(t.fused_bytes + extra);
        return true;
    }
    if (packed + per_wave(kPacked) <= maxl && packed <= 96 * 1024) {
        *layout = kPacked;
        *lds = static_cast<uint32_t>(packed);
        return true;
    }
    if (two + per_wave(kTwoLevel) <= maxl) {
        *layout = kTwoLevel;
        *lds = static_cast<uint32_t>(two);
        return true;
    }
    return false;
}

void fill_decode_tables(const DevTable& t, Layout layout, DecodeArgs* a)
{
    if (layout == kFused) {
        a->tab0 = t.fused;
        a->tab0_bytes = static_cast<uint32_t>(t.fused_bytes);
        a->tab1 = nullptr;
        a->tab1_bytes = 0;
    } else if (layout == kPacked) {
        a->tab0 = t.dec;
        a->tab0_bytes = static_cast<uint32_t>(t.dec_bytes);
        a->tab1 = t.sym;
        a->tab1_bytes = static_cast<uint32_t>(t.sym_bytes);
    } else {
        a->tab0 = t.sym;
        a->tab0_bytes = static_cast<uint32_t>(t.sym_bytes);
        a->tab1 = t.fc;
        a->tab1_bytes = static_cast<uint32_t>(t.fc_bytes);
    }
}

}  // namespace rans

using namespace rans;

extern "C" int rans_params_check(const rans_params* params) { return check_params(params); }

extern "C" uint64_t rans_encode_bound(uint64_t n, const rans_params* p)
{
    if (check_params(p) != RANS_OK)
        return 0;
    uint64_t C = p->chunk_syms ? p->chunk_syms : n;
    if (n == 0 || C == 0)
        return kHeaderBytes;
    if (C > 0xFFFFFFFFull)
        return 0;
    const uint64_t nch = (n + C - 1) / C;
    const uint64_t per = uint64_t(max_digits(p->prob_bits, p->radix_bits) +
                                  (p->escape ? raw_digits(p->radix_bits) : 0)) *
                         (p->radix_bits / 8);
    const uint64_t full = nch - 1, last = n - full * C;
    auto a16 = [](uint64_t v) { return (v + 15) & ~uint64_t(15); };
    return a16(kHeaderBytes + kDirEntryBytes * nch) +
           full * a16(4ull * p->interleave + per * C) + a16(4ull * p->interleave + per * last);
}

extern "C" const char* rans_strerror(int code)
{
    switch (code) {
    case RANS_OK: return "ok";
    case RANS_EINVAL: return "invalid argument or parameters";
    case RANS_EPREC: return "more distinct symbols than 2^prob_bits";
    case RANS_ENOSYM: return "symbol with zero frequency or outside the alphabet";
    case RANS_ENOSPC: return "output buffer too small";
    case RANS_ECORRUPT: return "corrupt or truncated stream";
    case RANS_EDEVICE: return "HIP runtime error";
    case RANS_ENOMEM: return "out of memory";
    default: return "unknown error";
    }
}

// The one-wave-per-chunk kernels move symbols in 16-byte pieces: every chunk
// must start 16-byte aligned in the symbol buffer.
static bool fast64(uint32_t N, uint32_t C, uint32_t W, const void* syms)
{
    return (N == 32 || N == 64) && (uint64_t(C) * W) % 16 == 0 &&
           (reinterpret_cast<uintptr_t>(syms) & 15) == 0;
}

// Validates an encode call and fills the launch arguments (host only).
// pfx: the prefix-code family multiplexed as Section 4 describes.
int rans::prepare_encode(const rans_table* table, const rans_params* params, const void* d_syms,
                         uint64_t n, void* d_out, EncodeArgs* ea, ScanArgs* sa, CompactArgs* ca,
                   PlaceArgs* pa, uint64_t* ws_need, bool pfx)
{
    if (!table || !d_out)
        return RANS_EINVAL;
    int rc = check_params(params);
    if (rc != RANS_OK)
        return rc;
    const DevTable& t = *dev_table(table);
    const rans_params& p = *params;
    if (t.k != p.prob_bits || (n && !d_syms))
        return RANS_EINVAL;
    if ((reinterpret_cast<uintptr_t>(d_out) & 15) ||
        (reinterpret_cast<uintptr_t>(d_syms) & (p.sym_bytes - 1)))
        return RANS_EINVAL;
    const uint64_t C64 = p.chunk_syms ? p.chunk_syms : n;
    if (C64 > 0xFFFFFFFFull)
        return RANS_EINVAL;
    const uint32_t C = static_cast<uint32_t>(C64);
    const uint64_t nch64 = n ? (n + C - 1) / C : 0;
    if (nch64 > 0xFFFFFFFFull)
        return RANS_EINVAL;
    const uint32_t nch = static_cast<uint32_t>(nch64);
    const uint32_t R = p.radix_bits, N = p.interleave;
    // prefix-code family: 16-bit words, no rANS variants, the one-wave-per-
    // chunk kernel only, and a table whose symbols fit its code entries
    if (pfx && (R != 16 || p.state_lbits != 16 || p.digit_order || p.escape || !t.pfx_enc ||
                (n && !fast64(N, C, p.sym_bytes, d_syms))))
        return RANS_EINVAL;
    // a prefix-coded chunk holds at most a word per symbol plus one per coder
    const uint64_t sb = pfx ? (2 * (uint64_t(C) + 64) + 255) & ~uint64_t(255)
                            : slot_bytes_for(C, p.prob_bits, R, p.escape != 0);
    const EncodeLayout el = encode_layout(nch, N, sb);
    *ws_need = el.total;

    *ea = EncodeArgs{};
    ea->syms = d_syms;
    ea->n = n;
    ea->C = C;
    ea->n_chunks = nch;
    ea->N = N;
    ea->log2N = log2u(N);
    ea->k = p.prob_bits;
    ea->l = p.state_lbits;
    ea->alphabet = t.alphabet;
    ea->bf = p.digit_order;
    ea->esc = p.escape;
    ea->one = R == 8 && !p.escape && t.one_digit ? 1u : 0u;
    ea->enc = pfx ? reinterpret_cast<const uint4*>(t.pfx_enc) : t.enc;
    ea->enc_bytes = static_cast<uint32_t>(pfx ? t.pfx_enc_bytes : t.enc_bytes);
    ea->slot_bytes = sb;
    ea->slot_stride = sb + kSlotPad;

    *sa = ScanArgs{};
    sa->n_chunks = nch;
    sa->N = N;
    sa->digit_bytes = R / 8;
    sa->out = static_cast<uint8_t*>(d_out);
    make_header(sa->hdr, p, C, n, nch);
    if (pfx)
        sa->hdr[9] = 4;  // flags: the prefix-code family

    *ca = CompactArgs{};
    ca->slot_bytes = sb;
    ca->slot_stride = sb + kSlotPad;
    ca->n_chunks = nch;
    ca->N = N;
    ca->digit_bytes = R / 8;
    ca->out = sa->out;
    // workspace offsets are stored now and rebased in bind_workspace
    ea->slots = reinterpret_cast<uint8_t*>(el.slots);
    ea->states = reinterpret_cast<uint32_t*>(el.states);
    ea->ndig = reinterpret_cast<uint32_t*>(el.ndig);
    sa->chunk_off = reinterpret_cast<uint64_t*>(el.chunk_off);
    sa->total = reinterpret_cast<uint64_t*>(el.flags + 8);
    *pa = PlaceArgs{};
    pa->ticket = reinterpret_cast<uint32_t*>(el.lookback + 8 * (nch + (uint64_t(nch) + 63) / 64));
    pa->lookback = reinterpret_cast<uint64_t*>(el.lookback);
    pa->out = sa->out;
    std::memcpy(pa->hdr, sa->hdr, 32);
    return RANS_OK;
}

void rans::bind_workspace(uint8_t* base, EncodeArgs* ea, ScanArgs* sa, CompactArgs* ca, PlaceArgs* pa)
{
    auto rb = [base](auto* p) { return reinterpret_cast<decltype(p)>(base + reinterpret_cast<uintptr_t>(p)); };
    ea->slots = rb(ea->slots);
    ea->states = rb(ea->states);
    ea->ndig = rb(ea->ndig);
    sa->chunk_off = rb(sa->chunk_off);
    sa->total = rb(sa->total);
    sa->ndig = ea->ndig;
    ca->slots = ea->slots;
    ca->states = ea->states;
    ca->ndig = ea->ndig;
    ca->chunk_off = sa->chunk_off;
    ca->total = sa->total;
    pa->ticket = rb(pa->ticket);
    pa->lookback = rb(pa->lookback);
    pa->total = sa->total;
}

hipError_t rans::enqueue_encode(const EncodeArgs& ea, const ScanArgs& sa, const CompactArgs& ca,
                                const PlaceArgs& pa, int R, int W, hipStream_t st, bool pfx, bool timed)
{
    hipError_t e;
    if (pfx) {
        if (ea.n_chunks == 0)  // the header alone: the scan kernel writes it
            return launch_scan(sa, st);
        // the look-back words and the ticket after them start at zero
        e = launch_fill_u32(reinterpret_cast<uint32_t*>(pa.lookback), 0,
                            2 * (ea.n_chunks + (ea.n_chunks + 63) / 64 + 1), st);
        if (e != hipSuccess)
            return e;
        TimingScope ts(RANS_KERNEL_ENCODE, st, timed);
        return launch_pfx_encode64(ea, pa, W, st);
    }
    if (ea.n_chunks > 0 && fast64(ea.N, ea.C, W, ea.syms)) {
        // one kernel: encode and place by look-back (the look-back words and
        // the ticket after them start at zero: one fill)
        e = launch_fill_u32(reinterpret_cast<uint32_t*>(pa.lookback), 0,
                            2 * (ea.n_chunks + (ea.n_chunks + 63) / 64 + 1), st);
        if (e != hipSuccess)
            return e;
        TimingScope ts(RANS_KERNEL_ENCODE, st, timed);
        return launch_encode64_place(ea, pa, R, W, st);
    }
    {
        TimingScope ts(RANS_KERNEL_ENCODE, st, timed);
        e = launch_encode(ea, R, W, st);
    }
    if (e == hipSuccess) {
        TimingScope ts(RANS_KERNEL_SCAN, st, timed);
        e = launch_scan(sa, st);
    }
    if (e == hipSuccess) {
        TimingScope ts(RANS_KERNEL_COMPACT, st, timed);
        e = launch_compact(ca, st);
    }
    return e;
}

static hipError_t enqueue_decode(const DecodeArgs& da, int R, int W, Layout layout, hipStream_t st)
{
    TimingScope ts(RANS_KERNEL_DECODE, st);
    if (da.lut_w)
        return launch_decode64_lut(da, R, layout, st);
    return fast64(da.N, da.C, W, da.out) ? launch_decode64(da, R, W, layout, st)
                                         : launch_decode(da, R, W, layout, st);
}

static int encode_async(const rans_table* table, const rans_params* params, const void* d_syms,
                        uint64_t n, void* d_out, uint64_t out_cap, uint64_t* d_out_len,
                        int32_t* d_status, void* stream, bool pfx)
{
    if (!d_status)
        return RANS_EINVAL;
    EncodeArgs ea;
    ScanArgs sa;
    CompactArgs ca;
    PlaceArgs pa;
    uint64_t need = 0;
    int rc = prepare_encode(table, params, d_syms, n, d_out, &ea, &sa, &ca, &pa, &need, pfx);
    if (rc != RANS_OK)
        return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Workspace* ws = workspace_for(st);
    if (!ws)
        return RANS_ENOMEM;
    std::lock_guard<std::mutex> lk(ws->mu);
    rc = ws->reserve(need);
    if (rc != RANS_OK)
        return rc;
    bind_workspace(static_cast<uint8_t*>(ws->dev), &ea, &sa, &ca, &pa);
    ea.status = sa.status = d_status;
    sa.out_cap = ca.out_cap = pa.out_cap = out_cap;
    sa.total_out = pa.total_out = d_out_len;
    return enqueue_encode(ea, sa, ca, pa, params->radix_bits, params->sym_bytes, st, pfx) == hipSuccess
               ? RANS_OK
               : RANS_EDEVICE;
}

static int encode_sync(const rans_table* table, const rans_params* params, const void* d_syms,
                       uint64_t n, void* d_out, uint64_t out_cap, uint64_t* out_len, void* stream,
                       bool pfx)
{
    if (!out_len)
        return RANS_EINVAL;
    *out_len = 0;
    EncodeArgs ea;
    ScanArgs sa;
    CompactArgs ca;
    PlaceArgs pa;
    uint64_t need = 0;
    int rc = prepare_encode(table, params, d_syms, n, d_out, &ea, &sa, &ca, &pa, &need, pfx);
    if (rc != RANS_OK)
        return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Workspace* ws = workspace_for(st);
    if (!ws)
        return RANS_ENOMEM;
    std::lock_guard<std::mutex> lk(ws->mu);
    rc = ws->reserve(need);
    if (rc != RANS_OK)
        return rc;
    uint8_t* base = static_cast<uint8_t*>(ws->dev);
    bind_workspace(base, &ea, &sa, &ca, &pa);
    int32_t* status = reinterpret_cast<int32_t*>(base);  // flags word at offset 0
    ea.status = sa.status = status;
    sa.out_cap = ca.out_cap = pa.out_cap = out_cap;
    sa.total_out = pa.total_out = nullptr;
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(status), 0, 1, st);
    if (e == hipSuccess)
        e = enqueue_encode(ea, sa, ca, pa, params->radix_bits, params->sym_bytes, st, pfx);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws->host, base, 16, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e != hipSuccess)
        return RANS_EDEVICE;
    int32_t code;
    uint64_t total;
    std::memcpy(&code, ws->host, 4);
    std::memcpy(&total, static_cast<uint8_t*>(ws->host) + 8, 8);
    *out_len = total;
    return code;
}

extern "C" int rans_encode_async(const rans_table* table, const rans_params* params,
                                 const void* d_syms, uint64_t n, void* d_out, uint64_t out_cap,
                                 uint64_t* d_out_len, int32_t* d_status, void* stream)
{
    return encode_async(table, params, d_syms, n, d_out, out_cap, d_out_len, d_status, stream, false);
}

extern "C" int rans_encode(const rans_table* table, const rans_params* params, const void* d_syms,
                           uint64_t n, void* d_out, uint64_t out_cap, uint64_t* out_len,
                           void* stream)
{
    return encode_sync(table, params, d_syms, n, d_out, out_cap, out_len, stream, false);
}

extern "C" int rans_pfx_encode_async(const rans_table* table, const rans_params* params,
                                     const void* d_syms, uint64_t n, void* d_out, uint64_t out_cap,
                                     uint64_t* d_out_len, int32_t* d_status, void* stream)
{
    return encode_async(table, params, d_syms, n, d_out, out_cap, d_out_len, d_status, stream, true);
}

extern "C" int rans_pfx_encode(const rans_table* table, const rans_params* params, const void* d_syms,
                               uint64_t n, void* d_out, uint64_t out_cap, uint64_t* out_len,
                               void* stream)
{
    return encode_sync(table, params, d_syms, n, d_out, out_cap, out_len, stream, true);
}

// Validates a decode call against a host copy of the header.  lut_w != 0:
// the fused lookup variant (output element i = d_lut[symbol i], lut_w
// bytes; the one-wave-per-chunk kernels only).
static int prepare_decode(const rans_table* table, const void* d_in, uint64_t in_len,
                          const uint8_t* h_header, void* d_syms, uint64_t syms_cap,
                          DecodeArgs* da, Header* h, Layout* layout, const void* d_lut = nullptr,
                          uint32_t lut_w = 0)
{
    int rc = parse_header(h_header, in_len, h);
    if (rc != RANS_OK)
        return rc;
    const DevTable& t = *dev_table(table);
    if (t.k != h->p.prob_bits)
        return RANS_EINVAL;
    if (lut_w == 0) {
        if (h->p.sym_bytes == 1 && t.sym_w != 1)
            return RANS_EINVAL;
        if (h->n > syms_cap)
            return RANS_ENOSPC;
        if (h->n && (!d_syms || (reinterpret_cast<uintptr_t>(d_syms) & (h->p.sym_bytes - 1))))
            return RANS_EINVAL;
    } else {
        if ((lut_w != 2 && lut_w != 4) || !d_lut || (reinterpret_cast<uintptr_t>(d_lut) & (lut_w - 1)))
            return RANS_EINVAL;
        if (h->p.escape)  // escaped values lie outside the table, so outside the LUT
            return RANS_EINVAL;
        if (h->n > syms_cap)
            return RANS_ENOSPC;
        if (h->n && (!d_syms || !fast64(h->p.interleave, h->p.chunk_syms, lut_w, d_syms)))
            return RANS_EINVAL;
    }
    if (h->pfx && (lut_w || !t.pfx_dec ||
                   (h->n && !fast64(h->p.interleave, h->p.chunk_syms, h->p.sym_bytes, d_syms))))
        return RANS_EINVAL;  // the one-wave-per-chunk decoder, symbol output only
    uint32_t lds;
    const uint32_t seg_n = lut_w == 0 && !h->p.escape && !h->pfx ? h->p.interleave : 0;
    if (!choose_layout(t, layout, &lds, lut_w ? lut_lds_bytes(t.alphabet, lut_w) : 0, seg_n))
        return RANS_EINVAL;
    *da = DecodeArgs{};
    da->in = static_cast<const uint8_t*>(d_in);
    da->in_len = in_len;
    da->out = d_syms;
    da->n = h->n;
    da->C = h->p.chunk_syms;
    da->n_chunks = h->n_chunks;
    da->N = h->p.interleave;
    da->log2N = log2u(da->N);
    da->k = h->p.prob_bits;
    da->l = h->p.state_lbits;
    da->alphabet = t.alphabet;
    da->bf = h->p.digit_order;
    da->esc = h->p.escape;
    da->one = h->p.radix_bits == 8 && !h->p.escape && !h->pfx && t.one_digit ? 1u : 0u;
    da->lut = d_lut;
    da->lut_w = lut_w;
    fill_decode_tables(t, *layout, da);
    if (h->pfx) {  // its lookup table stands in for the packed layout's entries
        da->pfx = 1;
        da->k = t.pfx_maxlen;
        da->tab0 = t.pfx_dec;
        da->tab0_bytes = static_cast<uint32_t>(t.pfx_dec_bytes);
        da->tab1 = nullptr;
        da->tab1_bytes = 0;
        *layout = kPacked;
    }
    return RANS_OK;
}

// Shared body of the stream-ordered decodes.
static int decode_async(const rans_table* table, const void* d_in, uint64_t in_len,
                        const void* h_header, void* d_out, uint64_t cap, const void* d_lut,
                        uint32_t lut_w, int32_t* d_status, void* stream)
{
    if (!table || !d_in || !h_header || !d_status)
        return RANS_EINVAL;
    if (in_len < kHeaderBytes)
        return RANS_ECORRUPT;
    if (reinterpret_cast<uintptr_t>(d_in) & 15)
        return RANS_EINVAL;
    DecodeArgs da;
    Header h;
    Layout layout;
    int rc = prepare_decode(table, d_in, in_len, static_cast<const uint8_t*>(h_header), d_out, cap,
                            &da, &h, &layout, d_lut, lut_w);
    if (rc != RANS_OK || h.n == 0)
        return rc;
    da.status = d_status;
    return enqueue_decode(da, h.p.radix_bits, h.p.sym_bytes, layout,
                          static_cast<hipStream_t>(stream)) == hipSuccess
               ? RANS_OK
               : RANS_EDEVICE;
}

// Shared body of the synchronous decodes (header read back, status read back).
static int decode_sync(const rans_table* table, const void* d_in, uint64_t in_len, void* d_out,
                       uint64_t cap, const void* d_lut, uint32_t lut_w, uint64_t* n_syms, void* stream)
{
    if (!table || !d_in || !n_syms)
        return RANS_EINVAL;
    *n_syms = 0;
    if (in_len < kHeaderBytes)
        return RANS_ECORRUPT;
    if (reinterpret_cast<uintptr_t>(d_in) & 15)
        return RANS_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Workspace* ws = workspace_for(st);
    if (!ws)
        return RANS_ENOMEM;
    std::lock_guard<std::mutex> lk(ws->mu);
    int rc = ws->reserve(256);
    if (rc != RANS_OK)
        return rc;
    if (hipMemcpyAsync(ws->host, d_in, kHeaderBytes, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return RANS_EDEVICE;
    uint8_t hdr[kHeaderBytes];
    std::memcpy(hdr, ws->host, kHeaderBytes);
    DecodeArgs da;
    Header h;
    Layout layout;
    rc = prepare_decode(table, d_in, in_len, hdr, d_out, cap, &da, &h, &layout, d_lut, lut_w);
    if (rc == RANS_OK || rc == RANS_ENOSPC)
        *n_syms = h.n;
    if (rc != RANS_OK || h.n == 0)
        return rc;
    uint8_t* base = static_cast<uint8_t*>(ws->dev);
    da.status = reinterpret_cast<int32_t*>(base);
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(base), 0, 1, st);
    if (e == hipSuccess)
        e = enqueue_decode(da, h.p.radix_bits, h.p.sym_bytes, layout, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws->host, base, 16, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e != hipSuccess)
        return RANS_EDEVICE;
    int32_t code;
    std::memcpy(&code, ws->host, 4);
    return code;
}

extern "C" int rans_decode_async(const rans_table* table, const void* d_in, uint64_t in_len,
                                 const void* h_header, void* d_syms, uint64_t syms_cap,
                                 int32_t* d_status, void* stream)
{
    return decode_async(table, d_in, in_len, h_header, d_syms, syms_cap, nullptr, 0, d_status, stream);
}

extern "C" int rans_decode(const rans_table* table, const void* d_in, uint64_t in_len, void* d_syms,
                           uint64_t syms_cap, uint64_t* n_syms, void* stream)
{
    return decode_sync(table, d_in, in_len, d_syms, syms_cap, nullptr, 0, n_syms, stream);
}

extern "C" int rans_decode_lut_async(const rans_table* table, const void* d_in, uint64_t in_len,
                                     const void* h_header, const void* d_lut, uint32_t lut_bytes,
                                     void* d_out, uint64_t out_cap, int32_t* d_status, void* stream)
{
    if (lut_bytes == 0)
        return RANS_EINVAL;
    return decode_async(table, d_in, in_len, h_header, d_out, out_cap, d_lut, lut_bytes, d_status,
                        stream);
}

extern "C" int rans_decode_lut(const rans_table* table, const void* d_in, uint64_t in_len,
                               const void* d_lut, uint32_t lut_bytes, void* d_out, uint64_t out_cap,
                               uint64_t* n_syms, void* stream)
{
    if (lut_bytes == 0)
        return RANS_EINVAL;
    return decode_sync(table, d_in, in_len, d_out, out_cap, d_lut, lut_bytes, n_syms, stream);
}
