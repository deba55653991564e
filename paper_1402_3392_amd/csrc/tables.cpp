// Static order-0 model: quantisation of counts to M = 2^k and the device
// tables the kernels stage into LDS.  The paper evaluates a static order-0
// model determined once per input (Section 7) and names rANS as the coder
// (Sections 2 and 7); the tables below serve its C and D functions.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "rans_internal.h"

struct rans_table {
    rans::DevTable dev;
    std::vector<uint32_t> freq;
    int device;
};

namespace rans {

// Integer largest-remainder quantiser (see rans_quantize in librans.h).
int quantize(const uint64_t* counts, uint32_t alphabet, uint32_t k, uint32_t* f)
{
    if (!counts || !f || alphabet == 0 || k < 1 || k > 16)
        return RANS_EINVAL;
    const uint64_t M = 1ull << k, lim = 1ull << 47;
    uint64_t total = 0, present = 0;
    for (uint32_t s = 0; s < alphabet; ++s) {
        if (counts[s] >= lim)
            return RANS_EINVAL;
        total += counts[s];
        present += counts[s] != 0;
    }
    if (total == 0 || total >= lim)
        return RANS_EINVAL;
    if (present > M)
        return RANS_EPREC;

    std::vector<uint64_t> rem(alphabet);
    std::vector<uint32_t> grow;  // present, not forced: candidates for +1
    uint64_t sum = 0;
    for (uint32_t s = 0; s < alphabet; ++s) {
        const uint64_t scaled = counts[s] * M;
        f[s] = static_cast<uint32_t>(scaled / total);
        rem[s] = scaled % total;
        if (counts[s] != 0) {
            if (f[s] == 0)
                f[s] = 1;  // forced
            else
                grow.push_back(s);
        }
        sum += f[s];
    }
    if (sum < M) {
        // index-ascending list, stable sort on remainder: ties keep index order
        std::stable_sort(grow.begin(), grow.end(),
                         [&](uint32_t a, uint32_t b) { return rem[a] > rem[b]; });
        const uint64_t need = M - sum;
        for (uint64_t t = 0; t < need && t < grow.size(); ++t)
            f[grow[t]] += 1;
    }
    while (sum > M) {
        uint32_t best = alphabet;
        for (uint32_t s = 0; s < alphabet; ++s)
            if (f[s] > 1 && (best == alphabet || f[s] > f[best]))
                best = s;
        f[best] -= 1;
        --sum;
    }
    return RANS_OK;
}

// Division constants for q = floor(x / f) with one 32-bit multiply-high
// (A. D. Robison, "N-bit unsigned division via N-bit multiply-add", ARITH
// 2005): q = mulhi(x + inc, m) >> sh.  For f = 2^t, t >= 1: m = 2^31,
// sh = t - 1, inc = 0 (exact for every 32-bit x).  f = 1: m = 2^32 - 1,
// inc = 1, sh = 0.  Otherwise, with t = floor(log2 f), m0 = floor(2^(32+t)
// / f) and r = 2^(32+t) - m0 f: the rounded-up multiplier m0 + 1 is exact
// when f - r <= 2^t, else the rounded-down m0 with the increment is (then
// r < 2^t); both for every x < 2^32 - 1.  The encoder's states stay below
// f 2^(l+r-k) <= 2^32, so only f = M = 2^k (a power of two >= 2) meets
// x = 2^32 - 1.
static void div_constants(uint32_t f, uint32_t* magic, uint32_t* inc, uint32_t* sh)
{
    uint32_t t = 0;
    while ((2ull << t) <= f)
        ++t;
    if (f == 1) {
        *magic = 0xFFFFFFFFu;
        *inc = 1;
        *sh = 0;
    } else if ((f & (f - 1)) == 0) {
        *magic = 1u << 31;
        *inc = 0;
        *sh = t - 1;
    } else {
        const uint64_t p = 1ull << (32 + t);
        const uint64_t m0 = p / f, r = p - m0 * f;
        const bool up = f - r <= (1ull << t);
        *magic = static_cast<uint32_t>(up ? m0 + 1 : m0);
        *inc = up ? 0 : 1;
        *sh = t;
    }
}

static inline uint32_t div_apply(uint32_t x, uint32_t magic, uint32_t inc, uint32_t sh)
{
    const uint32_t xi = x + inc;  // 32-bit, as on the device
    return static_cast<uint32_t>((static_cast<uint64_t>(magic) * xi) >> 32) >> sh;
}

static uint64_t pad16(uint64_t v) { return (v + 15) & ~uint64_t(15); }

// Canonical prefix code for the second coder family (Section 4's
// multiplexer): length max(1, ceil(log2(M / f_s))) for every symbol with
// f_s > 0 (the Kraft sum is at most sum f_s / M = 1, so a prefix code with
// these lengths exists, and no length exceeds k); codes canonical --
// symbols ordered by (length, index) take consecutive values, doubled at
// each length step.  enc[s] = code | len << 16 (len 0: not codable);
// dec[v] for the 2^maxlen values v of the next maxlen bits = symbol |
// len << 12 of the code that prefixes v (len 0 where none does).
static void prefix_code(const std::vector<uint32_t>& f, uint32_t k, std::vector<uint32_t>& enc,
                        std::vector<uint16_t>& dec, uint32_t* maxlen)
{
    const uint32_t n = static_cast<uint32_t>(f.size());
    const uint64_t M = 1ull << k;
    std::vector<uint32_t> len(n, 0);
    uint32_t ml = 0;
    for (uint32_t s = 0; s < n; ++s) {
        if (f[s] == 0)
            continue;
        uint32_t l = 0;
        while ((uint64_t(f[s]) << l) < M)
            ++l;
        len[s] = l < 1 ? 1 : l;
        ml = len[s] > ml ? len[s] : ml;
    }
    enc.assign(n + 1, 0);
    dec.assign(size_t(1) << ml, 0);
    uint32_t next = 0;
    for (uint32_t l = 1; l <= ml; ++l) {
        for (uint32_t s = 0; s < n; ++s) {
            if (len[s] != l)
                continue;
            enc[s] = next | (l << 16);
            // every ml-bit value that starts with this code decodes to s
            const uint32_t lo = next << (ml - l), cnt = 1u << (ml - l);
            for (uint32_t v = 0; v < cnt; ++v)
                dec[lo + v] = static_cast<uint16_t>(s | (l << 12));
            ++next;
        }
        next <<= 1;
    }
    *maxlen = ml;
}

const DevTable* dev_table(const rans_table* t) { return t ? &t->dev : nullptr; }

}  // namespace rans

using namespace rans;

extern "C" int rans_quantize(const uint64_t* counts, uint32_t alphabet, uint32_t prob_bits,
                             uint32_t* freqs_out)
{
    return quantize(counts, alphabet, prob_bits, freqs_out);
}

extern "C" int rans_tables_build(const uint64_t* counts, uint32_t alphabet, uint32_t prob_bits,
                                 rans_table** out)
{
    if (!out)
        return RANS_EINVAL;
    *out = nullptr;
    if (alphabet == 0 || alphabet > 65536 || prob_bits < 8 || prob_bits > 15)
        return RANS_EINVAL;
    const uint32_t k = prob_bits, M = 1u << k;
    std::vector<uint32_t> f(alphabet);
    int rc = quantize(counts, alphabet, k, f.data());
    if (rc != RANS_OK)
        return rc;

    const uint32_t sym_w = alphabet <= 256 ? 1 : 2;
    std::vector<uint32_t> cum(alphabet + 1, 0);
    for (uint32_t s = 0; s < alphabet; ++s)
        cum[s + 1] = cum[s] + f[s];

    DevTable d{};
    d.alphabet = alphabet;
    d.k = k;
    // with b = 2^8 a state needs a second digit in one step only for a
    // symbol with 0 < f < M / 256: after one digit it is below L, and L is
    // at most the symbol's bound f b L / M exactly when f >= M / 256
    d.one_digit = 1;
    for (uint32_t s = 0; s < alphabet; ++s)
        if (f[s] != 0 && f[s] < (M >> 8))
            d.one_digit = 0;
    d.sym_w = sym_w;
    d.dec_bytes = pad16(uint64_t(M) * 4);
    d.sym_bytes = pad16(uint64_t(M) * sym_w);
    d.fc_bytes = pad16(uint64_t(alphabet) * 4);
    d.enc_bytes = pad16(uint64_t(alphabet + 1) * 16);
    const bool fused = alphabet <= 256 && k <= 14;
    d.fused_bytes = fused ? uint64_t(M) * 8 : 0;
    // the prefix-code family (symbols fit the 12-bit field of its entries)
    std::vector<uint32_t> h_penc;
    std::vector<uint16_t> h_pdec;
    if (alphabet <= 4096) {
        prefix_code(f, k, h_penc, h_pdec, &d.pfx_maxlen);
        d.pfx_enc_bytes = pad16(h_penc.size() * 4);
        d.pfx_dec_bytes = pad16(h_pdec.size() * 2);
    }

    std::vector<uint8_t> h_dec(d.dec_bytes, 0), h_sym(d.sym_bytes, 0), h_fc(d.fc_bytes, 0),
        h_enc(d.enc_bytes, 0), h_fused(d.fused_bytes, 0);
    uint32_t* fz = reinterpret_cast<uint32_t*>(h_fused.data());
    uint32_t* dec = reinterpret_cast<uint32_t*>(h_dec.data());
    uint32_t* fc = reinterpret_cast<uint32_t*>(h_fc.data());
    uint32_t* enc = reinterpret_cast<uint32_t*>(h_enc.data());
    for (uint32_t s = 0; s < alphabet; ++s) {
        for (uint32_t slot = cum[s]; slot < cum[s + 1]; ++slot) {
            dec[slot] = (f[s] << 16) | (slot - cum[s]);
            if (fused) {
                fz[2 * slot] = slot - cum[s];
                fz[2 * slot + 1] = f[s] | (s << 24);
            }
            if (sym_w == 1)
                h_sym[slot] = static_cast<uint8_t>(s);
            else {
                h_sym[2 * slot] = static_cast<uint8_t>(s);
                h_sym[2 * slot + 1] = static_cast<uint8_t>(s >> 8);
            }
        }
        fc[s] = f[s] | (cum[s] << 16);
        uint32_t magic = 0, inc = 0, sh = 0;
        if (f[s] != 0)
            div_constants(f[s], &magic, &inc, &sh);
        enc[4 * s + 0] = magic;
        enc[4 * s + 1] = f[s] | (cum[s] << 16);
        enc[4 * s + 2] = inc | (sh << 8);
        enc[4 * s + 3] = M - f[s];
    }
    // entry `alphabet` stays all-zero: f = 0 marks "not encodable"

    rans_table* t = new (std::nothrow) rans_table();
    if (!t)
        return RANS_ENOMEM;
    t->freq = f;
    if (hipGetDevice(&t->device) != hipSuccess) {
        delete t;
        return RANS_EDEVICE;
    }
    void* blob = nullptr;
    const uint64_t base = d.dec_bytes + d.sym_bytes + d.fc_bytes + d.enc_bytes + d.fused_bytes;
    const uint64_t total = base + d.pfx_enc_bytes + d.pfx_dec_bytes;
    if (hipMalloc(&blob, total) != hipSuccess) {
        delete t;
        return RANS_ENOMEM;
    }
    uint8_t* p = static_cast<uint8_t*>(blob);
    d.dec = reinterpret_cast<uint32_t*>(p);
    d.sym = p + d.dec_bytes;
    d.fc = reinterpret_cast<uint32_t*>(p + d.dec_bytes + d.sym_bytes);
    d.enc = reinterpret_cast<uint4*>(p + d.dec_bytes + d.sym_bytes + d.fc_bytes);
    d.fused = fused ? reinterpret_cast<uint2*>(p + d.dec_bytes + d.sym_bytes + d.fc_bytes + d.enc_bytes)
                    : nullptr;
    std::vector<uint8_t> host(total);
    std::memcpy(host.data(), h_dec.data(), d.dec_bytes);
    std::memcpy(host.data() + d.dec_bytes, h_sym.data(), d.sym_bytes);
    std::memcpy(host.data() + d.dec_bytes + d.sym_bytes, h_fc.data(), d.fc_bytes);
    std::memcpy(host.data() + d.dec_bytes + d.sym_bytes + d.fc_bytes, h_enc.data(),
                d.enc_bytes);
    if (fused)
        std::memcpy(host.data() + d.dec_bytes + d.sym_bytes + d.fc_bytes + d.enc_bytes,
                    h_fused.data(), d.fused_bytes);
    if (d.pfx_enc_bytes) {
        d.pfx_enc = reinterpret_cast<uint32_t*>(p + base);
        d.pfx_dec = reinterpret_cast<uint16_t*>(p + base + d.pfx_enc_bytes);
        std::memcpy(host.data() + base, h_penc.data(), h_penc.size() * 4);
        std::memcpy(host.data() + base + d.pfx_enc_bytes, h_pdec.data(), h_pdec.size() * 2);
    }
    if (hipMemcpy(blob, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(blob);
        delete t;
        return RANS_EDEVICE;
    }
    t->dev = d;
    *out = t;
    return RANS_OK;
}

extern "C" int rans_table_freqs(const rans_table* table, uint32_t* freqs_out)
{
    if (!table || !freqs_out)
        return RANS_EINVAL;
    std::memcpy(freqs_out, table->freq.data(), table->freq.size() * sizeof(uint32_t));
    return RANS_OK;
}

extern "C" uint32_t rans_table_alphabet(const rans_table* table)
{
    return table ? table->dev.alphabet : 0;
}

extern "C" uint32_t rans_table_prob_bits(const rans_table* table)
{
    return table ? table->dev.k : 0;
}

extern "C" void rans_table_destroy(rans_table* table)
{
    if (!table)
        return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(table->device);
    (void)hipFree(table->dev.dec);  // start of the single allocation
    (void)hipSetDevice(cur);
    delete table;
}

// Host-side check of the division constants (not part of the C ABI header):
// for every f in [1, fmax] compares mulhi(x + inc, m) >> sh with x / f at
// the ends of the domain (x = 2^32 - 1 only for powers of two >= 2), around
// multiples of f and at `samples` pseudo-random x.  Returns the number of
// mismatches.
extern "C" uint64_t rans_internal_check_division(uint32_t fmax, uint32_t samples)
{
    uint64_t bad = 0, seed = 0x9E3779B97F4A7C15ull;
    for (uint32_t f = 1; f <= fmax; ++f) {
        uint32_t magic, inc, sh;
        div_constants(f, &magic, &inc, &sh);
        const bool full = f >= 2 && (f & (f - 1)) == 0;
        auto chk = [&](uint32_t x) {
            if (x != 0xFFFFFFFFu || full)
                bad += div_apply(x, magic, inc, sh) != x / f;
        };
        chk(0);
        chk(0xFFFFFFFFu);
        chk(0xFFFFFFFEu);
        chk(0xFFFFFFFEu - f);
        for (uint64_t m = f; m < (1ull << 32); m += (uint64_t(f) << 12) + f) {
            chk(static_cast<uint32_t>(m));
            chk(static_cast<uint32_t>(m - 1));
        }
        for (uint32_t i = 0; i < samples; ++i) {
            seed ^= seed << 13;
            seed ^= seed >> 7;
            seed ^= seed << 17;
            chk(static_cast<uint32_t>(seed));
        }
    }
    return bad;
}
