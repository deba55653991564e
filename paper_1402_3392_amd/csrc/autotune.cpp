// Autotuner for the batched path.  Two kinds of knobs:
//  * bitstream-visible, chosen at encode time: the interleave factor N (32
//    or 64 coders per chunk, i.e. lanes per stream: a decoding wave codes
//    64 / N chunks at once) and the chunk size C (smaller chunks mean more
//    independent waves but 4N bytes of states and 16 bytes of directory per
//    chunk);
//  * bitstream-invisible, chosen at decode time: waves per work item,
//    persistent blocks per CU, and the LDS table layout.
// Every candidate is timed on the caller's sample with the real batched
// kernels (median of a few runs, HIP events on a private stream).  Results
// are cached in a text file keyed by device, parameters, alphabet class and
// size class.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "rans_internal.h"
#include "workspace.h"

namespace rans {
namespace {

struct DevBuf {
    void* p = nullptr;
    ~DevBuf()
    {
        if (p)
            (void)hipFree(p);
    }
    bool alloc(uint64_t n) { return hipMalloc(&p, n ? n : 16) == hipSuccess; }
};

std::string cache_key(const rans_params& p, uint32_t alphabet, uint64_t bytes)
{
    int dev = 0;
    hipDeviceProp_t prop{};
    (void)hipGetDevice(&dev);
    (void)hipGetDeviceProperties(&prop, dev);
    uint32_t size_class = 0;
    while ((1ull << (size_class + 1)) <= bytes)
        ++size_class;
    uint32_t alpha_class = 0;
    while ((1u << alpha_class) < alphabet)
        ++alpha_class;
    std::ostringstream os;
    os << prop.gcnArchName << "|k" << int(p.prob_bits) << "|r" << int(p.radix_bits) << "|l"
       << int(p.state_lbits) << "|w" << int(p.sym_bytes) << "|o" << int(p.digit_order) << "|a"
       << alpha_class << "|s" << size_class << "|n" << int(p.interleave);
    std::string k = os.str();
    std::replace(k.begin(), k.end(), ' ', '_');
    return k;
}

bool cache_lookup(const char* path, const std::string& key, rans_tune_result* r)
{
    if (!path || !*path)
        return false;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        std::istringstream is(line);
        std::string k;
        rans_tune_result t{};
        if (is >> k >> t.chunk_syms >> t.waves_per_group >> t.groups_per_cu >> t.table_layout >>
                t.encode_gbps >> t.decode_gbps >> t.use_graph >> t.interleave >> t.lanes_per_stream >>
                t.chunks_per_wave &&
            k == key) {
            *r = t;
            return true;
        }
    }
    return false;
}

void cache_store(const char* path, const std::string& key, const rans_tune_result& r)
{
    if (!path || !*path)
        return;
    std::ofstream out(path, std::ios::app);
    out << key << ' ' << r.chunk_syms << ' ' << r.waves_per_group << ' ' << r.groups_per_cu << ' '
        << r.table_layout << ' ' << r.encode_gbps << ' ' << r.decode_gbps << ' ' << r.use_graph << ' '
        << r.interleave << ' ' << r.lanes_per_stream << ' ' << r.chunks_per_wave << '\n';
}

// Median time (ms) of `reps` runs of fn() on stream st.
template <typename F>
double time_ms(hipStream_t st, int reps, F fn, int* rc)
{
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    std::vector<double> ts;
    *rc = fn();  // warm-up (also captures the graph)
    for (int i = 0; i < reps && *rc == RANS_OK; ++i) {
        (void)hipEventRecord(a, st);
        *rc = fn();
        (void)hipEventRecord(b, st);
        (void)hipEventSynchronize(b);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, a, b);
        ts.push_back(ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (ts.empty())
        return 1e30;
    std::sort(ts.begin(), ts.end());
    return ts[ts.size() / 2];
}

// One stream of a tuning sample: symbols on the device, coded with table.
struct Sample {
    const rans_table* table;
    const void* d_syms;
    uint64_t n;  // symbols
};

// The search shared by both entry points: every chunk size, then every
// decode shape for its containers, each timed on the whole sample with the
// batched kernels; finally graph replay against direct launches for the
// best shape.  Applies the winner as the process-wide batch config.
int tune(const std::vector<Sample>& smp, const rans_params& p, const std::string& key,
         const char* cache_path, rans_tune_result* out)
{
    const uint32_t w = p.sym_bytes;
    const uint32_t nj = static_cast<uint32_t>(smp.size());
    // one tuning stream per process (its library workspace stays cached)
    static hipStream_t st = nullptr;
    if (!st && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
        return RANS_EDEVICE;
    rans_params small = p;
    small.chunk_syms = 4096;  // the smallest candidate with 64 coders bounds every container
    small.interleave = 64;
    std::vector<uint64_t> cap(nj), coff(nj), doff(nj);
    uint64_t ctot = 0, dtot = 0, total = 0;
    for (uint32_t j = 0; j < nj; ++j) {
        cap[j] = rans_encode_bound(smp[j].n, &small);
        coff[j] = ctot;
        ctot += (cap[j] + 255) & ~uint64_t(255);
        doff[j] = dtot;
        dtot += (smp[j].n * w + 255) & ~uint64_t(255);
        total += smp[j].n * w;
    }
    DevBuf cont, dec, meta;
    if (!cont.alloc(ctot) || !dec.alloc(dtot) || !meta.alloc(16ull * nj))
        return RANS_ENOMEM;
    uint64_t* d_len = static_cast<uint64_t*>(meta.p);
    int32_t* d_status = reinterpret_cast<int32_t*>(static_cast<uint8_t*>(meta.p) + 8ull * nj);
    std::vector<rans_job> ej(nj), dj(nj);
    for (uint32_t j = 0; j < nj; ++j) {
        ej[j] = rans_job{smp[j].table, smp[j].d_syms, smp[j].n * w,
                         static_cast<uint8_t*>(cont.p) + coff[j], cap[j], d_len + j, d_status + j};
        dj[j] = rans_job{smp[j].table, static_cast<uint8_t*>(cont.p) + coff[j], 0,
                         static_cast<uint8_t*>(dec.p) + doff[j], smp[j].n * w, d_len + j, d_status + j};
    }
    std::vector<uint64_t> clen(nj);
    std::vector<int32_t> cst(nj);
    auto statuses_ok = [&](bool lengths) {
        (void)hipMemcpy(cst.data(), d_status, 4ull * nj, hipMemcpyDeviceToHost);
        for (int32_t v : cst)
            if (v != RANS_OK)
                return false;
        if (lengths)
            (void)hipMemcpy(clen.data(), d_len, 8ull * nj, hipMemcpyDeviceToHost);
        return true;
    };

    rans_batch_config base_cfg = batch_config();
    base_cfg.use_graph = 1;
    double best_score = 1e30, ref_bytes = 0;
    rans_tune_result best{};
    const uint32_t chunk_sizes[] = {65536, 32768, 16384, 8192, 4096};
    // the caller's interleave factor, or both when it leaves it open (0)
    std::vector<uint32_t> interleaves;
    if (p.interleave)
        interleaves.push_back(p.interleave);
    else
        interleaves = {64, 32};
    for (uint32_t N : interleaves)
    for (uint32_t C : chunk_sizes) {
        if ((uint64_t(C) * w) % 16 != 0)
            continue;
        rans_params pc = p;
        pc.chunk_syms = C;
        pc.interleave = static_cast<uint16_t>(N);
        int e = RANS_OK;
        const double enc_ms = time_ms(st, 5, [&] {
            return run_batch(ej.data(), nj, &pc, st, false, &base_cfg);
        }, &e);
        if (e != RANS_OK || !statuses_ok(true))
            continue;
        double bytes = 0;
        for (uint32_t j = 0; j < nj; ++j) {
            dj[j].in_len = clen[j];
            bytes += double(clen[j]);
        }
        if (ref_bytes == 0)
            ref_bytes = bytes;  // the first candidate: the largest chunks (and N = 64 when open)
        // decode shapes for these containers
        for (uint32_t G : {16u, 8u, 4u}) {
            for (uint32_t gpc : {1u, 2u, 4u}) {
                for (uint32_t lay : {3u, 1u, 2u}) {
                    rans_batch_config cfg{G, gpc, lay, 1};
                    int de = RANS_OK;
                    const double dec_ms = time_ms(st, 5, [&] {
                        return run_batch(dj.data(), nj, &pc, st, true, &cfg);
                    }, &de);
                    if (de != RANS_OK || !statuses_ok(false))
                        continue;  // e.g. the layout does not fit LDS with G waves
                    // size overhead beyond 1% over the largest chunks counts as time
                    const double over = std::max(0.0, bytes / ref_bytes - 1.01);
                    const double score = (enc_ms + dec_ms) * (1.0 + 10.0 * over);
                    if (score < best_score) {
                        best_score = score;
                        best.chunk_syms = C;
                        best.interleave = N;
                        best.lanes_per_stream = N;
                        best.chunks_per_wave = 64 / N;
                        best.waves_per_group = G;
                        best.groups_per_cu = gpc;
                        best.table_layout = lay;
                        best.encode_gbps = double(total) / (enc_ms * 1e6);
                        best.decode_gbps = double(total) / (dec_ms * 1e6);
                    }
                }
            }
        }
    }
    if (best.chunk_syms == 0)
        return RANS_EDEVICE;
    // graph replay against direct launches, for the best shape
    {
        rans_params pc = p;
        pc.chunk_syms = best.chunk_syms;
        pc.interleave = static_cast<uint16_t>(best.interleave);
        double t[2] = {0, 0};
        for (uint32_t g = 0; g < 2; ++g) {
            rans_batch_config cfg{best.waves_per_group, best.groups_per_cu, best.table_layout, g};
            int e = RANS_OK;
            t[g] = time_ms(st, 5, [&] { return run_batch(ej.data(), nj, &pc, st, false, &cfg); }, &e);
            if (e == RANS_OK && statuses_ok(true)) {
                for (uint32_t j = 0; j < nj; ++j)
                    dj[j].in_len = clen[j];
                t[g] += time_ms(st, 5, [&] { return run_batch(dj.data(), nj, &pc, st, true, &cfg); }, &e);
            }
            if (e != RANS_OK)
                t[g] = 1e30;
        }
        best.use_graph = t[1] <= t[0] ? 1u : 0u;
    }
    (void)hipStreamSynchronize(st);
    *out = best;
    cache_store(cache_path, key, best);
    rans_batch_config cfg{best.waves_per_group, best.groups_per_cu, best.table_layout, best.use_graph};
    return rans_batch_set_config(&cfg);
}

}  // namespace
}  // namespace rans

using namespace rans;

extern "C" int rans_autotune(const rans_table* table, const void* d_syms, uint64_t n_syms,
                             const rans_params* base, const char* cache_path, rans_tune_result* out)
{
    if (!table || !base || !out || (n_syms && !d_syms) || (reinterpret_cast<uintptr_t>(d_syms) & 15))
        return RANS_EINVAL;
    rans_params p = *base;
    if (p.interleave != 0 && p.interleave != 32 && p.interleave != 64)
        return RANS_EINVAL;
    const uint16_t n_fixed = p.interleave;  // 0: searched over 32 and 64
    p.interleave = 64;
    p.chunk_syms = 65536;
    int rc = check_params(&p);
    if (rc != RANS_OK)
        return rc;
    p.interleave = n_fixed;
    const DevTable* t = dev_table(table);
    if (t->k != p.prob_bits)
        return RANS_EINVAL;
    const std::string key = cache_key(p, t->alphabet, n_syms * p.sym_bytes);
    if (cache_lookup(cache_path, key, out)) {
        rans_batch_config cfg{out->waves_per_group, out->groups_per_cu, out->table_layout, out->use_graph};
        return rans_batch_set_config(&cfg);
    }
    if (n_syms == 0)
        return RANS_EINVAL;
    return tune({Sample{table, d_syms, n_syms}}, p, key, cache_path, out);
}

extern "C" int rans_autotune_batch(const rans_job* jobs, uint32_t njobs, const rans_params* base,
                                   const char* cache_path, rans_tune_result* out)
{
    if (!jobs || njobs == 0 || !base || !out)
        return RANS_EINVAL;
    rans_params p = *base;
    if (p.interleave != 0 && p.interleave != 32 && p.interleave != 64)
        return RANS_EINVAL;
    const uint16_t n_fixed = p.interleave;  // 0: searched over 32 and 64
    p.interleave = 64;
    p.chunk_syms = 65536;
    int rc = check_params(&p);
    if (rc != RANS_OK)
        return rc;
    p.interleave = n_fixed;
    std::vector<Sample> smp;
    uint64_t total = 0;
    uint32_t alpha = 0;
    for (uint32_t j = 0; j < njobs; ++j) {
        const rans_job& jb = jobs[j];
        const DevTable* t = dev_table(jb.table);
        if (!t || t->k != p.prob_bits || (jb.in_len % p.sym_bytes) != 0 ||
            (jb.in_len && !jb.in) || (reinterpret_cast<uintptr_t>(jb.in) & 15))
            return RANS_EINVAL;
        if (jb.in_len == 0)
            continue;
        smp.push_back(Sample{jb.table, jb.in, jb.in_len / p.sym_bytes});
        total += jb.in_len;
        alpha = std::max(alpha, t->alphabet);
    }
    if (smp.empty())
        return RANS_EINVAL;
    // the key adds the number of streams (its power-of-two class)
    uint32_t nclass = 0;
    while ((1u << (nclass + 1)) <= smp.size())
        ++nclass;
    const std::string key = cache_key(p, alpha, total) + "|j" + std::to_string(nclass);
    if (cache_lookup(cache_path, key, out)) {
        rans_batch_config cfg{out->waves_per_group, out->groups_per_cu, out->table_layout, out->use_graph};
        return rans_batch_set_config(&cfg);
    }
    return tune(smp, p, key, cache_path, out);
}
