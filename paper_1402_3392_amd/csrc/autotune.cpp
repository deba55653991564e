// Autotuner for the batched path.  Two kinds of knobs:
//  * bitstream-visible, chosen at encode time: the chunk size C (smaller
//    chunks mean more independent waves but 256 bytes of states and 16 bytes
//    of directory per chunk);
//  * bitstream-invisible, chosen at decode time: waves per work item (the
//    lanes that work on one stream together: 64 per wave), persistent blocks
//    per CU, and the LDS table layout.
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
       << alpha_class << "|s" << size_class;
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
                t.encode_gbps >> t.decode_gbps >> t.use_graph &&
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
        << r.table_layout << ' ' << r.encode_gbps << ' ' << r.decode_gbps << ' ' << r.use_graph << '\n';
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

}  // namespace
}  // namespace rans

using namespace rans;

extern "C" int rans_autotune(const rans_table* table, const void* d_syms, uint64_t n_syms,
                             const rans_params* base, const char* cache_path, rans_tune_result* out)
{
    if (!table || !base || !out || (n_syms && !d_syms) || (reinterpret_cast<uintptr_t>(d_syms) & 15))
        return RANS_EINVAL;
    rans_params p = *base;
    p.interleave = 64;
    p.chunk_syms = 65536;
    int rc = check_params(&p);
    if (rc != RANS_OK)
        return rc;
    const DevTable* t = dev_table(table);
    if (t->k != p.prob_bits)
        return RANS_EINVAL;
    const uint32_t w = p.sym_bytes;
    const std::string key = cache_key(p, t->alphabet, n_syms * w);
    if (cache_lookup(cache_path, key, out)) {
        rans_batch_config cfg{out->waves_per_group, out->groups_per_cu, out->table_layout, out->use_graph};
        return rans_batch_set_config(&cfg);
    }
    if (n_syms == 0)
        return RANS_EINVAL;

    // one tuning stream per process (its library workspace stays cached)
    static hipStream_t st = nullptr;
    if (!st && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
        return RANS_EDEVICE;
    DevBuf cont, dec, meta;
    rans_params big = p;
    big.chunk_syms = 1024;  // the smallest candidate bounds every container
    const uint64_t cap = rans_encode_bound(n_syms, &big);
    if (!cont.alloc(cap) || !dec.alloc(n_syms * w) || !meta.alloc(64))
        return RANS_ENOMEM;
    uint64_t* d_len = static_cast<uint64_t*>(meta.p);
    int32_t* d_status = reinterpret_cast<int32_t*>(static_cast<uint8_t*>(meta.p) + 16);

    rans_batch_config base_cfg = batch_config();
    base_cfg.use_graph = 1;
    double best_score = 1e30, ref_bytes = 0;
    rans_tune_result best{};
    const uint32_t chunk_sizes[] = {65536, 32768, 16384, 8192, 4096};
    for (uint32_t C : chunk_sizes) {
        if ((uint64_t(C) * w) % 16 != 0)
            continue;
        rans_params pc = p;
        pc.chunk_syms = C;
        rans_job ej{table, d_syms, n_syms * w, cont.p, cap, d_len, d_status};
        int e = RANS_OK;
        const double enc_ms = time_ms(st, 5, [&] {
            return run_batch(&ej, 1, &pc, st, false, &base_cfg);
        }, &e);
        uint64_t clen = 0;
        int32_t cst = 0;
        (void)hipMemcpy(&clen, d_len, 8, hipMemcpyDeviceToHost);
        (void)hipMemcpy(&cst, d_status, 4, hipMemcpyDeviceToHost);
        if (e != RANS_OK || cst != RANS_OK)
            continue;
        if (ref_bytes == 0)
            ref_bytes = double(clen);
        // decode shapes for this container
        for (uint32_t G : {16u, 8u, 4u}) {
            for (uint32_t gpc : {1u, 2u}) {
                for (uint32_t lay : {3u, 1u, 2u}) {
                    rans_batch_config cfg{G, gpc, lay, 1};
                    rans_job dj{table, cont.p, clen, dec.p, n_syms * w, d_len, d_status};
                    int de = RANS_OK;
                    const double dec_ms = time_ms(st, 5, [&] {
                        return run_batch(&dj, 1, &pc, st, true, &cfg);
                    }, &de);
                    int32_t dst = 0;
                    (void)hipMemcpy(&dst, d_status, 4, hipMemcpyDeviceToHost);
                    if (de != RANS_OK || dst != RANS_OK)
                        continue;  // e.g. the layout does not fit LDS with G waves
                    // size overhead beyond 1% over the largest chunk counts as time
                    const double over = std::max(0.0, double(clen) / ref_bytes - 1.01);
                    const double score = (enc_ms + dec_ms) * (1.0 + 10.0 * over);
                    if (score < best_score) {
                        best_score = score;
                        best.chunk_syms = C;
                        best.waves_per_group = G;
                        best.groups_per_cu = gpc;
                        best.table_layout = lay;
                        best.encode_gbps = double(n_syms * w) / (enc_ms * 1e6);
                        best.decode_gbps = double(n_syms * w) / (dec_ms * 1e6);
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
        double t[2] = {0, 0};
        for (uint32_t g = 0; g < 2; ++g) {
            rans_batch_config cfg{best.waves_per_group, best.groups_per_cu, best.table_layout, g};
            rans_job ej{table, d_syms, n_syms * w, cont.p, cap, d_len, d_status};
            int e = RANS_OK;
            t[g] = time_ms(st, 5, [&] { return run_batch(&ej, 1, &pc, st, false, &cfg); }, &e);
            uint64_t clen = 0;
            (void)hipMemcpy(&clen, d_len, 8, hipMemcpyDeviceToHost);
            rans_job dj{table, cont.p, clen, dec.p, n_syms * w, d_len, d_status};
            t[g] += time_ms(st, 5, [&] { return run_batch(&dj, 1, &pc, st, true, &cfg); }, &e);
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
