// Serving runtime: continuous batching of encode/decode requests under an
// HBM budget.
//
//  * The whole budget is one device allocation made at creation: every
//    stream's control region (job descriptors, work-item map, status words)
//    comes first, the rest is an arena from which each admitted request's
//    output (and, to encode, its digit slots and placement words) is carved
//    by a first-fit allocator.  The loop itself never calls the HIP
//    allocator, never synchronises a stream, and the device memory the server
//    holds is exactly its budget.
//  * Admission is FIFO: the oldest waiting request is admitted as soon as its
//    cost (input + output capacity + coding scratch) fits the remaining
//    budget; nothing overtakes it.
//  * Admitted requests are launched as soon as one of the server's streams
//    is idle: all admitted requests of one kind form one batched launch
//    (persistent kernel), so requests arriving while others run join the
//    next launch and run concurrently with them on another stream.
//  * Per-request status and output length are written by the kernels into a
//    per-stream device array, copied to pinned host memory behind the batch
//    on the same stream; completion is detected with hipEventQuery.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "rans_internal.h"
#include "workspace.h"

namespace rans {
namespace {

using Clock = std::chrono::steady_clock;

double us_since(Clock::time_point t0, Clock::time_point t1)
{
    return std::chrono::duration<double, std::micro>(t1 - t0).count();
}

// First-fit allocator of arena offsets in 256-byte units, coalescing frees.
class Arena {
public:
    void init(uint64_t bytes)
    {
        free_.clear();
        free_[0] = bytes;
    }
    bool alloc(uint64_t bytes, uint64_t* off)
    {
        bytes = (bytes + 255) & ~uint64_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const uint64_t rest = it->second - bytes;
                const uint64_t start = it->first + bytes;
                free_.erase(it);
                if (rest)
                    free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes)
    {
        bytes = (bytes + 255) & ~uint64_t(255);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

private:
    std::map<uint64_t, uint64_t> free_;
};

struct Request {
    uint64_t id = 0;
    int op = 0;  // RANS_OP_ENCODE / RANS_OP_DECODE
    const rans_table* table = nullptr;
    const void* d_in = nullptr;
    // out_alloc: arena bytes of the request (output, then encode scratch)
    uint64_t in_len = 0, out_cap = 0, out_alloc = 0, scratch = 0, cost = 0, out_off = 0;
    uint32_t slot = 0;  // index in its launch's status arrays
    Clock::time_point t_arrive, t_launch;
    bool admitted = false;
};

struct Lane {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;
    std::vector<Request*> reqs;
    uint8_t* ctrl = nullptr;      // control region of the lane's batched launches
    int32_t* d_status = nullptr;  // max_batch entries each, device
    uint64_t* d_len = nullptr;
    int32_t* h_status = nullptr;  // pinned copies
    uint64_t* h_len = nullptr;
    uint8_t* h_jobs = nullptr;    // pinned staging of job descriptors: encode half, decode half
};

}  // namespace
}  // namespace rans

struct rans_server {
    std::mutex mu;
    rans::Arena arena;
    uint8_t* mem = nullptr;   // the one device allocation (budget bytes)
    uint8_t* base = nullptr;  // the arena inside it
    uint64_t budget = 0, fixed = 0, used = 0, peak = 0;
    rans_params params{};
    rans_batch_config cfg{};  // launch shape of every batched launch
    uint32_t max_batch = 0;
    uint64_t ctrl_cap = 0;    // control bytes per lane
    uint64_t launches = 0, multi_launches = 0;
    uint32_t max_launch_reqs = 0, peak_busy = 0;
    std::vector<rans::Lane> lanes;
    std::deque<rans::Request*> waiting;
    std::vector<rans::Request*> ready;
    std::map<uint64_t, rans::Request*> live;  // admitted or waiting, by id
    std::vector<rans::Request*> done_keep;    // completed, output still held
    uint64_t next_id = 1;
    std::vector<rans_completion> finished;
};

namespace rans {
namespace {

uint64_t up256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

// What a request holds while admitted: its input (caller memory, counted
// against the budget all the same), its output and, to encode, the digit
// slots and placement words of its chunks (both in the arena).
uint64_t request_cost(uint64_t in_len, uint64_t out_alloc) { return up256(in_len) + up256(out_alloc); }

// Work items of one launch: at most max_batch requests whose inputs together
// fit the budget.
uint64_t lane_item_bound(const rans_params& p, uint64_t budget, uint32_t max_batch, uint32_t G)
{
    const uint64_t dec_chunks = budget / (uint64_t(kDirEntryBytes) + 4ull * p.interleave);
    const uint64_t enc_chunks = p.chunk_syms ? budget / (uint64_t(p.chunk_syms) * p.sym_bytes) : 0;
    return std::max(dec_chunks, enc_chunks) / G + 2ull * max_batch;
}

void launch_ready(rans_server* s, Lane& ln)
{
    std::vector<Request*> take;
    while (!s->ready.empty() && take.size() < s->max_batch) {
        take.push_back(s->ready.front());
        s->ready.erase(s->ready.begin());
    }
    if (take.empty())
        return;
    std::vector<rans_job> enc, dec;
    std::vector<Request*> encr, decr;
    const auto now = Clock::now();
    uint32_t slot = 0;
    for (Request* r : take) {
        r->slot = slot++;
        rans_job j{};
        j.table = r->table;
        j.in = r->d_in;
        j.in_len = r->in_len;
        j.out = s->base + r->out_off;
        j.out_cap = r->out_cap;
        j.d_out_len = ln.d_len + r->slot;
        j.d_status = ln.d_status + r->slot;
        r->t_launch = now;
        if (r->op == RANS_OP_ENCODE) {
            enc.push_back(j);
            encr.push_back(r);
        } else {
            dec.push_back(j);
            decr.push_back(r);
        }
    }
    // batch sizes vary from launch to launch: direct launches, no graphs.
    // Encode runs first, then decode, in stream order on the lane, so both
    // use the lane's control region; each stages through its own half of
    // the pinned buffer (both copies are queued before either runs).
    int rc = RANS_OK;
    const uint64_t half = sizeof(BatchJob) * uint64_t(s->max_batch);
    for (int pass = 0; pass < 2 && rc == RANS_OK; ++pass) {
        const bool decode = pass == 1;
        const std::vector<rans_job>& js = decode ? dec : enc;
        if (js.empty())
            continue;
        BatchPlan plan;
        rc = plan_batch(js.data(), static_cast<uint32_t>(js.size()), &s->params, decode, s->cfg, &plan);
        if (rc == RANS_OK && plan.ctrl_bytes > s->ctrl_cap)
            rc = RANS_EINVAL;  // cannot happen for admitted requests (bounded at creation)
        if (rc != RANS_OK)
            break;
        if (!decode)
            for (size_t i = 0; i < encr.size(); ++i)
                bind_encode_scratch(&plan.hj[i], s->base + encr[i]->out_off + up256(encr[i]->out_alloc - encr[i]->scratch),
                                    encr[i]->in_len, s->params);
        rc = launch_planned(plan, ln.ctrl, ln.h_jobs + (decode ? half : 0), ln.st, false, nullptr);
    }
    const uint32_t m = static_cast<uint32_t>(take.size());
    ++s->launches;
    if (m > 1)
        ++s->multi_launches;
    s->max_launch_reqs = std::max(s->max_launch_reqs, m);
    (void)hipMemcpyAsync(ln.h_status, ln.d_status, m * sizeof(int32_t), hipMemcpyDeviceToHost, ln.st);
    (void)hipMemcpyAsync(ln.h_len, ln.d_len, m * sizeof(uint64_t), hipMemcpyDeviceToHost, ln.st);
    (void)hipEventRecord(ln.ev, ln.st);
    if (rc != RANS_OK) {  // nothing was enqueued for some jobs: report the launch error
        (void)hipEventSynchronize(ln.ev);
        for (Request* r : take)
            ln.h_status[r->slot] = rc;
    }
    ln.busy = true;
    ln.reqs = take;
    uint32_t busy = 0;
    for (auto& l : s->lanes)
        busy += l.busy;
    s->peak_busy = std::max(s->peak_busy, busy);
}

void admit(rans_server* s)
{
    while (!s->waiting.empty()) {
        Request* r = s->waiting.front();
        if (s->used + r->cost > s->budget)  // used starts at the fixed control bytes
            break;
        if (!s->arena.alloc(r->out_alloc, &r->out_off))
            break;  // fragmentation: wait for releases
        s->waiting.pop_front();
        s->used += r->cost;
        s->peak = std::max(s->peak, s->used);
        r->admitted = true;
        s->ready.push_back(r);
    }
}

void collect(rans_server* s, Lane& ln, bool keep)
{
    const auto now = Clock::now();
    for (Request* r : ln.reqs) {
        rans_completion c{};
        c.id = r->id;
        c.status = ln.h_status[r->slot];
        c.out_len = ln.h_len[r->slot];
        c.d_out = s->base + r->out_off;
        c.latency_us = us_since(r->t_arrive, now);
        c.queue_us = us_since(r->t_arrive, r->t_launch);
        c.op = r->op;
        c.in_len = r->in_len;
        s->finished.push_back(c);
        if (keep) {
            s->done_keep.push_back(r);
        } else {
            s->arena.release(r->out_off, r->out_alloc);
            s->used -= r->cost;
            s->live.erase(r->id);
            delete r;
        }
    }
    ln.reqs.clear();
    ln.busy = false;
}

}  // namespace
}  // namespace rans

using namespace rans;

extern "C" int rans_server_create(const rans_server_config* cfg, rans_server** out)
{
    if (!cfg || !out || cfg->streams < 1 || cfg->streams > 16 || cfg->max_batch < 1 ||
        cfg->max_batch > (1u << 16) || cfg->hbm_budget < (1u << 20))
        return RANS_EINVAL;
    *out = nullptr;
    int rc = check_params(&cfg->params);
    if (rc != RANS_OK)
        return rc;
    if (cfg->params.escape)  // requests run on the batched kernels
        return RANS_EINVAL;
    if (cfg->params.interleave != 32 && cfg->params.interleave != 64)
        return RANS_EINVAL;
    rans_server* s = new rans_server();
    s->budget = cfg->hbm_budget;
    s->params = cfg->params;
    s->max_batch = cfg->max_batch;
    s->cfg = batch_config();  // fixed for the server's life: it sizes the control regions
    s->cfg.use_graph = 0;
    {
        // waves per block that fit next to the largest two-level table of
        // these parameters (a launch never runs with fewer, so the work-item
        // bound below holds)
        const uint32_t w = cfg->params.sym_bytes;
        const uint64_t tab = (uint64_t(1) << cfg->params.prob_bits) * w + 4ull * (w == 1 ? 256 : 4096) + 256;
        const uint64_t per = decode_seg_lds_per_wave(kTwoLevel, cfg->params.interleave);
        const uint64_t maxl = static_cast<uint64_t>(max_lds_bytes());
        const uint64_t fit = maxl > tab ? (maxl - tab) / per : 0;
        if (fit == 0) {
            delete s;
            return RANS_EINVAL;
        }
        s->cfg.waves_per_group = static_cast<uint32_t>(std::min<uint64_t>(s->cfg.waves_per_group, fit));
    }
    // per lane: the control region of a launch of max_batch requests whose
    // inputs fit the budget, then the status words
    s->ctrl_cap = batch_ctrl_bytes(cfg->max_batch,
                                   lane_item_bound(s->params, s->budget, cfg->max_batch, s->cfg.waves_per_group));
    const uint64_t per_lane = s->ctrl_cap + up256(16ull * cfg->max_batch);
    s->fixed = per_lane * cfg->streams;
    if (s->fixed + (1u << 16) > s->budget) {
        delete s;
        return RANS_ENOMEM;  // the budget does not even hold the control regions
    }
    void* mem = nullptr;
    if (hipMalloc(&mem, s->budget) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return RANS_ENOMEM;
    }
    s->mem = static_cast<uint8_t*>(mem);
    s->base = s->mem + s->fixed;
    s->arena.init(s->budget - s->fixed);
    s->used = s->peak = s->fixed;
    s->lanes.resize(cfg->streams);
    for (size_t i = 0; i < s->lanes.size(); ++i) {
        auto& ln = s->lanes[i];
        ln.ctrl = s->mem + i * per_lane;
        ln.d_len = reinterpret_cast<uint64_t*>(ln.ctrl + s->ctrl_cap);
        ln.d_status = reinterpret_cast<int32_t*>(ln.ctrl + s->ctrl_cap + 8ull * cfg->max_batch);
        if (hipStreamCreateWithFlags(&ln.st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ln.ev, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void**>(&ln.h_status), 4ull * cfg->max_batch,
                          hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void**>(&ln.h_len), 8ull * cfg->max_batch,
                          hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void**>(&ln.h_jobs), 2 * sizeof(BatchJob) * uint64_t(cfg->max_batch),
                          hipHostMallocDefault) != hipSuccess) {
            rans_server_destroy(s);
            return RANS_EDEVICE;
        }
    }
    *out = s;
    return RANS_OK;
}

extern "C" void rans_server_destroy(rans_server* s)
{
    if (!s)
        return;
    for (auto& ln : s->lanes) {
        if (ln.st)
            (void)hipStreamSynchronize(ln.st);
        if (ln.ev)
            (void)hipEventDestroy(ln.ev);
        if (ln.st)
            (void)hipStreamDestroy(ln.st);
        if (ln.h_status)
            (void)hipHostFree(ln.h_status);
        if (ln.h_len)
            (void)hipHostFree(ln.h_len);
        if (ln.h_jobs)
            (void)hipHostFree(ln.h_jobs);
    }
    for (auto& kv : s->live)
        delete kv.second;
    if (s->mem)
        (void)hipFree(s->mem);
    delete s;
}

extern "C" int rans_server_submit(rans_server* s, int op, const rans_table* table, const void* d_in,
                                  uint64_t in_len, uint64_t out_cap, uint64_t* id)
{
    if (!s || !table || !id || (op != RANS_OP_ENCODE && op != RANS_OP_DECODE) || (in_len && !d_in))
        return RANS_EINVAL;
    if (op == RANS_OP_ENCODE && in_len % s->params.sym_bytes)
        return RANS_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    Request* r = new Request();
    r->op = op;
    r->table = table;
    r->d_in = d_in;
    r->in_len = in_len;
    r->out_cap = out_cap;
    r->scratch = op == RANS_OP_ENCODE ? batch_encode_scratch(in_len, s->params) : 0;
    r->out_alloc = up256(out_cap ? out_cap : 16) + r->scratch;
    r->cost = request_cost(in_len, r->out_alloc);
    if (r->cost > s->budget - s->fixed) {
        delete r;
        return RANS_ENOMEM;
    }
    r->id = s->next_id++;
    r->t_arrive = Clock::now();
    s->waiting.push_back(r);
    s->live[r->id] = r;
    *id = r->id;
    return RANS_OK;
}

extern "C" int rans_server_poll(rans_server* s, int keep_outputs, rans_completion* out,
                                uint32_t max_out, uint32_t* n_out)
{
    if (!s || !n_out || (max_out && !out))
        return RANS_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto& ln : s->lanes) {
        if (ln.busy && hipEventQuery(ln.ev) == hipSuccess)
            collect(s, ln, keep_outputs != 0);
    }
    admit(s);
    for (auto& ln : s->lanes) {
        if (s->ready.empty())
            break;
        if (!ln.busy)
            launch_ready(s, ln);
    }
    const uint32_t n = static_cast<uint32_t>(std::min<size_t>(max_out, s->finished.size()));
    for (uint32_t i = 0; i < n; ++i)
        out[i] = s->finished[i];
    s->finished.erase(s->finished.begin(), s->finished.begin() + n);
    *n_out = n;
    return RANS_OK;
}

extern "C" int rans_server_release(rans_server* s, uint64_t id)
{
    if (!s)
        return RANS_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = std::find_if(s->done_keep.begin(), s->done_keep.end(),
                           [id](const Request* r) { return r->id == id; });
    if (it == s->done_keep.end())
        return RANS_EINVAL;
    Request* r = *it;
    s->done_keep.erase(it);
    s->arena.release(r->out_off, r->out_alloc);
    s->used -= r->cost;
    s->live.erase(r->id);
    delete r;
    return RANS_OK;
}

extern "C" int rans_server_stats(rans_server* s, rans_server_stats_t* st)
{
    if (!s || !st)
        return RANS_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    st->budget = s->budget;
    st->used = s->used;
    st->peak = s->peak;
    st->waiting = static_cast<uint32_t>(s->waiting.size());
    st->ready = static_cast<uint32_t>(s->ready.size());
    uint32_t busy = 0;
    for (auto& ln : s->lanes)
        busy += ln.busy;
    st->busy_streams = busy;
    st->peak_busy_streams = s->peak_busy;
    st->launches = s->launches;
    st->multi_request_launches = s->multi_launches;
    st->max_launch_requests = s->max_launch_reqs;
    st->fixed = s->fixed;
    return RANS_OK;
}

// Replays an arrival schedule (microseconds from the call) against the
// server and waits for every request; completions land in results[i] for
// request i.  Outputs are released as they complete unless keep_outputs.
extern "C" int rans_server_replay(rans_server* s, const rans_server_request* reqs, uint32_t n,
                                  int keep_outputs, rans_completion* results, double* makespan_us)
{
    if (!s || (n && (!reqs || !results)))
        return RANS_EINVAL;
    std::vector<uint64_t> ids(n, 0);
    std::map<uint64_t, uint32_t> index;
    const auto t0 = Clock::now();
    uint32_t submitted = 0, completed = 0;
    std::vector<rans_completion> buf(256);
    while (completed < n) {
        const double now = us_since(t0, Clock::now());
        while (submitted < n && reqs[submitted].arrival_us <= now) {
            const rans_server_request& q = reqs[submitted];
            uint64_t id = 0;
            int rc = rans_server_submit(s, q.op, q.table, q.d_in, q.in_len, q.out_cap, &id);
            if (rc != RANS_OK) {
                results[submitted] = rans_completion{};
                results[submitted].status = rc;
                ++completed;
            } else {
                // latency counts from the scheduled arrival
                std::lock_guard<std::mutex> lk(s->mu);
                s->live[id]->t_arrive = t0 + std::chrono::duration_cast<Clock::duration>(
                                                 std::chrono::duration<double, std::micro>(q.arrival_us));
                index[id] = submitted;
            }
            ++submitted;
        }
        uint32_t got = 0;
        int rc = rans_server_poll(s, keep_outputs, buf.data(), static_cast<uint32_t>(buf.size()), &got);
        if (rc != RANS_OK)
            return rc;
        for (uint32_t i = 0; i < got; ++i) {
            results[index[buf[i].id]] = buf[i];
            ++completed;
        }
        if (!got) {
            // nothing running, nothing launchable, everything arrived: the
            // waiting requests can never be admitted (outputs kept by the
            // caller hold the budget)
            rans_server_stats_t stt;
            rans_server_stats(s, &stt);
            if (submitted == n && stt.busy_streams == 0 && stt.ready == 0 && stt.waiting > 0)
                return RANS_ENOMEM;
            std::this_thread::yield();
        }
    }
    if (makespan_us)
        *makespan_us = us_since(t0, Clock::now());
    return RANS_OK;
}
