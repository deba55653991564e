// Optional kernel timing: when enabled, each kernel launch the library makes
// is bracketed by two HIP events recorded on the launch stream.  Reading the
// totals waits for the recorded events.
#include <mutex>
#include <vector>

#include "timing.h"

namespace rans {

namespace {
struct Rec {
    int kind;
    hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t get_event()
{
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    // a device-scope release: a system-scope one (the default) writes the
    // caches back between the kernels being timed and slows the stream down
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventReleaseToDevice) != hipSuccess)
        return nullptr;
    return e;
}
}  // namespace

TimingScope::TimingScope(int kind, hipStream_t st, bool allowed) : kind_(kind), st_(st)
{
    if (!allowed)
        return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on)
        return;
    a_ = get_event();
    b_ = get_event();
    if (a_ && b_)
        (void)hipEventRecord(a_, st_);
}

TimingScope::~TimingScope()
{
    if (!a_ || !b_)
        return;
    std::lock_guard<std::mutex> lk(g_mu);
    (void)hipEventRecord(b_, st_);
    g_recs.push_back({kind_, a_, b_});
}

}  // namespace rans

using namespace rans;

extern "C" int rans_timing_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
    return RANS_OK;
}

extern "C" int rans_timing_reset(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& r : g_recs) {
        (void)hipEventSynchronize(r.b);
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.clear();
    return RANS_OK;
}

extern "C" int rans_timing_read(int kind, uint64_t* launches, double* total_ms)
{
    if (!launches || !total_ms)
        return RANS_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    uint64_t n = 0;
    double ms = 0;
    for (auto& r : g_recs) {
        if (r.kind != kind)
            continue;
        if (hipEventSynchronize(r.b) != hipSuccess)
            return RANS_EDEVICE;
        float t = 0;
        if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess)
            return RANS_EDEVICE;
        ms += t;
        ++n;
    }
    *launches = n;
    *total_ms = ms;
    return RANS_OK;
}
