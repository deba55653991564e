#include "workspace.h"

#include <map>
#include <utility>

namespace rans {

static std::mutex g_mu;
static std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;

Workspace* workspace_for(hipStream_t stream)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_pair(dev, stream);
    auto it = g_ws.find(key);
    if (it != g_ws.end())
        return it->second;
    Workspace* w = new Workspace();
    w->device = dev;
    w->stream = stream;
    if (hipHostMalloc(&w->host, 4096, hipHostMallocDefault) != hipSuccess) {
        delete w;
        return nullptr;
    }
    g_ws[key] = w;
    return w;
}

void release_workspace(hipStream_t stream)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return;
    Workspace* w = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_ws.find(std::make_pair(dev, stream));
        if (it == g_ws.end())
            return;
        w = it->second;
        g_ws.erase(it);
    }
    {
        // no call holds it any more once it is out of the map and its lock
        // has been taken once
        std::lock_guard<std::mutex> lk(w->mu);
        (void)hipStreamSynchronize(stream);
        w->drop_graphs();
        if (w->dev)
            (void)hipFree(w->dev);
        if (w->pinned)
            (void)hipHostFree(w->pinned);
        if (w->host)
            (void)hipHostFree(w->host);
        if (w->staged)
            (void)hipEventDestroy(w->staged);
        if (w->capture)
            (void)hipStreamDestroy(w->capture);
    }
    delete w;
}

void Workspace::drop_graphs()
{
    for (auto& g : graphs)
        (void)hipGraphExecDestroy(g.second);
    graphs.clear();
}

int Workspace::reserve_pinned(uint64_t need)
{
    if (staged_pending) {
        if (hipEventSynchronize(staged) != hipSuccess)
            return RANS_EDEVICE;
        staged_pending = false;
    }
    if (need <= pinned_bytes)
        return RANS_OK;
    if (pinned)
        (void)hipHostFree(pinned);
    pinned = nullptr;
    pinned_bytes = 0;
    const uint64_t want = need + need / 2 + 4096;
    if (hipHostMalloc(&pinned, want, hipHostMallocDefault) != hipSuccess) {
        pinned = nullptr;
        return RANS_ENOMEM;
    }
    pinned_bytes = want;
    return RANS_OK;
}

int Workspace::reserve(uint64_t need)
{
    if (need <= bytes)
        return RANS_OK;
    if (dev) {
        if (hipStreamSynchronize(stream) != hipSuccess)
            return RANS_EDEVICE;
        drop_graphs();  // they hold pointers into the old buffer
        (void)hipFree(dev);
        dev = nullptr;
        bytes = 0;
    }
    // grow geometrically so that a sequence of slightly larger calls does
    // not reallocate every time
    uint64_t want = need + need / 4;
    if (hipMalloc(&dev, want) != hipSuccess) {
        dev = nullptr;
        if (hipMalloc(&dev, need) != hipSuccess) {
            dev = nullptr;
            (void)hipGetLastError();
            return RANS_ENOMEM;
        }
        want = need;
    }
    bytes = want;
    return RANS_OK;
}

static uint64_t up256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

EncodeLayout encode_layout(uint64_t n_chunks, uint32_t N, uint64_t slot_bytes)
{
    EncodeLayout l;
    l.flags = 0;
    l.ndig = 256;
    l.chunk_off = up256(l.ndig + 4 * n_chunks);
    l.states = up256(l.chunk_off + 8 * n_chunks);
    l.slots = up256(l.states + 4ull * N * n_chunks);
    l.lookback = up256(l.slots + (slot_bytes + kSlotPad) * n_chunks);
    l.total = up256(l.lookback + 8 * (n_chunks + (n_chunks + 63) / 64 + 1));
    return l;
}

}  // namespace rans

extern "C" int rans_workspace_release(void* stream)
{
    rans::release_workspace(static_cast<hipStream_t>(stream));
    return RANS_OK;
}
