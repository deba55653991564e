// Batched entry points: host validation of the job descriptors, workspace
// layout, and one HIP graph per launch image (captured on first use, then
// replayed: one graph launch per batch).  The job descriptors are the only
// per-call input; they are copied into the workspace ahead of the replay.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "rans_internal.h"
#include "timing.h"
#include "workspace.h"

namespace rans {
namespace {

std::mutex g_cfg_mu;
rans_batch_config g_cfg = {16, 1, 0, 1};

uint64_t up256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

int num_cus()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
        return 256;
    return v;
}

}  // namespace

uint32_t batch_chunks_per_item(const rans_params& p, bool decode, uint32_t G)
{
    // a wave codes 64 / N chunks (two with 32 coders per chunk)
    (void)decode;
    return G * (64u / p.interleave);
}

uint64_t batch_item_bound(const rans_job& jb, const rans_params& p, bool decode, uint32_t G)
{
    uint64_t nch;
    if (decode) {
        // a chunk costs at least a directory entry and N states: the same
        // bound the device's header check enforces, so no accepted job can
        // have more chunks than this
        const uint64_t per_chunk = uint64_t(kDirEntryBytes) + 4ull * p.interleave;
        nch = jb.in_len >= kHeaderBytes ? (jb.in_len - kHeaderBytes) / per_chunk : 0;
    } else {
        const uint64_t n = jb.in_len / p.sym_bytes;
        nch = p.chunk_syms ? (n + p.chunk_syms - 1) / p.chunk_syms : 0;
    }
    const uint32_t cpi = batch_chunks_per_item(p, decode, G);
    return (nch + cpi - 1) / cpi;
}

uint64_t batch_encode_scratch(uint64_t in_len, const rans_params& p)
{
    const uint64_t n = in_len / p.sym_bytes;
    const uint64_t nch = p.chunk_syms ? (n + p.chunk_syms - 1) / p.chunk_syms : 0;
    const uint64_t stride = slot_bytes_for(p.chunk_syms, p.prob_bits, p.radix_bits) + kSlotPad;
    return up256(nch * stride) + up256(8 * (nch + (nch + 63) / 64));
}

void bind_encode_scratch(BatchJob* jb, uint8_t* base, uint64_t in_len, const rans_params& p)
{
    const uint64_t n = in_len / p.sym_bytes;
    const uint64_t nch = p.chunk_syms ? (n + p.chunk_syms - 1) / p.chunk_syms : 0;
    const uint64_t stride = slot_bytes_for(p.chunk_syms, p.prob_bits, p.radix_bits) + kSlotPad;
    jb->slots = base;
    jb->lookback = reinterpret_cast<uint64_t*>(base + up256(nch * stride));
}

uint64_t batch_ctrl_bytes(uint32_t njobs, uint64_t max_items)
{
    return up256(256 + sizeof(BatchJob) * uint64_t(njobs)) + up256(4 * (max_items ? max_items : 1));
}

int plan_batch(const rans_job* jobs, uint32_t njobs, const rans_params* params, bool decode,
               const rans_batch_config& cfg, BatchPlan* plan)
{
    int rc = check_params(params);
    if (rc != RANS_OK)
        return rc;
    if (!jobs && njobs)
        return RANS_EINVAL;
    const rans_params& p = *params;
    const uint32_t w = p.sym_bytes, R = p.radix_bits;
    // the batched kernels code one chunk per wave: 32 or 64 coders per chunk, and
    // chunks must start 16-byte aligned in the symbol buffers
    if (p.interleave != 64 && p.interleave != 32)
        return RANS_EINVAL;
    if (p.escape)  // escape coding runs on the single-buffer entry points only
        return RANS_EINVAL;
    if (!decode && (p.chunk_syms == 0 || (uint64_t(p.chunk_syms) * w) % 16 != 0))
        return RANS_EINVAL;
    if (cfg.waves_per_group < 1 || cfg.waves_per_group > 16 || cfg.groups_per_cu < 1)
        return RANS_EINVAL;
    uint32_t G = cfg.waves_per_group;

    // host checks of every descriptor and the launch shape they imply
    uint64_t max_items = 0;
    uint32_t tab_lds = 0, sw = 0;
    Layout layout = kPacked;
    std::vector<BatchJob>& hj = plan->hj;
    hj.assign(njobs, BatchJob{});
    for (uint32_t j = 0; j < njobs; ++j) {
        const rans_job& jb = jobs[j];
        const DevTable* t = dev_table(jb.table);
        if (!t || t->k != p.prob_bits || !jb.d_out_len || !jb.d_status)
            return RANS_EINVAL;
        if ((jb.in_len && !jb.in) || (jb.out_cap && !jb.out) ||
            (reinterpret_cast<uintptr_t>(jb.in) & 15) || (reinterpret_cast<uintptr_t>(jb.out) & 15))
            return RANS_EINVAL;
        if (w == 1 && t->sym_w != 1)
            return RANS_EINVAL;
        if (j == 0)
            sw = t->sym_w;
        else if (t->sym_w != sw)
            return RANS_EINVAL;
        BatchJob& b = hj[j];
        b.in = static_cast<const uint8_t*>(jb.in);
        b.in_len = jb.in_len;
        b.out = static_cast<uint8_t*>(jb.out);
        b.out_cap = jb.out_cap;
        b.d_out_len = jb.d_out_len;
        b.d_status = jb.d_status;
        b.alphabet = t->alphabet;
        b.one = p.radix_bits == 8 && t->one_digit ? 1u : 0u;
        b.enc = t->enc;
        b.enc_bytes = static_cast<uint32_t>(t->enc_bytes);
        if (!decode) {
            if (jb.in_len % w)
                return RANS_EINVAL;
            if ((jb.in_len / w + p.chunk_syms - 1) / p.chunk_syms > 0xFFFFFFFFull)
                return RANS_EINVAL;
            const uint32_t el = enc_lds_bytes(b.enc_bytes, w);
            tab_lds = tab_lds > el ? tab_lds : el;
        }
    }
    if (decode) {
        // table layout: the configured one, or the best one every table has
        // (fused > packed > two-level) that fits LDS next to G waves' rings
        bool all_fused = true;
        uint64_t max_packed = 0, max_fused = 0;
        for (uint32_t j = 0; j < njobs; ++j) {
            const DevTable* t = dev_table(jobs[j].table);
            all_fused = all_fused && t->fused;
            max_packed = std::max<uint64_t>(max_packed, t->sym_bytes + t->dec_bytes);
            max_fused = std::max<uint64_t>(max_fused, t->fused_bytes);
        }
        // 256 bytes stay free for the persistent kernel's static LDS
        const uint64_t room_fused =
            uint64_t(max_lds_bytes()) - uint64_t(G) * decode_seg_lds_per_wave(kFused, p.interleave) - 256;
        const uint64_t room =
            uint64_t(max_lds_bytes()) - uint64_t(G) * decode_seg_lds_per_wave(kPacked, p.interleave) - 256;
        if (cfg.table_layout == 1)
            layout = kPacked;
        else if (cfg.table_layout == 2)
            layout = kTwoLevel;
        else if (cfg.table_layout == 3) {
            if (!all_fused)
                return RANS_EINVAL;
            layout = kFused;
        } else if (all_fused && max_fused <= room_fused)
            layout = kFused;
        else if (max_packed <= room && max_packed <= 96 * 1024)
            layout = kPacked;
        else
            layout = kTwoLevel;
        for (uint32_t j = 0; j < njobs; ++j) {
            const DevTable* t = dev_table(jobs[j].table);
            BatchJob& b = hj[j];
            if (layout == kFused) {
                b.tab_sym = nullptr;
                b.sym_bytes = 0;
                b.tab_ent = t->fused;
                b.ent_bytes = static_cast<uint32_t>(t->fused_bytes);
            } else if (layout == kPacked) {
                b.tab_sym = t->sym;
                b.sym_bytes = static_cast<uint32_t>(t->sym_bytes);
                b.tab_ent = t->dec;
                b.ent_bytes = static_cast<uint32_t>(t->dec_bytes);
            } else {
                b.tab_sym = t->sym;
                b.sym_bytes = static_cast<uint32_t>(t->sym_bytes);
                b.tab_ent = t->fc;
                b.ent_bytes = static_cast<uint32_t>(t->fc_bytes);
            }
            tab_lds = tab_lds > b.sym_bytes + b.ent_bytes ? tab_lds : b.sym_bytes + b.ent_bytes;
        }
    }
    // waves_per_group is a maximum: fewer waves per block when their rings
    // and the table do not fit LDS together
    const uint32_t per_wave = decode ? decode_seg_lds_per_wave(layout, p.interleave) : kEncWaveLdsBytes;
    while (G > 1 && uint64_t(tab_lds) + uint64_t(G) * per_wave + 256 > uint64_t(max_lds_bytes()))
        --G;
    if (uint64_t(tab_lds) + uint64_t(G) * per_wave + 256 > uint64_t(max_lds_bytes()))
        return RANS_EINVAL;
    for (uint32_t j = 0; j < njobs; ++j)
        max_items += batch_item_bound(jobs[j], p, decode, G);
    if (max_items > 0xFFFFFFF0ull)
        return RANS_EINVAL;

    const uint64_t slot_bytes = decode ? 0 : slot_bytes_for(p.chunk_syms, p.prob_bits, R);
    BatchArgs& a = plan->a;
    a = BatchArgs{};
    a.njobs = njobs;
    a.k = p.prob_bits;
    a.r = R;
    a.l = p.state_lbits;
    a.w = w;
    a.N = p.interleave;
    a.C = p.chunk_syms;
    a.bf = p.digit_order;
    a.G = G;
    a.cpi = batch_chunks_per_item(p, decode, G);
    a.max_items = static_cast<uint32_t>(max_items ? max_items : 1);
    a.slot_bytes = slot_bytes;
    a.slot_stride = decode ? 0 : slot_bytes + kSlotPad;
    a.tab_lds = (tab_lds + 15) & ~15u;
    a.grid = static_cast<uint32_t>(num_cus()) * cfg.groups_per_cu;
    plan->layout = layout;
    plan->sw = sw;
    plan->decode = decode;
    plan->ctrl_bytes = batch_ctrl_bytes(njobs, max_items);
    return RANS_OK;
}

int launch_planned(BatchPlan& plan, uint8_t* ctrl, void* pinned, hipStream_t st, bool use_graph,
                   Workspace* ws)
{
    BatchArgs& a = plan.a;
    if (a.njobs == 0)
        return RANS_OK;
    const bool decode = plan.decode;
    a.counter = reinterpret_cast<uint32_t*>(ctrl);  // counter + totals
    a.totals = a.counter + 4;
    a.jobs = reinterpret_cast<BatchJob*>(ctrl + 256);
    a.item_job = reinterpret_cast<uint32_t*>(ctrl + up256(256 + sizeof(BatchJob) * uint64_t(a.njobs)));

    // job descriptors -> pinned staging -> device, ordered on `st`
    const uint64_t jb_bytes = sizeof(BatchJob) * uint64_t(a.njobs);
    std::memcpy(pinned, plan.hj.data(), jb_bytes);
    if (hipMemcpyAsync(a.jobs, pinned, jb_bytes, hipMemcpyHostToDevice, st) != hipSuccess)
        return RANS_EDEVICE;

    const int R = static_cast<int>(a.r), W = static_cast<int>(a.w), SW = static_cast<int>(plan.sw);
    const int kind = decode ? RANS_KERNEL_BATCH_DECODE : RANS_KERNEL_BATCH_ENCODE;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cap) != hipSuccess)
        return RANS_EDEVICE;
    if (!use_graph || !ws || cap != hipStreamCaptureStatusNone) {
        TimingScope ts(kind, st);
        return launch_batch(a, decode, R, W, SW, plan.layout, a.grid, st) == hipSuccess ? RANS_OK
                                                                                       : RANS_EDEVICE;
    }
    // one graph per launch image: the kernel arguments and template choice
    std::string key(reinterpret_cast<const char*>(&a), sizeof(a));
    const int shape[5] = {decode ? 1 : 0, SW, static_cast<int>(plan.layout), static_cast<int>(a.grid), R};
    key.append(reinterpret_cast<const char*>(shape), sizeof(shape));
    auto it = ws->graphs.find(key);
    if (it == ws->graphs.end()) {
        if (!ws->capture && hipStreamCreateWithFlags(&ws->capture, hipStreamNonBlocking) != hipSuccess)
            return RANS_EDEVICE;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        if (hipStreamBeginCapture(ws->capture, hipStreamCaptureModeRelaxed) != hipSuccess)
            return RANS_EDEVICE;
        const hipError_t le = launch_batch(a, decode, R, W, SW, plan.layout, a.grid, ws->capture);
        const hipError_t ce = hipStreamEndCapture(ws->capture, &graph);
        if (le != hipSuccess || ce != hipSuccess || !graph) {
            if (graph)
                (void)hipGraphDestroy(graph);
            return RANS_EDEVICE;
        }
        const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess)
            return RANS_EDEVICE;
        it = ws->graphs.emplace(key, exec).first;
    }
    TimingScope ts(kind, st);
    return hipGraphLaunch(it->second, st) == hipSuccess ? RANS_OK : RANS_EDEVICE;
}

int run_batch(const rans_job* jobs, uint32_t njobs, const rans_params* params, hipStream_t st,
              bool decode, const rans_batch_config* cfg_override)
{
    rans_batch_config cfg;
    if (cfg_override) {
        cfg = *cfg_override;
    } else {
        std::lock_guard<std::mutex> lk(g_cfg_mu);
        cfg = g_cfg;
    }
    BatchPlan plan;
    int rc = plan_batch(jobs, njobs, params, decode, cfg, &plan);
    if (rc != RANS_OK || njobs == 0)
        return rc;
    // workspace: control region, then (encode) every job's slots and
    // placement words
    uint64_t need = plan.ctrl_bytes;
    if (!decode)
        for (uint32_t j = 0; j < njobs; ++j)
            need += batch_encode_scratch(jobs[j].in_len, *params);
    Workspace* ws = workspace_for(st);
    if (!ws)
        return RANS_ENOMEM;
    std::lock_guard<std::mutex> lk(ws->mu);
    if ((rc = ws->reserve(need)) != RANS_OK)
        return rc;
    if ((rc = ws->reserve_pinned(sizeof(BatchJob) * uint64_t(njobs))) != RANS_OK)
        return rc;
    uint8_t* base = static_cast<uint8_t*>(ws->dev);
    if (!decode) {
        uint64_t off = plan.ctrl_bytes;
        for (uint32_t j = 0; j < njobs; ++j) {
            bind_encode_scratch(&plan.hj[j], base + off, jobs[j].in_len, *params);
            off += batch_encode_scratch(jobs[j].in_len, *params);
        }
    }
    rc = launch_planned(plan, base, ws->pinned, st, cfg.use_graph != 0, ws);
    // the staging buffer is free again once the copy out of it has run
    if (!ws->staged && hipEventCreateWithFlags(&ws->staged, hipEventDisableTiming) != hipSuccess)
        return RANS_EDEVICE;
    if (hipEventRecord(ws->staged, st) != hipSuccess)
        return RANS_EDEVICE;
    ws->staged_pending = true;
    return rc;
}

rans_batch_config batch_config()
{
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    return g_cfg;
}

}  // namespace rans

using namespace rans;

extern "C" int rans_encode_batch(const rans_job* jobs, uint32_t njobs, const rans_params* params,
                                 void* stream)
{
    return run_batch(jobs, njobs, params, static_cast<hipStream_t>(stream), false, nullptr);
}

extern "C" int rans_decode_batch(const rans_job* jobs, uint32_t njobs, const rans_params* params,
                                 void* stream)
{
    return run_batch(jobs, njobs, params, static_cast<hipStream_t>(stream), true, nullptr);
}

extern "C" int rans_batch_set_config(const rans_batch_config* cfg)
{
    if (!cfg || cfg->waves_per_group < 1 || cfg->waves_per_group > 16 || cfg->groups_per_cu < 1 ||
        cfg->groups_per_cu > 16 || cfg->table_layout > 3)
        return RANS_EINVAL;
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    g_cfg = *cfg;
    return RANS_OK;
}

extern "C" int rans_batch_get_config(rans_batch_config* cfg)
{
    if (!cfg)
        return RANS_EINVAL;
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    *cfg = g_cfg;
    return RANS_OK;
}
