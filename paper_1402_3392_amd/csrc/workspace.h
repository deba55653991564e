// Per-(device, stream) device workspace and host-side helpers shared by the
// single-buffer and batched entry points.
#pragma once

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "rans_internal.h"

namespace rans {

// Device scratch owned by the library, one per (device, HIP stream), so that
// calls on different streams never share scratch.  Grows on demand; growth
// waits for the stream first, since earlier work may still use the old
// buffer.  `host` is a small pinned buffer for status read-back.
struct Workspace {
    std::mutex mu;
    int device = 0;
    hipStream_t stream = nullptr;
    void* dev = nullptr;
    uint64_t bytes = 0;
    void* host = nullptr;  // 4 KiB pinned
    // batched calls: pinned staging for job descriptors, the event that says
    // the last copy out of it has finished, captured graphs by launch image
    void* pinned = nullptr;
    uint64_t pinned_bytes = 0;
    hipEvent_t staged = nullptr;
    bool staged_pending = false;
    hipStream_t capture = nullptr;
    std::map<std::string, hipGraphExec_t> graphs;
    int reserve(uint64_t need);
    int reserve_pinned(uint64_t need);
    void drop_graphs();
};

Workspace* workspace_for(hipStream_t stream);

struct Header {
    rans_params p;
    uint64_t n;
    uint32_t n_chunks;
    bool pfx;  // the prefix-code family (header flags 4)
};

// Byte offsets inside the workspace for one encode call.
struct EncodeLayout {
    uint64_t flags;      // 32 B: i32 status, pad, u64 container length
    uint64_t ndig;       // n_chunks u32
    uint64_t chunk_off;  // n_chunks u64
    uint64_t states;     // n_chunks * N u32
    uint64_t slots;      // n_chunks * slot_stride
    uint64_t lookback;   // n_chunks + ceil(n_chunks / 64) u64 (in-kernel placement), then the
                         // u64 whose low half is the start ticket (one fill clears all)
    uint64_t total;
};

EncodeLayout encode_layout(uint64_t n_chunks, uint32_t N, uint64_t slot_bytes);

int check_params(const rans_params* p);
uint32_t log2u(uint32_t v);
uint32_t max_digits(uint32_t k, uint32_t r);
uint32_t raw_digits(uint32_t r);
uint64_t slot_bytes_for(uint32_t C, uint32_t k, uint32_t r, bool esc = false);
void make_header(uint8_t* h, const rans_params& p, uint32_t C, uint64_t n, uint32_t nch);
int parse_header(const uint8_t* h, uint64_t in_len, Header* out);
bool choose_layout(const DevTable& t, Layout* layout, uint32_t* lds, uint32_t extra = 0,
                   uint32_t seg_n = 0);
int run_batch(const rans_job* jobs, uint32_t njobs, const rans_params* params, hipStream_t st,
              bool decode, const rans_batch_config* cfg_override);

// A batched launch planned on the host: validated job descriptors and the
// launch shape.  Its device memory is bound by the caller: a control region
// of ctrl_bytes (counter, job array, item map) and, to encode, each job's
// scratch (batch_encode_scratch bytes, bound with bind_encode_scratch).
struct BatchPlan {
    BatchArgs a{};
    std::vector<BatchJob> hj;
    Layout layout = kPacked;
    uint32_t sw = 1;
    bool decode = false;
    uint64_t ctrl_bytes = 0;
};
int plan_batch(const rans_job* jobs, uint32_t njobs, const rans_params* params, bool decode,
               const rans_batch_config& cfg, BatchPlan* plan);
// Chunks one work item covers: waves per block times chunks per wave.
uint32_t batch_chunks_per_item(const rans_params& p, bool decode, uint32_t G);
// Work items job `jb` can take at most (decode: from its container length).
uint64_t batch_item_bound(const rans_job& jb, const rans_params& p, bool decode, uint32_t G);
// Control bytes of a launch of njobs jobs and max_items work items.
uint64_t batch_ctrl_bytes(uint32_t njobs, uint64_t max_items);
// Encode scratch of one job of in_len symbol bytes: its digit slots and
// placement words (256-byte aligned parts).
uint64_t batch_encode_scratch(uint64_t in_len, const rans_params& p);
void bind_encode_scratch(BatchJob* jb, uint8_t* base, uint64_t in_len, const rans_params& p);
// Copies the job descriptors through `pinned` (host, pinned, free to
// overwrite) into ctrl and enqueues the planning and persistent kernels on
// st: replayed as a graph cached in ws when use_graph, else launched.
int launch_planned(BatchPlan& plan, uint8_t* ctrl, void* pinned, hipStream_t st, bool use_graph,
                   Workspace* ws);
// Single-buffer encode (api.cpp).  prepare_encode validates the call on the
// host and lays out its scratch as offsets (*ws_need bytes in all);
// bind_workspace rebases them onto the scratch at `base`; enqueue_encode
// launches the kernels on st.  pfx: the prefix-code family; timed = false
// keeps the launches out of the diagnostic timing (which creates events).
int prepare_encode(const rans_table* table, const rans_params* params, const void* d_syms,
                   uint64_t n, void* d_out, EncodeArgs* ea, ScanArgs* sa, CompactArgs* ca,
                   PlaceArgs* pa, uint64_t* ws_need, bool pfx = false);
void bind_workspace(uint8_t* base, EncodeArgs* ea, ScanArgs* sa, CompactArgs* ca, PlaceArgs* pa);
hipError_t enqueue_encode(const EncodeArgs& ea, const ScanArgs& sa, const CompactArgs& ca,
                          const PlaceArgs& pa, int R, int W, hipStream_t st, bool pfx = false,
                          bool timed = true);

// Frees the workspace of (current device, stream), if there is one; waits
// for the stream first.
void release_workspace(hipStream_t stream);
rans_batch_config batch_config();
void fill_decode_tables(const DevTable& t, Layout layout, DecodeArgs* a);

}  // namespace rans
