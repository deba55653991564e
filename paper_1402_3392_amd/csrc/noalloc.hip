// Stream-ordered encode that allocates nothing: the digit slots, chunk
// offsets and placement words that rans_encode_async keeps in a per-stream
// workspace come from a fixed array in device memory instead, so callers
// that cannot allocate (code under graph capture, tight serving loops) can
// still encode.  The kernels are the ones rans_encode_async launches.
#include <mutex>

#include "rans_internal.h"
#include "workspace.h"

namespace rans {
namespace {

// Every GPU the library runs on holds one copy of this array for the life
// of the process.  Host code never passes its name to a kernel: that is a
// host-side stand-in, not the device address.  The address comes from
// hipGetSymbolAddress, once per device with that device current.
constexpr uint64_t kNoAllocScratchBytes = 64ull << 20;
__device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint8_t* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, or null (and the HIP
// error code in *err) when it cannot be had.
uint8_t* scratch_for_current_device(hipError_t* err)
{
    int dev = 0;
    *err = hipGetDevice(&dev);
    if (*err != hipSuccess)
        return nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (*err != hipSuccess)
            return nullptr;
        g_ptr[dev] = static_cast<uint8_t*>(p);
    }
    return g_ptr[dev];
}

}  // namespace
}  // namespace rans

using namespace rans;

extern "C" int rans_encode_async_noalloc(const rans_table* table, const rans_params* params,
                                         const void* d_syms, uint64_t n, void* d_out, uint64_t out_cap,
                                         uint64_t* d_out_len, int32_t* d_status, void* stream)
{
    if (!d_status)
        return RANS_EINVAL;
    EncodeArgs ea;
    ScanArgs sa;
    CompactArgs ca;
    PlaceArgs pa;
    uint64_t need = 0;
    int rc = prepare_encode(table, params, d_syms, n, d_out, &ea, &sa, &ca, &pa, &need, false);
    if (rc != RANS_OK)
        return rc;
    if (need > kNoAllocScratchBytes)
        return RANS_ENOMEM;  // more scratch than the fixed array holds
    hipError_t e = hipSuccess;
    uint8_t* base = scratch_for_current_device(&e);
    if (!base)
        return RANS_EDEVICE;
    bind_workspace(base, &ea, &sa, &ca, &pa);
    ea.status = sa.status = d_status;
    sa.out_cap = ca.out_cap = pa.out_cap = out_cap;
    sa.total_out = pa.total_out = d_out_len;
    // the kernels clear what must start at zero (the placement words and the
    // start ticket) themselves, with a fill kernel ahead of the encoder
    e = enqueue_encode(ea, sa, ca, pa, params->radix_bits, params->sym_bytes,
                       static_cast<hipStream_t>(stream), false, false);
    return e == hipSuccess ? RANS_OK : RANS_EDEVICE;
}
