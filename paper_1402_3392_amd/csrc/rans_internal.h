// Internal declarations shared by the librans host code and its HIP kernels.
// Nothing here is part of the C ABI (include/librans.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/librans.h"

namespace rans {

constexpr uint32_t kMagic = 0x534E4172u;  // "rANS" read little-endian
constexpr uint32_t kHeaderBytes = 32;
constexpr uint32_t kDirEntryBytes = 16;

// Kernels report failures by atomicMin of a negative RANS_E* code into an
// int32 status word the caller zeroed; the most negative code wins.

// Decoder table layouts in LDS.
//   kPacked: per slot one u32 (f << 16 | (slot - cum_s)) plus the slot's
//            symbol (w bytes): one dependent LDS read on the state chain.
//   kTwoLevel: per slot the symbol, per symbol one u32 (f | cum << 16):
//            two dependent LDS reads, much smaller for large M.
//   kFused: per slot one u64 {bias, f | sym << 24}: a single LDS read gives
//            f, bias and the symbol (8-bit alphabets, M <= 2^14: <= 128 KiB).
enum Layout : int { kPacked = 1, kTwoLevel = 2, kFused = 3 };

// Device-resident table (see tables.cpp for how each array is built).
struct DevTable {
    uint32_t alphabet;  // symbols 0 .. alphabet-1
    uint32_t k;         // M = 2^k
    uint32_t sym_w;     // bytes per slot->symbol entry (1 if alphabet <= 256)
    uint32_t* dec;      // [M]      packed slot entries (kPacked)
    void* sym;          // [M]      slot -> symbol, sym_w bytes each
    uint32_t* fc;       // [alpha]  f | cum << 16 (kTwoLevel)
    uint4* enc;         // [alpha+1] encoder entries; the extra one has f = 0
    uint2* fused;       // [M]      kFused entries, or null
    uint64_t dec_bytes, sym_bytes, fc_bytes, enc_bytes, fused_bytes;  // padded to 16
    // prefix-code family (alphabet <= 4096, else null): per symbol
    // code | len << 16 (alphabet + 1 entries, the last one len 0), and per
    // value of the next pfx_maxlen bits symbol | len << 12
    uint32_t* pfx_enc;
    uint16_t* pfx_dec;
    uint32_t pfx_maxlen;
    uint64_t pfx_enc_bytes, pfx_dec_bytes;
    // every f is 0 or at least M / 256: with byte digits (b = 2^8) no state
    // moves two digits in one renormalisation (Algorithm 1's loop runs at
    // most once), so coders may take the single-digit step
    uint32_t one_digit;
};

// Encoder entry, one per symbol (uint4):
//   x = m                (q = x / f = mulhi(x + inc, m) >> sh: Robison,
//                         "N-bit unsigned division via N-bit multiply-add")
//   y = f | cum << 16
//   z = inc | sh << 8
//   w = M - f            (C(s,x) = x + q*(M - f) + cum)

struct DecodeArgs {
    const uint8_t* in;
    uint64_t in_len;
    void* out;
    uint64_t n;          // symbols in the container
    uint32_t C;          // symbols per chunk
    uint32_t n_chunks;
    uint32_t N;          // coders per chunk (power of two <= 64)
    uint32_t log2N;
    uint32_t k, l;
    uint32_t alphabet;
    uint32_t bf;         // breadth-first digit order (Section 5)
    uint32_t esc;        // escape coding with raw digits (16-bit symbols)
    uint32_t pfx;        // prefix-code family (k = its longest code length)
    uint32_t one;        // byte digits and a one-digit table: single-digit refills
    const void* lut;     // fused consumer: alphabet entries of lut_w bytes (device)
    uint32_t lut_w;      // 0 (symbol output), 2 or 4
    const void* tab0;    // kPacked: dec; kTwoLevel: sym
    const void* tab1;    // kPacked: sym; kTwoLevel: fc
    uint32_t tab0_bytes, tab1_bytes;  // multiples of 16
    int32_t* status;
};

struct EncodeArgs {
    const void* syms;
    uint64_t n;
    uint32_t C;
    uint32_t n_chunks;
    uint32_t N;
    uint32_t log2N;
    uint32_t k, l;
    uint32_t alphabet;
    uint32_t bf;          // breadth-first digit order (Section 5)
    uint32_t esc;         // escape coding with raw digits (16-bit symbols)
    uint32_t one;         // byte digits, a one-digit table, no escapes: single-digit steps
    const uint4* enc;     // alphabet + 1 entries
    uint32_t enc_bytes;   // multiple of 16
    uint8_t* slots;       // n_chunks slots, slot_stride apart
    uint64_t slot_bytes;  // digit capacity of a slot in bytes (multiple of 16);
                          // digits end at slot + slot_bytes
    uint64_t slot_stride; // slot_bytes + a 256-byte junk area
    uint32_t* states;     // n_chunks * N final states
    uint32_t* ndig;       // n_chunks digit counts
    int32_t* status;
};

// Placement of encoded chunks inside the encode kernel (N = 32, 64): each
// chunk publishes its aligned length, sums the published lengths of the
// chunks below it (two lane-parallel levels: its group of 64, then the group
// totals) and copies itself to its final offset.
struct PlaceArgs {
    uint32_t* ticket;      // chunk tickets in start order (zeroed before)
    uint64_t* lookback;    // n_chunks + ceil(n_chunks / 64) words: flag << 62 | value (zeroed before)
    uint8_t* out;
    uint64_t out_cap;
    uint64_t* total;       // container length (workspace)
    uint64_t* total_out;   // optional caller copy
    uint8_t hdr[32];
};

struct ScanArgs {
    const uint32_t* ndig;
    uint32_t n_chunks;
    uint32_t N;
    uint32_t digit_bytes;
    uint8_t* out;
    uint64_t out_cap;
    uint8_t hdr[32];      // header image written by the scan kernel
    uint64_t* chunk_off;  // n_chunks destination offsets (scratch)
    uint64_t* total;      // container length (workspace)
    uint64_t* total_out;  // optional second copy (caller's device word)
    int32_t* status;
};

struct CompactArgs {
    const uint8_t* slots;
    uint64_t slot_bytes;
    uint64_t slot_stride;
    const uint32_t* states;
    const uint32_t* ndig;
    const uint64_t* chunk_off;
    const uint64_t* total;
    uint32_t n_chunks;
    uint32_t N;
    uint32_t digit_bytes;
    uint8_t* out;
    uint64_t out_cap;
};

// One job of a batch, device-resident (written by the host, then completed
// by the planning kernel).
struct BatchJob {
    const uint8_t* in;     // decode: container; encode: symbols
    uint64_t in_len;       // bytes
    uint8_t* out;          // decode: symbols; encode: container
    uint64_t out_cap;      // bytes
    uint64_t* d_out_len;
    int32_t* d_status;
    const void* tab_sym;   // decode tables of the batch's layout
    const void* tab_ent;
    const uint4* enc;      // encoder entries (alphabet + 1)
    uint32_t sym_bytes, ent_bytes, enc_bytes, alphabet;
    uint32_t one;          // encode with byte digits and a one-digit table: single-digit steps
    // plan
    uint64_t n;            // symbols
    uint64_t total;        // encode: container length
    uint32_t C, nch;       // symbols per chunk, chunks (0 when the job failed)
    uint32_t item_base;    // first work item
    // encode scratch of this job, set by the host: one digit slot per chunk
    // (BatchArgs::slot_stride apart) and the placement words (nch chunk
    // words, then one per group of 64 chunks), zeroed by the planning kernel
    uint8_t* slots;
    uint64_t* lookback;
};

struct BatchArgs {
    BatchJob* jobs;
    uint32_t njobs;
    uint32_t k, r, l, w, N, C;  // C: encode chunk size (0 = whole input)
    uint32_t bf;                // breadth-first digit order (Section 5)
    uint32_t G;                 // waves per block
    uint32_t cpi;               // chunks per work item: G times the chunks one wave decodes
    uint32_t* counter;          // work-queue head, set by the planning kernel
    uint32_t* totals;           // [0] work items, [1] chunks
    uint32_t* item_job;         // work item -> job
    uint32_t max_items;         // entries of item_job
    uint64_t slot_bytes, slot_stride;  // encode digit slots (BatchJob::slots)
    uint32_t tab_lds;           // LDS bytes reserved for the largest table
    uint32_t grid;              // persistent blocks; decode: block b starts with work item b
};

// Launchers (kernels.hip).  All asynchronous on `stream`.
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, uint32_t count, hipStream_t stream);
hipError_t launch_decode(const DecodeArgs& a, int R, int W, Layout layout, hipStream_t stream);
hipError_t launch_encode(const EncodeArgs& a, int R, int W, hipStream_t stream);
// One-wave-per-chunk fast paths for N = 32 or 64 (decode64.hip /
// encode64.hip); need (C * w) % 16 == 0 and 16-byte aligned symbol buffers.
hipError_t launch_decode64(const DecodeArgs& a, int R, int W, Layout layout, hipStream_t stream);
// Encode with in-kernel placement (no scan / compaction kernels).
hipError_t launch_encode64_place(const EncodeArgs& a, const PlaceArgs& p, int R, int W,
                                 hipStream_t stream);
// Prefix-code family encode, multiplexed and placed in-kernel; a.enc holds
// the code entries (a.enc_bytes), a.slots one slot of a.slot_bytes per chunk.
hipError_t launch_pfx_encode64(const EncodeArgs& a, const PlaceArgs& p, int W, hipStream_t stream);
uint32_t decode64_lds_per_wave(Layout layout);
// LDS per wave of the decoder that codes 64 / N chunks per wave (N = 32, 64).
uint32_t decode_seg_lds_per_wave(Layout layout, uint32_t N);
// Decode fused with a table lookup: out[i] = lut[symbol i] (a.lut, a.lut_w).
hipError_t launch_decode64_lut(const DecodeArgs& a, int R, Layout layout, hipStream_t stream);
// LDS bytes of a staged lookup table of `alphabet` entries of lw bytes.
inline uint32_t lut_lds_bytes(uint32_t alphabet, int lw) { return (alphabet * uint32_t(lw) + 15) & ~15u; }
// LDS per wave of the encoders: a 4 KiB digit ring, a 1 KiB symbol block and
// 128 bytes for the stores of lanes with nothing to emit.
constexpr uint32_t kEncWaveLdsBytes = 5248;
// Encoder digit slots: sizes are multiples of kSlotAlign (the encoder
// writes whole windows of that size, aligned to multiples of it), and
// kSlotPad bytes follow every slot (stores that pad a block's window count,
// and reads just past a chunk's digits).
constexpr uint64_t kSlotAlign = 1024;
constexpr uint64_t kSlotPad = 1024;
// LDS bytes of an encoder table staged for w-byte symbols: with 8-bit
// symbols all 256 entries are staged (those at or above the alphabet mark
// the symbol as not encodable), so a symbol indexes the table unclamped.
__host__ __device__ inline uint32_t enc_lds_bytes(uint32_t enc_bytes, uint32_t w)
{
    return w == 1 && enc_bytes < 256 * 16 ? 256 * 16 : enc_bytes;
}

// Batched pass (batch.hip).  `decode` selects the direction.
hipError_t launch_batch(const BatchArgs& a, bool decode, int R, int W, int SW, Layout layout,
                        uint32_t grid, hipStream_t stream);
hipError_t launch_scan(const ScanArgs& a, hipStream_t stream);
hipError_t launch_compact(const CompactArgs& a, hipStream_t stream);

// Host helpers (tables.cpp / api.cpp).
int quantize(const uint64_t* counts, uint32_t alphabet, uint32_t k, uint32_t* f);
const DevTable* dev_table(const rans_table* t);
int max_lds_bytes();

}  // namespace rans
