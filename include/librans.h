/*
 * librans -- interleaved streaming rANS on AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Plain pointers and sizes only; "device" pointers are HIP device
 * allocations (any allocator: hipMalloc, a torch tensor's data_ptr(), ...),
 * "host" pointers are ordinary process memory.  `stream` is a hipStream_t
 * passed as void* (NULL = the default stream).
 *
 * Method: F. Giesen, "Interleaved entropy coders" (arXiv:1402.3392).
 *   - coding pair C / D and streaming renormalisation into I = [L, bL):
 *     Section 2, Algorithm 1;
 *   - N coders with separate states share one stream with no metadata,
 *     symbol i belonging to coder (i mod N): Sections 3 and 4;
 *   - the encoder walks the message backwards and writes the stream
 *     backwards; its final states travel with the stream: Section 2;
 *   - refill/flush offsets of the coders that renormalise in a step come
 *     from a ballot of "this coder does I/O" plus a prefix count: Section 6.
 * The coder used is rANS: C(s,x) = M*floor(x/f_s) + (x mod f_s) + cum_s,
 * D(x) = (s, f_s*floor(x/M) + (x mod M) - cum_s) with s the symbol whose
 * slot range [cum_s, cum_s+f_s) holds x mod M; M = 2^k.  (The paper's worked
 * example in Section 2.1 is this coder with M = 4, f = (1, 3).)
 *
 * Stream format (container).  All fields little-endian.
 *   header, 32 bytes: u32 magic 0x534E4172 ("rANS"), u8 version 1, u8 k,
 *     u8 r, u8 l, u8 w, u8 flags (bit 0: breadth-first digit order, bit 1:
 *     escape coding, not both; or 4 alone: the prefix-code family below),
 *     u16 N, u32 C, u64 n, u32 n_chunks, u32 0
 *   directory: n_chunks x { u64 offset, u32 length, u32 0 }
 *   chunk streams, each at a 16-byte aligned offset, zero padding between;
 *     the first at align16(32 + 16*n_chunks); the total length is
 *     align16(end of the last chunk) (32 when n == 0).
 *   chunk c covers symbols [c*C, min(n, (c+1)*C)); its stream is the N final
 *     encoder states (u32, coder 0 first) followed by the digits in decoder
 *     order: u16 words when b = 2^16, bytes when b = 2^8.  A coder that
 *     renormalises by two digits for one symbol reads the more significant
 *     digit first.  Digit order of one step (Section 5): depth-first puts
 *     each coder's digits together, coders ascending; breadth-first puts the
 *     first digit of every coder that reads one (coders ascending), then the
 *     second digit of every coder that reads two.  The orders coincide when
 *     b >= M (at most one digit per step: always with b = 2^16, as k <= 15),
 *     so they differ only for b = 2^8 with k > 8.
 *   escape coding (flags bit 1; 16-bit symbols, depth-first): the table's
 *     last symbol E = alphabet - 1 is an escape.  A value v is coded as the
 *     symbol v when v < E and its frequency is not 0, otherwise as E followed
 *     by 16 raw bits holding v (one u16 word, or two bytes high first); in a
 *     coder's share of a step the raw digits follow its renormalisation
 *     digits.  Raw digits never touch a coder state (Section 3: encoder and
 *     decoder run in lockstep, so raw data needs no bypass mode), so any
 *     16-bit value can be coded with a table of the frequent ones.  The
 *     one-wave-per-chunk and generic kernels support it; the batched entry
 *     points, the server and rans_decode_lut reject it (RANS_EINVAL).
 *   prefix-code family (flags 4; r = 16, l recorded as 16 and unused): the
 *     multiplexer of Section 4 applied to a second coder family, a canonical
 *     prefix code with lengths max(1, ceil(log2(M / f_s))) (at most k bits;
 *     symbols ordered by (length, index) take consecutive code values).
 *     Coder j codes symbols j, j+N, ... into its own bit sequence (codes
 *     most significant bit first, 16-bit words); its decoder reads one word
 *     before a symbol whenever it holds fewer than 16 bits.  The chunk
 *     stream is the N coders' bit counts (u32, in place of the states), then
 *     their words in the order the N decoders, stepping through the chunk's
 *     symbols, read them -- what an instrumented decoder copying every word
 *     it reads produces -- so the stream needs no per-coder metadata.  The
 *     last word of a coder is zero padded, and a coder whose rule reads one
 *     word beyond its bits reads a word of zeros.  Decoding checks that every
 *     coder consumed exactly its bit count.  Chunks are the periodic flush
 *     that bounds the encoder's buffering.
 *     Every coder starts encoding in state L;
 *     when a chunk's length is not a multiple of N, the last step only
 *     involves coders 0 .. (len mod N)-1.
 *
 * Error behaviour: every entry point returns RANS_OK (0) or a negative
 * RANS_E* code; nothing aborts the process.  A decode whose coders do not all
 * end in state L with their chunk stream exactly consumed reports
 * RANS_ECORRUPT (the decoder retraces the encoder's states in reverse,
 * Section 3); the symbols written for such a chunk are unspecified.
 * No entry point reads or writes outside the buffers and lengths it is given,
 * whatever the content of a container.
 */
#ifndef LIBRANS_H
#define LIBRANS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RANS_OK 0
#define RANS_EINVAL (-1)   /* parameters out of range or inconsistent        */
#define RANS_EPREC (-2)    /* more distinct symbols present than M = 2^k      */
#define RANS_ENOSYM (-3)   /* a symbol with frequency 0 (or >= alphabet)      */
#define RANS_ENOSPC (-4)   /* output capacity too small                       */
#define RANS_ECORRUPT (-5) /* malformed container or failed end-of-chunk check */
#define RANS_EDEVICE (-6)  /* a HIP runtime call failed                       */
#define RANS_ENOMEM (-7)   /* host or device allocation failed                */

/* Coder parameters.  Constraints checked by rans_params_check:
 *   8 <= prob_bits (k) <= 15          M = 2^k, the frequencies' denominator
 *   radix_bits (r) in {8, 16}         b = 2^r, digits are bytes or u16 words
 *   k <= state_lbits (l), l + r <= 32 L = 2^l; L a multiple of M makes every
 *                                     precursor set b-unique (Section 2) and
 *                                     the state fits 32 bits
 *   sym_bytes (w) in {1, 2}           uint8 or uint16 symbols
 *   interleave (N) in {1,2,4,...,64}  coders per chunk (one per wave lane)
 *   digit_order in {0, 1}             0 depth-first, 1 breadth-first digit
 *                                     order within a step (Section 5);
 *                                     recorded in the container header, so
 *                                     decoding takes it from there
 *   escape in {0, 1}                  escape coding with raw digits (Section
 *                                     3: raw data interleaved in the stream
 *                                     at agreed points); needs sym_bytes 2
 *                                     and digit_order 0; see below
 *   chunk_syms (C)                    symbols per chunk; 0 = the whole input
 *                                     (then n must fit 32 bits)            */
typedef struct rans_params {
    uint8_t prob_bits;
    uint8_t radix_bits;
    uint8_t state_lbits;
    uint8_t sym_bytes;
    uint16_t interleave;
    uint8_t digit_order;
    uint8_t escape;
    uint32_t chunk_syms;
} rans_params;

/* Opaque static order-0 model (Section 7: one static distribution per
 * input): frequencies, cumulative frequencies, slot->symbol map and the
 * encoder's per-symbol division constants, resident in device memory.
 * Owned by the library; the device copy lives on the device that was
 * current when it was built. */
typedef struct rans_table rans_table;

/* Host only, touches no GPU.  Quantises counts[alphabet] (host) to
 * freqs_out[alphabet] (host) summing to 2^prob_bits: integer largest
 * remainder, f_s = floor(c_s*M/T) with the deficit given to the largest
 * remainders (ties: lower symbol), present symbols forced to >= 1, an excess
 * taken from the largest frequencies.  Counts already summing to M map to
 * themselves.  Errors: RANS_EINVAL (alphabet 0, prob_bits outside 1..16, all
 * counts 0, a total >= 2^47), RANS_EPREC (more present symbols than M). */
int rans_quantize(const uint64_t *counts, uint32_t alphabet, uint32_t prob_bits,
                  uint32_t *freqs_out);

/* Builds a table from host counts[alphabet] (quantised as rans_quantize
 * does) on the current device.  alphabet <= 65536, prob_bits 8..15.
 * The table is the coding pair's data (Section 2: f_s and cum_s with
 * M = 2^k, the symbol of every slot of [0, M) for D) plus, per symbol, the
 * renormalisation bound of Algorithm 1's encoder and an exact reciprocal
 * of f_s for C's division; one static table per input, as Section 7's
 * order-0 model.  *out receives a handle to destroy with rans_table_destroy.
 * Errors: RANS_EINVAL, RANS_EPREC (as rans_quantize), RANS_ENOMEM,
 * RANS_EDEVICE.  Synchronous. */
int rans_tables_build(const uint64_t *counts, uint32_t alphabet, uint32_t prob_bits,
                      rans_table **out);

/* Copies the table's quantised frequencies to freqs_out[alphabet] (host). */
int rans_table_freqs(const rans_table *table, uint32_t *freqs_out);

/* Alphabet size and prob_bits of a table (0 for NULL). */
uint32_t rans_table_alphabet(const rans_table *table);
uint32_t rans_table_prob_bits(const rans_table *table);

/* Releases a table (NULL is a no-op). */
void rans_table_destroy(rans_table *table);

/* Host only.  RANS_OK or RANS_EINVAL for the constraints listed above. */
int rans_params_check(const rans_params *params);

/* Host only.  An upper bound on the container length rans_encode can
 * produce for n_syms symbols (each symbol emits at most ceil(k/r) digits,
 * plus 16/r raw digits with escape coding).  Returns 0 for invalid
 * parameters. */
uint64_t rans_encode_bound(uint64_t n_syms, const rans_params *params);

/* Encodes d_syms[n_syms] (device; uint8 or uint16 per params->sym_bytes)
 * into a container at d_out (device, out_cap bytes).  Each chunk is coded by
 * N interleaved coders (Section 3: symbol i of the chunk goes to coder
 * i mod N), each one Algorithm 1's encoder (Section 2): starting from state
 * L and walking the chunk backwards, a coder emits low digits of its state
 * while it is at or above f_s*b*L/M, then applies C(s, x); the digits of a
 * step are written in the order the decoders will read them, and the final
 * states go to the head of the chunk's stream.  The table's
 * prob_bits must equal params->prob_bits.  *out_len (host) receives the
 * container length.  Blocks until the result is known (stream-ordered
 * before that).  Errors: RANS_EINVAL, RANS_ENOSYM (a symbol of frequency 0
 * or >= the alphabet; the output is then unspecified), RANS_ENOSPC (out_cap
 * below the container length, which is still reported in *out_len),
 * RANS_EDEVICE, RANS_ENOMEM. */
int rans_encode(const rans_table *table, const rans_params *params, const void *d_syms,
                uint64_t n_syms, void *d_out, uint64_t out_cap, uint64_t *out_len,
                void *stream);

/* Decodes the container d_in[in_len] (device) into d_syms (device,
 * syms_cap symbols of the container's width).  Per chunk, the N coders start
 * from the transmitted states and take the chunk's symbols round-robin
 * (Section 3); each step is Algorithm 1's decoder (Section 2): (s, x) = D(x),
 * then, while x < L, x = b*x + the next digit, the reading coders taking
 * consecutive digits in coder order (Section 6's ballot and prefix count).  The table must be the one
 * the container was encoded with (same prob_bits; the library cannot check
 * more).  *n_syms (host) receives the symbol count.  The header is read
 * through a small device-to-host copy; the call blocks until the decode has
 * finished.  Errors: RANS_ECORRUPT, RANS_ENOSPC (syms_cap < n),
 * RANS_EINVAL, RANS_EDEVICE. */
int rans_decode(const rans_table *table, const void *d_in, uint64_t in_len, void *d_syms,
                uint64_t syms_cap, uint64_t *n_syms, void *stream);

/* Stream-ordered encode: validates on the host, enqueues the kernels on
 * `stream` and returns without waiting.  *d_status (device int32) must hold
 * RANS_OK when the stream reaches the call; the kernels lower it to the most
 * negative failure code (RANS_ENOSYM, RANS_ENOSPC).  *d_out_len (device
 * u64) receives the container length.  Host-side validation errors are
 * returned directly.  The library's per-stream workspace is reused in
 * stream order, so back-to-back calls on one stream are safe. */
int rans_encode_async(const rans_table *table, const rans_params *params, const void *d_syms,
                      uint64_t n_syms, void *d_out, uint64_t out_cap, uint64_t *d_out_len,
                      int32_t *d_status, void *stream);

/* rans_encode_async for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same container, but the scratch that
 * rans_encode_async keeps in a per-stream workspace (digit slots, chunk
 * offsets, placement words) lives in one fixed 64 MiB array of device
 * memory that every GPU the library runs on holds until the process ends.
 * The call allocates nothing (no hipMalloc, no pinned memory, no events) and
 * clears what must start at zero with a kernel.  A call needing more scratch
 * than the array holds (about 2 bytes per symbol plus 1.3 KiB per chunk:
 * some 31 million symbols in 64 KiB chunks) returns RANS_ENOMEM and launches
 * nothing.  Every call on a GPU shares that GPU's array: calls that overlap
 * on one GPU (two streams, or two host threads) race and must be ordered by
 * the caller.  Arguments, errors and d_status / d_out_len as
 * rans_encode_async (rANS only). */
int rans_encode_async_noalloc(const rans_table *table, const rans_params *params,
                              const void *d_syms, uint64_t n_syms, void *d_out, uint64_t out_cap,
                              uint64_t *d_out_len, int32_t *d_status, void *stream);

/* Stream-ordered decode.  h_header (host) is a copy of the container's first
 * 32 bytes, which the caller already holds (it is validated here, so no
 * device-to-host copy is needed).  *d_status as for rans_encode_async
 * (RANS_ECORRUPT from the end-of-chunk check).  Returns without waiting. */
int rans_decode_async(const rans_table *table, const void *d_in, uint64_t in_len,
                      const void *h_header, void *d_syms, uint64_t syms_cap, int32_t *d_status,
                      void *stream);

/* Encode with the prefix-code family instead of rANS (format above; the
 * container decodes with rans_decode / rans_decode_async, which read the
 * family from the header).  params as for rans_encode with radix_bits 16,
 * state_lbits 16, digit_order 0, escape 0, interleave 32 or 64, chunk_syms *
 * sym_bytes a multiple of 16 and a 16-byte aligned d_syms; the table's
 * alphabet at most 4096.  Otherwise RANS_EINVAL.  Errors, out_len and
 * blocking as rans_encode / rans_encode_async. */
int rans_pfx_encode(const rans_table *table, const rans_params *params, const void *d_syms,
                    uint64_t n_syms, void *d_out, uint64_t out_cap, uint64_t *out_len,
                    void *stream);
int rans_pfx_encode_async(const rans_table *table, const rans_params *params, const void *d_syms,
                          uint64_t n_syms, void *d_out, uint64_t out_cap, uint64_t *d_out_len,
                          int32_t *d_status, void *stream);

/* Decode fused with a table-lookup consumer (Section 6: the decoder is small
 * enough to be fused into the kernel that uses its output).  Output element
 * i is d_lut[symbol i]: lut_bytes (2 or 4) bytes copied bit for bit, e.g. the
 * bf16 / fp16 / fp32 value of a codebook index when a tensor was stored as
 * entropy-coded codes.  The symbols themselves never reach memory.
 *   d_lut   device, the table's alphabet entries of lut_bytes each, aligned
 *           to lut_bytes; read once per block into LDS.
 *   d_out   device, out_cap elements of lut_bytes, 16-byte aligned.
 * Needs a container with N = 32 or 64 and chunk_syms * lut_bytes a multiple
 * of 16 (the one-wave-per-chunk kernels), else RANS_EINVAL.  *n_syms, errors
 * and blocking as rans_decode (RANS_ENOSPC when out_cap < n). */
int rans_decode_lut(const rans_table *table, const void *d_in, uint64_t in_len, const void *d_lut,
                    uint32_t lut_bytes, void *d_out, uint64_t out_cap, uint64_t *n_syms,
                    void *stream);

/* Stream-ordered form of rans_decode_lut; h_header and d_status as for
 * rans_decode_async. */
int rans_decode_lut_async(const rans_table *table, const void *d_in, uint64_t in_len,
                          const void *h_header, const void *d_lut, uint32_t lut_bytes, void *d_out,
                          uint64_t out_cap, int32_t *d_status, void *stream);

/* One stream of a batch.  `table` is a host handle; every other pointer is
 * device memory.  Encode: in = symbols, in_len = their count in BYTES
 * (a multiple of sym_bytes), out = container buffer of out_cap bytes,
 * *d_out_len = container length (with RANS_ENOSPC: the length the container
 * needs).  Decode: in = container of in_len bytes,
 * out = symbol buffer of out_cap BYTES, *d_out_len = symbols decoded.
 * *d_status = RANS_OK or the job's RANS_E* code.  A failing job never
 * affects another job's output. */
typedef struct rans_job {
    const rans_table *table;
    const void *in;
    uint64_t in_len;
    void *out;
    uint64_t out_cap;
    uint64_t *d_out_len;
    int32_t *d_status;
} rans_job;

/* Batched encode of njobs independent streams with shared params in one
 * persistent-kernel pass (replayed as a HIP graph).  Every job is coded as
 * rans_encode codes it (same container, byte for byte), with its own table;
 * chunks of all jobs are independent coding units (Section 3), which is
 * what lets one launch hold thousands of streams.  Asynchronous: results
 * are in the jobs' d_out_len / d_status once `stream` reaches this point.
 * Returns RANS_EINVAL for invalid params or job descriptors (checked on the
 * host), RANS_ENOMEM / RANS_EDEVICE for runtime failures. */
int rans_encode_batch(const rans_job *jobs, uint32_t njobs, const rans_params *params,
                      void *stream);

/* Batched decode of njobs containers, all encoded with params' k, r, l, w,
 * N and digit order (checked per job on the device; a mismatch fails that
 * job with RANS_EINVAL).  Each job decodes as rans_decode does (Sections 2,
 * 3 and 6).  Asynchronous, as rans_encode_batch. */
int rans_decode_batch(const rans_job *jobs, uint32_t njobs, const rans_params *params,
                      void *stream);

/* Launch shape of the batched entry points (process-wide; the autotuner
 * sets it).  waves_per_group: waves per persistent block sharing one staged
 * table (1..16; a maximum: a launch uses fewer when their rings and the
 * table do not fit LDS together); a work item covers waves_per_group
 * times 64 / N chunks (a wave codes 64 / N chunks); groups_per_cu:
 * persistent blocks per compute unit (1..16; blocks beyond what the
 * registers and LDS of a compute unit hold wait for others to end);
 * table_layout: decode table
 * layout in LDS, 0 = automatic, 1 = per-slot packed entries plus symbol
 * map, 2 = symbol map plus per-symbol entries, 3 = one 8-byte entry per slot
 * holding f, bias and symbol (8-bit alphabets, prob_bits <= 14); use_graph: replay the batch as a captured HIP
 * graph (1) or launch its kernels directly (0).  The batched kernels code
 * 32 or 64 interleaved coders per chunk (params->interleave 32 or 64; with
 * 32 a wave codes two chunks, lanes 0-31 and 32-63); batched encode
 * needs chunk_syms != 0 with chunk_syms * sym_bytes a multiple of 16, and
 * every buffer 16-byte aligned.  Batched calls on a stream that is being
 * captured launch directly (no nested graph). */
typedef struct rans_batch_config {
    uint32_t waves_per_group;
    uint32_t groups_per_cu;
    uint32_t table_layout;
    uint32_t use_graph;
} rans_batch_config;
int rans_batch_set_config(const rans_batch_config *cfg);
int rans_batch_get_config(rans_batch_config *cfg);

/* Autotuner.  Times the batched kernels on a sample (d_syms[n_syms],
 * device, 16-byte aligned, coded with `table` and base's k, r, l, w) over
 * the interleave factor N in {32, 64} (lanes per stream: a decoding wave
 * codes 64 / N chunks at once) and chunk sizes C in {4096 .. 65536} (both
 * chosen at encode time and written into the container), and decode
 * launch shapes (waves per work item, blocks per CU, table layout), then
 * whether the best shape runs faster replayed as a HIP graph or launched
 * directly.  base->interleave 0 searches N over {32, 64}; 32 or 64 keeps
 * it; base->chunk_syms is ignored.  A candidate's
 * score is its encode + decode time, penalised when its container exceeds
 * the container of 64 coders and 64 KiB chunks by more than 1%.  The best
 * shape becomes the process-wide rans_batch_config; *out reports it with
 * the measured rates (the caller encodes with out->interleave and
 * out->chunk_syms).  Results are appended to cache_path (text, one line
 * per device / parameter / alphabet class / size class; NULL disables the
 * cache) and reused on a hit. */
typedef struct rans_tune_result {
    uint32_t chunk_syms;
    uint32_t waves_per_group;
    uint32_t groups_per_cu;
    uint32_t table_layout;
    double encode_gbps;
    double decode_gbps;
    uint32_t use_graph;
    uint32_t interleave;       /* N: coders per chunk */
    uint32_t lanes_per_stream; /* lanes that code one chunk (N) */
    uint32_t chunks_per_wave;  /* chunks a decoding wave codes at once (64 / N) */
} rans_tune_result;
int rans_autotune(const rans_table *table, const void *d_syms, uint64_t n_syms,
                  const rans_params *base, const char *cache_path, rans_tune_result *out);

/* The same search on a whole batch: jobs are encode jobs as for
 * rans_encode_batch (symbols in `in`, each with its table; their out,
 * d_out_len and d_status are not touched -- the tuner encodes into memory of
 * its own).  Every candidate is timed on all of the jobs together, so launch
 * shapes that suit many short streams win where they should.  The cache key
 * adds the number of streams (power-of-two class). */
int rans_autotune_batch(const rans_job *jobs, uint32_t njobs, const rans_params *base,
                        const char *cache_path, rans_tune_result *out);

/* ---------------------------------------------------------------- serving --
 * Continuous-batching request server (not in the paper: the serving shape
 * around Section 3's independent coders).  Requests (encode or decode of one
 * device-resident buffer, each with its own table) are admitted first come
 * first served while the sum of their costs fits hbm_budget; admitted
 * requests are launched as batched persistent kernels on whichever of the
 * server's `streams` is idle, up to max_batch per launch, so requests that
 * arrive while others run are launched alongside them.
 * Memory: rans_server_create makes ONE device allocation of exactly
 * hbm_budget bytes.  Its first part holds every stream's control region
 * (job descriptors, work-item map, status words; sized at creation for
 * max_batch requests whose inputs fit the budget, and reported as `fixed`);
 * the rest is an arena holding each admitted request's output capacity and,
 * to encode, its digit slots and placement words (about ceil(k/r)*r/8
 * bytes per symbol plus 1 KiB per chunk).  A request's cost is its input
 * length (caller memory, counted all the same) plus those arena bytes; the
 * sum of admitted costs plus `fixed` never exceeds hbm_budget.  Polling,
 * admission and launches allocate no device memory and wait for no stream.
 * The launch shape (rans_batch_config) in force at creation is kept for
 * the server's life.  All requests use config->params (decode: the
 * containers must carry those parameters; interleave 32 or 64).  The calls
 * are thread-safe. */
#define RANS_OP_ENCODE 0
#define RANS_OP_DECODE 1

typedef struct rans_server rans_server;

typedef struct rans_server_config {
    uint64_t hbm_budget; /* bytes, >= 1 MiB */
    uint32_t streams;    /* 1..16 */
    uint32_t max_batch;  /* requests per launch, >= 1 */
    rans_params params;
} rans_server_config;

/* One finished request.  d_out (device, inside the server's arena) holds
 * out_len bytes (encode: the container) or symbols (decode) until the
 * request is released (immediately, unless polled with keep_outputs).
 * latency_us: arrival to completion seen by the host; queue_us: arrival to
 * launch. */
typedef struct rans_completion {
    uint64_t id;
    int32_t status;
    int32_t op;
    uint64_t in_len;
    uint64_t out_len;
    void *d_out;
    double latency_us;
    double queue_us;
} rans_completion;

/* budget: hbm_budget; fixed: the control regions' bytes; used / peak: fixed
 * plus the costs of the admitted requests (now / at most so far); waiting,
 * ready: requests queued for admission / admitted but not launched;
 * busy_streams: streams with a launch in flight now, peak_busy_streams: at
 * most at once so far; launches: batched launches so far, of which
 * multi_request_launches held more than one request; max_launch_requests:
 * the most requests one launch held. */
typedef struct rans_server_stats_t {
    uint64_t budget, used, peak;
    uint32_t waiting, ready, busy_streams, peak_busy_streams;
    uint64_t launches, multi_request_launches, fixed;
    uint32_t max_launch_requests, reserved;
} rans_server_stats_t;

/* A request of an arrival schedule for rans_server_replay. */
typedef struct rans_server_request {
    int32_t op;
    uint32_t reserved;
    const rans_table *table;
    const void *d_in;
    uint64_t in_len;     /* bytes */
    uint64_t out_cap;    /* bytes */
    double arrival_us;   /* from the start of the replay, non-decreasing */
} rans_server_request;

int rans_server_create(const rans_server_config *config, rans_server **out);
void rans_server_destroy(rans_server *server);
/* Queues a request (RANS_ENOMEM if its cost alone exceeds the budget). */
int rans_server_submit(rans_server *server, int op, const rans_table *table, const void *d_in,
                       uint64_t in_len, uint64_t out_cap, uint64_t *id);
/* Advances the server (collects finished launches, admits, launches) and
 * returns up to max_out completions. */
int rans_server_poll(rans_server *server, int keep_outputs, rans_completion *out, uint32_t max_out,
                     uint32_t *n_out);
/* Frees a kept output. */
int rans_server_release(rans_server *server, uint64_t id);
int rans_server_stats(rans_server *server, rans_server_stats_t *stats);
/* Submits reqs[i] at its arrival time (microseconds after the call), polls
 * until all have completed, and stores request i's completion in results[i];
 * *makespan_us receives the elapsed time.  RANS_ENOMEM if kept outputs make
 * the remaining requests impossible to admit. */
int rans_server_replay(rans_server *server, const rans_server_request *reqs, uint32_t n,
                       int keep_outputs, rans_completion *results, double *makespan_us);

/* Kernel timing (diagnostics).  While enabled, every kernel launch the
 * library makes is bracketed by two HIP events recorded on the stream it is
 * launched on.  rans_timing_read waits for the recorded events and returns
 * the number of launches and their summed duration (milliseconds) for one
 * kind; rans_timing_reset forgets all records.  Kinds: */
#define RANS_KERNEL_DECODE 0       /* plain chunk decoder                    */
#define RANS_KERNEL_ENCODE 1       /* plain chunk encoder (into workspace)   */
#define RANS_KERNEL_SCAN 2         /* chunk-length scan + directory          */
#define RANS_KERNEL_COMPACT 3      /* chunk compaction into the container    */
#define RANS_KERNEL_BATCH_DECODE 4 /* persistent batched decoder             */
#define RANS_KERNEL_BATCH_ENCODE 5 /* persistent batched encoder             */
#define RANS_KERNEL_BATCH_PLAN 6   /* batch planning (headers, work items)   */
int rans_timing_enable(int on);
int rans_timing_reset(void);
int rans_timing_read(int kind, uint64_t *launches, double *total_ms);

/* Frees the device workspace, pinned staging and cached graphs the library
 * keeps for `stream` on the current device (they are created on the first
 * call that needs them and grow on demand).  Waits for the stream first.
 * Call it before destroying a stream the library was used on; it must not
 * overlap another call on the same stream.  A later call on the stream
 * creates a new workspace. */
int rans_workspace_release(void *stream);

/* Static description of an error code. */
const char *rans_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* LIBRANS_H */
