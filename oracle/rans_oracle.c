/*
 * rans_oracle.c -- CPU oracle for interleaved streaming rANS.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the GPU library computes.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it; the product library
 * never links, loads or calls it, and it shares no source with the product.
 *
 * Paper: F. Giesen, "Interleaved entropy coders" (arXiv:1402.3392).
 *
 * Everything is integer arithmetic on 64-bit unsigned values, with plain '/'
 * and '%', in the order the paper states it:
 *   - the coding pair C / D                       (Section 2; example in 2.1)
 *   - streaming renormalisation into I = [L, bL)  (Section 2, Algorithm 1)
 *   - the encoder walks the message backwards and writes the stream
 *     backwards; the decoder runs forwards        (Section 2)
 *   - the final encoder state travels with the stream (Section 2)
 *   - N coders with separate states share one stream, symbol i belonging to
 *     coder (i mod N), coders visited in ascending order within a round
 *                                                  (Sections 3 and 4)
 *   - depth-first digit order: each coder performs its whole renormalisation
 *     before the next coder runs, exactly as N scalar Algorithm-1 coders
 *     sharing one buffer would                     (Section 5)
 *   - breadth-first order (renormalisation rounds across the coders of one
 *     step) is provided as the alternative Section 5 describes.
 *
 * Readings of points the paper leaves open (the paper names rANS but never
 * writes its formula; it gives no quantiser, no initial state, no flush
 * layout, no tail rule and no container):
 *   Q1  C(s,x) = M*floor(x/f_s) + (x mod f_s) + cum_s, M = 2^k.  The paper's
 *       worked example (Section 2.1) is exactly this with M=4, f=(1,3),
 *       cum=(0,1).
 *   Q2  quantiser: integer largest remainder (orc_quantize below).
 *   Q3  every coder starts in state L.
 *   Q4  the N final states are stored at the head of a chunk stream as
 *       little-endian u32, coder 0 first; digits follow as little-endian u16
 *       words (b = 2^16) or bytes (b = 2^8).
 *   Q5  a coder that emits several digits for one symbol puts its most
 *       significant digit first in stream order (follows from x <- b*x + read).
 *   Q7  when the chunk length is not a multiple of N, the last round only
 *       involves coders 0 .. (len mod N)-1; idle coders keep state L.
 *   Q8  container: 32-byte header, chunk directory, chunk streams at 16-byte
 *       aligned offsets with zero padding (layout in orc_encode).  Header
 *       byte 9 holds flags: bit 0 breadth-first digit order (Section 5; the
 *       two orders coincide when b >= M), bit 1 escape coding (Q16).
 *   Q16 raw digits (Section 3 says raw data can be mixed into an ANS stream
 *       at agreed points): escape coding of 16-bit symbols.  The model's
 *       last symbol E is an escape; a value v is coded as symbol v when
 *       v < E and f_v > 0, else as E followed by 16/r raw digits holding v
 *       (most significant first); in each coder's share of a step the raw
 *       digits follow the renormalisation digits; depth-first order only.
 *   Q17 Section 4's multiplexer needs a second coder family, which the paper
 *       leaves open: a canonical prefix code with lengths
 *       max(1, ceil(log2(M/f_s))), 16-bit words, a decoder that reads one
 *       word whenever it holds fewer than 16 bits before a symbol.  The N
 *       coders' streams are multiplexed in the order that decoder reads
 *       them; a chunk stream starts with the N coders' bit counts (u32, an
 *       end check) instead of rANS states.  Header byte 9 = 4, r = 16.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

enum {
    ORC_OK = 0,
    ORC_EINVAL = -1,
    ORC_EPREC = -2,
    ORC_ENOSYM = -3,
    ORC_ENOSPC = -4,
    ORC_ECORRUPT = -5,
    ORC_ENOMEM = -6
};

#define ORC_MAGIC 0x534E4172u /* "rANS" read as little-endian bytes */

/* ------------------------------------------------------------------------ */
/* Model: symbol frequencies f_s summing to M = 2^k (Section 2: alphabet and
 * probabilities p_s = f_s / M).                                            */

typedef struct {
    uint32_t n;        /* alphabet size                                  */
    uint32_t k;        /* M = 2^k                                        */
    const uint32_t *f; /* f[s], sum = M                                  */
    uint64_t *cum;     /* cum[s] = f[0] + ... + f[s-1], cum[n] = M        */
    uint32_t *slot;    /* slot[j] = the s with cum[s] <= j < cum[s]+f[s] */
} model_t;

static void model_free(model_t *m)
{
    free(m->cum);
    free(m->slot);
    m->cum = NULL;
    m->slot = NULL;
}

/* Builds cum and the slot->symbol map straight from their definitions. */
static int model_init(model_t *m, const uint32_t *f, uint32_t n, uint32_t k)
{
    uint64_t M, s, j, total = 0;
    m->n = n;
    m->k = k;
    m->f = f;
    m->cum = NULL;
    m->slot = NULL;
    if (n == 0 || k == 0 || k > 16)
        return ORC_EINVAL;
    M = (uint64_t)1 << k;
    for (s = 0; s < n; s++)
        total += f[s];
    if (total != M)
        return ORC_EINVAL;
    m->cum = (uint64_t *)malloc(sizeof(uint64_t) * (n + 1));
    m->slot = (uint32_t *)malloc(sizeof(uint32_t) * M);
    if (!m->cum || !m->slot) {
        model_free(m);
        return ORC_ENOMEM;
    }
    m->cum[0] = 0;
    for (s = 0; s < n; s++)
        m->cum[s + 1] = m->cum[s] + f[s];
    for (s = 0; s < n; s++)
        for (j = m->cum[s]; j < m->cum[s] + f[s]; j++)
            m->slot[j] = (uint32_t)s;
    return ORC_OK;
}

/* C(s, x): encodes symbol s into state x (Section 2, reading Q1). */
static uint64_t coder_C(const model_t *m, uint32_t s, uint64_t x)
{
    uint64_t M = (uint64_t)1 << m->k;
    uint64_t fs = m->f[s];
    return M * (x / fs) + (x % fs) + m->cum[s];
}

/* D(x) = (s, x'): the inverse of C (Section 2, reading Q1). */
static uint32_t coder_D(const model_t *m, uint64_t x, uint64_t *x_prev)
{
    uint64_t M = (uint64_t)1 << m->k;
    uint64_t j = x % M;
    uint32_t s = m->slot[j];
    *x_prev = (uint64_t)m->f[s] * (x / M) + j - m->cum[s];
    return s;
}

/* Coder geometry: b = 2^r, L = 2^l, I = {L, ..., bL-1} (Section 2). */
typedef struct {
    uint64_t b, L;
    uint32_t N;
} geom_t;

static int in_I(const geom_t *g, uint64_t x)
{
    return x >= g->L && x < g->b * g->L;
}

static int check_geometry(uint32_t k, uint32_t r, uint32_t l, uint32_t N)
{
    /* b-uniqueness of the rANS precursor sets needs L to be a multiple of
     * M (Section 2); the state must fit in 32 bits (p = 32, Section 1). */
    if (k < 1 || k > 16 || r < 1 || r > 16 || l < k || l + r > 32 || N < 1)
        return ORC_EINVAL;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Reading Q2: quantise symbol counts to frequencies summing to M = 2^k.
 * Integer largest remainder, deterministic ties (lower symbol index first):
 *   f_s = floor(c_s*M/T), rem_s = c_s*M mod T; a present symbol whose f_s
 *   came out 0 is forced to 1; the deficit d = M - sum(f) goes, +1 each, to
 *   the first d non-forced present symbols ordered by (rem desc, index asc);
 *   an excess is removed one unit at a time from the symbol with the largest
 *   f_s > 1 (lowest index on ties).                                        */

static const uint64_t *g_sort_rem; /* qsort has no context argument */

static int cmp_rem_desc(const void *a, const void *b)
{
    uint32_t i = *(const uint32_t *)a, j = *(const uint32_t *)b;
    if (g_sort_rem[i] != g_sort_rem[j])
        return g_sort_rem[i] > g_sort_rem[j] ? -1 : 1;
    return i < j ? -1 : (i > j ? 1 : 0);
}

static pthread_mutex_t g_sort_lock = PTHREAD_MUTEX_INITIALIZER;

int orc_quantize(const uint64_t *counts, uint32_t n, uint32_t k, uint32_t *f)
{
    uint64_t M, T = 0, present = 0, sum = 0, s;
    uint64_t *rem;
    uint8_t *forced;
    uint32_t *order, norder = 0;
    int64_t d;

    if (n == 0 || k < 1 || k > 16)
        return ORC_EINVAL;
    M = (uint64_t)1 << k;
    for (s = 0; s < n; s++) {
        if (counts[s] >= ((uint64_t)1 << 47))
            return ORC_EINVAL;
        T += counts[s];
        present += counts[s] > 0;
    }
    if (T == 0 || T >= ((uint64_t)1 << 47))
        return ORC_EINVAL;
    if (present > M)
        return ORC_EPREC;

    rem = (uint64_t *)calloc(n, sizeof(uint64_t));
    forced = (uint8_t *)calloc(n, 1);
    order = (uint32_t *)calloc(n, sizeof(uint32_t));
    if (!rem || !forced || !order) {
        free(rem);
        free(forced);
        free(order);
        return ORC_ENOMEM;
    }
    for (s = 0; s < n; s++) {
        f[s] = (uint32_t)(counts[s] * M / T);
        rem[s] = counts[s] * M % T;
        if (counts[s] > 0 && f[s] == 0) {
            f[s] = 1;
            forced[s] = 1;
        }
        sum += f[s];
    }
    d = (int64_t)M - (int64_t)sum;
    if (d > 0) {
        for (s = 0; s < n; s++)
            if (counts[s] > 0 && !forced[s])
                order[norder++] = (uint32_t)s;
        pthread_mutex_lock(&g_sort_lock);
        g_sort_rem = rem;
        qsort(order, norder, sizeof(uint32_t), cmp_rem_desc);
        pthread_mutex_unlock(&g_sort_lock);
        for (s = 0; s < (uint64_t)d && s < norder; s++)
            f[order[s]] += 1;
    }
    while (d < 0) {
        uint64_t best = n;
        for (s = 0; s < n; s++)
            if (f[s] > 1 && (best == n || f[s] > f[best]))
                best = s;
        f[best] -= 1;
        d += 1;
    }
    free(rem);
    free(forced);
    free(order);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Single-function access for brute-force tests on tiny models.            */

uint64_t orc_C(const uint32_t *f, uint32_t n, uint32_t k, uint32_t s, uint64_t x)
{
    model_t m;
    uint64_t y;
    if (model_init(&m, f, n, k) != ORC_OK || s >= n || f[s] == 0)
        return UINT64_MAX;
    y = coder_C(&m, s, x);
    model_free(&m);
    return y;
}

int orc_D(const uint32_t *f, uint32_t n, uint32_t k, uint64_t x, uint32_t *s_out, uint64_t *x_out)
{
    model_t m;
    int rc = model_init(&m, f, n, k);
    if (rc != ORC_OK)
        return rc;
    *s_out = coder_D(&m, x, x_out);
    model_free(&m);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Interleaved chunk coder over an array of digits (one digit per uint32).
 * Stream (decoder order): digits[0 .. ndigits).  States: N values.        */

/* Algorithm 1, Encode, for one symbol on one coder.  Emitted digits are
 * prepended to the stream (the encoder writes backwards): buf[--*pos].   */
static int encode_symbol(const model_t *m, const geom_t *g, uint32_t s, uint64_t *x,
                         uint32_t *buf, uint64_t *pos)
{
    int guard = 0;
    if (s >= m->n || m->f[s] == 0)
        return ORC_ENOSYM;
    while (!in_I(g, coder_C(m, s, *x))) {
        if (*pos == 0)
            return ORC_ENOSPC;
        buf[--*pos] = (uint32_t)(*x % g->b);
        *x = *x / g->b;
        if (++guard > 64)
            return ORC_EINVAL;
    }
    *x = coder_C(m, s, *x);
    return ORC_OK;
}

/* Algorithm 1, Decode, for one symbol on one coder (depth-first reads). */
static int decode_symbol(const model_t *m, const geom_t *g, uint64_t *x, const uint32_t *dig,
                         uint64_t ndig, uint64_t *rd, uint32_t *s_out)
{
    uint64_t y;
    if (!in_I(g, *x))
        return ORC_ECORRUPT; /* Require: x in I */
    *s_out = coder_D(m, *x, &y);
    while (!in_I(g, y)) {
        if (*rd >= ndig)
            return ORC_ECORRUPT;
        y = g->b * y + dig[(*rd)++];
    }
    *x = y;
    return ORC_OK;
}

/* Depth-first interleaved encoder: symbol i goes to coder (i mod N); the
 * message is walked from its last symbol to its first.  On return
 * digits[*start .. cap) holds the stream in decoder order. */
static int encode_df(const model_t *m, const geom_t *g, const uint32_t *syms, uint64_t len,
                     uint64_t *states, uint32_t *digits, uint64_t cap, uint64_t *start,
                     uint64_t *trace)
{
    uint64_t i, pos = cap;
    uint32_t j;
    int rc;
    for (j = 0; j < g->N; j++)
        states[j] = g->L; /* reading Q3 */
    for (i = len; i-- > 0;) {
        j = (uint32_t)(i % g->N);
        rc = encode_symbol(m, g, syms[i], &states[j], digits, &pos);
        if (rc != ORC_OK)
            return rc;
        if (trace)
            trace[i] = states[j];
    }
    *start = pos;
    return ORC_OK;
}

/* Breadth-first interleaved encoder: within one round (the symbols
 * tN .. tN+N-1), the digits of all coders are laid out renormalisation round
 * by renormalisation round (first digit of every coder, then second, ...),
 * which is the order a decoder that loops over the whole vector reads. */
static int encode_bf(const model_t *m, const geom_t *g, const uint32_t *syms, uint64_t len,
                     uint64_t *states, uint32_t *digits, uint64_t cap, uint64_t *start,
                     uint64_t *trace)
{
    uint64_t pos = cap, nsteps, t;
    uint32_t j, q, maxd;
    uint32_t lane_dig[64][64]; /* per coder digits in emit order (<= 64 per symbol) */
    uint32_t lane_nd[64];
    if (g->N > 64)
        return ORC_EINVAL;
    for (j = 0; j < g->N; j++)
        states[j] = g->L;
    nsteps = (len + g->N - 1) / g->N;
    for (t = nsteps; t-- > 0;) {
        uint32_t active = (uint32_t)((len - t * g->N) < g->N ? (len - t * g->N) : g->N);
        maxd = 0;
        for (j = active; j-- > 0;) {
            uint64_t x = states[j];
            uint32_t s = syms[t * g->N + j];
            lane_nd[j] = 0;
            if (s >= m->n || m->f[s] == 0)
                return ORC_ENOSYM;
            while (!in_I(g, coder_C(m, s, x))) {
                if (lane_nd[j] >= 64)
                    return ORC_EINVAL;
                lane_dig[j][lane_nd[j]++] = (uint32_t)(x % g->b);
                x = x / g->b;
            }
            states[j] = coder_C(m, s, x);
            if (trace)
                trace[t * g->N + j] = states[j];
            if (lane_nd[j] > maxd)
                maxd = lane_nd[j];
        }
        /* Decoder read order for this step: q = 0, 1, ...; coders ascending;
         * coder j's q-th read is its (nd-1-q)-th emitted digit.  Prepend the
         * block in reverse read order. */
        for (q = maxd; q-- > 0;) {
            for (j = active; j-- > 0;) {
                if (q < lane_nd[j]) {
                    if (pos == 0)
                        return ORC_ENOSPC;
                    digits[--pos] = lane_dig[j][lane_nd[j] - 1 - q];
                }
            }
        }
    }
    *start = pos;
    return ORC_OK;
}

static int decode_df(const model_t *m, const geom_t *g, const uint64_t *states_in,
                     const uint32_t *dig, uint64_t ndig, uint32_t *syms, uint64_t len,
                     uint64_t *trace)
{
    uint64_t *x, i, rd = 0;
    uint32_t j;
    int rc = ORC_OK;
    x = (uint64_t *)malloc(sizeof(uint64_t) * g->N);
    if (!x)
        return ORC_ENOMEM;
    memcpy(x, states_in, sizeof(uint64_t) * g->N);
    for (i = 0; i < len; i++) {
        j = (uint32_t)(i % g->N);
        rc = decode_symbol(m, g, &x[j], dig, ndig, &rd, &syms[i]);
        if (rc != ORC_OK)
            goto out;
        if (trace)
            trace[i] = x[j];
    }
    /* The decoder retraces the encoder's states in reverse, so it must end
     * where the encoder started (Q3) with the stream fully consumed. */
    for (j = 0; j < g->N; j++)
        if (x[j] != g->L)
            rc = ORC_ECORRUPT;
    if (rd != ndig)
        rc = ORC_ECORRUPT;
out:
    free(x);
    return rc;
}

static int decode_bf(const model_t *m, const geom_t *g, const uint64_t *states_in,
                     const uint32_t *dig, uint64_t ndig, uint32_t *syms, uint64_t len,
                     uint64_t *trace)
{
    uint64_t *x, t, nsteps, rd = 0;
    uint32_t j;
    int rc = ORC_OK, any;
    x = (uint64_t *)malloc(sizeof(uint64_t) * g->N);
    if (!x)
        return ORC_ENOMEM;
    memcpy(x, states_in, sizeof(uint64_t) * g->N);
    nsteps = (len + g->N - 1) / g->N;
    for (t = 0; t < nsteps; t++) {
        uint32_t active = (uint32_t)((len - t * g->N) < g->N ? (len - t * g->N) : g->N);
        for (j = 0; j < active; j++) {
            uint64_t y;
            if (!in_I(g, x[j])) {
                rc = ORC_ECORRUPT;
                goto out;
            }
            syms[t * g->N + j] = coder_D(m, x[j], &y);
            x[j] = y;
        }
        do {
            any = 0;
            for (j = 0; j < active; j++) {
                if (x[j] < g->L) {
                    if (rd >= ndig) {
                        rc = ORC_ECORRUPT;
                        goto out;
                    }
                    x[j] = g->b * x[j] + dig[rd++];
                    any = 1;
                }
            }
        } while (any);
        if (trace)
            for (j = 0; j < active; j++)
                trace[t * g->N + j] = x[j];
    }
    for (j = 0; j < g->N; j++)
        if (x[j] != g->L)
            rc = ORC_ECORRUPT;
    if (rd != ndig)
        rc = ORC_ECORRUPT;
out:
    free(x);
    return rc;
}

/* Escape coding with raw digits (Section 3: because decoder and encoder run
 * in lockstep, an encoder may put raw digits into the stream at any point
 * both sides agree on, with no bypass mechanism).  The model's last symbol
 * E = n - 1 is the escape: a value v is coded as the symbol v when v < E and
 * f_v > 0, and otherwise as E plus nraw raw digits that hold v, most
 * significant first in stream order.  The encoder sends the raw digits just
 * before it encodes the escape, so the decoder reads them just after it has
 * decoded the escape and renormalised: per coder and step the stream holds
 * the symbol's renormalisation digits, then its raw digits.  Depth-first
 * order, coders ascending (reading Q16). */
static int encode_esc(const model_t *m, const geom_t *g, uint32_t nraw, const uint32_t *vals,
                      uint64_t len, uint64_t *states, uint32_t *digits, uint64_t cap,
                      uint64_t *start)
{
    uint64_t i, pos = cap;
    uint32_t j, q, E = m->n - 1;
    int rc;
    for (j = 0; j < g->N; j++)
        states[j] = g->L; /* reading Q3 */
    for (i = len; i-- > 0;) {
        uint32_t v = vals[i], s = v;
        j = (uint32_t)(i % g->N);
        if (v >= E || m->f[v] == 0) {
            uint64_t rest = v;
            for (q = 0; q < nraw; q++) { /* least significant digit is prepended first */
                if (pos == 0)
                    return ORC_ENOSPC;
                digits[--pos] = (uint32_t)(rest % g->b);
                rest /= g->b;
            }
            s = E;
        }
        rc = encode_symbol(m, g, s, &states[j], digits, &pos);
        if (rc != ORC_OK)
            return rc;
    }
    *start = pos;
    return ORC_OK;
}

static int decode_esc(const model_t *m, const geom_t *g, uint32_t nraw, const uint64_t *states_in,
                      const uint32_t *dig, uint64_t ndig, uint32_t *vals, uint64_t len)
{
    uint64_t *x, i, rd = 0;
    uint32_t j, q, s, E = m->n - 1;
    int rc = ORC_OK;
    x = (uint64_t *)malloc(sizeof(uint64_t) * g->N);
    if (!x)
        return ORC_ENOMEM;
    memcpy(x, states_in, sizeof(uint64_t) * g->N);
    for (i = 0; i < len; i++) {
        j = (uint32_t)(i % g->N);
        rc = decode_symbol(m, g, &x[j], dig, ndig, &rd, &s);
        if (rc != ORC_OK)
            goto out;
        if (s == E) {
            uint64_t v = 0;
            for (q = 0; q < nraw; q++) {
                if (rd >= ndig) {
                    rc = ORC_ECORRUPT;
                    goto out;
                }
                v = v * g->b + dig[rd++];
            }
            vals[i] = (uint32_t)v;
        } else {
            vals[i] = s;
        }
    }
    for (j = 0; j < g->N; j++)
        if (x[j] != g->L)
            rc = ORC_ECORRUPT;
    if (rd != ndig)
        rc = ORC_ECORRUPT;
out:
    free(x);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* A second coder family for Section 4's multiplexer (reading Q17): a static
 * canonical prefix code.  Code lengths come from the quantised frequencies,
 * len_s = max(1, ceil(log2(M / f_s))) for f_s > 0 and none for f_s = 0, so
 * sum 2^-len_s <= sum f_s / M = 1 (Kraft) and len_s <= k.  Codes are
 * canonical: symbols ordered by (length, index) take consecutive values, the
 * value doubling whenever the length grows.  Bits are written most
 * significant first into 16-bit words. */
typedef struct {
    uint32_t n, maxlen;
    uint32_t *len, *code;
    uint32_t first[17], count[17], start[17]; /* canonical decoding, per length */
    uint32_t *sorted;                         /* symbols by (length, index)     */
} pfx_t;

static void pfx_free(pfx_t *c)
{
    free(c->len);
    free(c->code);
    free(c->sorted);
}

static int pfx_init(pfx_t *c, const uint32_t *f, uint32_t n, uint32_t k)
{
    uint64_t M = (uint64_t)1 << k;
    uint32_t s, l, next = 0, m = 0;
    memset(c, 0, sizeof(*c));
    if (n == 0 || k < 1 || k > 16)
        return ORC_EINVAL;
    c->n = n;
    c->len = (uint32_t *)calloc(n, sizeof(uint32_t));
    c->code = (uint32_t *)calloc(n, sizeof(uint32_t));
    c->sorted = (uint32_t *)calloc(n, sizeof(uint32_t));
    if (!c->len || !c->code || !c->sorted) {
        pfx_free(c);
        return ORC_ENOMEM;
    }
    for (s = 0; s < n; s++) {
        if (f[s] == 0)
            continue;
        l = 0;
        while ((uint64_t)f[s] << l < M) /* smallest l with f 2^l >= M */
            l++;
        c->len[s] = l < 1 ? 1 : l;
        if (c->len[s] > c->maxlen)
            c->maxlen = c->len[s];
    }
    for (l = 1; l <= c->maxlen; l++) {
        c->first[l] = next;
        c->start[l] = m;
        for (s = 0; s < n; s++)
            if (c->len[s] == l) {
                c->code[s] = next++;
                c->sorted[m++] = s;
                c->count[l]++;
            }
        next <<= 1;
    }
    return ORC_OK;
}

/* Bit reader of one coder's decoder: before each symbol, while fewer than
 * 16 bits are buffered it reads one 16-bit word (one at most, since a code
 * has at most 16 bits); the symbol is the one whose code equals the next
 * len bits for the length len that matches (canonical decoding). */
typedef struct {
    uint64_t buf;
    uint32_t nb;
    uint64_t used; /* bits consumed */
} bitrd_t;

static int pfx_decode_symbol(const pfx_t *c, bitrd_t *d, uint32_t *s_out)
{
    uint32_t l;
    for (l = 1; l <= c->maxlen && l <= d->nb; l++) {
        uint32_t v = (uint32_t)((d->buf >> (d->nb - l)) & (((uint64_t)1 << l) - 1));
        if (v >= c->first[l] && v - c->first[l] < c->count[l]) {
            *s_out = c->sorted[c->start[l] + (v - c->first[l])];
            d->nb -= l;
            d->buf &= ((uint64_t)1 << d->nb) - 1;
            d->used += l;
            return ORC_OK;
        }
    }
    return ORC_ECORRUPT;
}

/* Encodes one chunk with N prefix coders (symbol i -> coder i mod N), each
 * into a stream of its own, then multiplexes them by running the
 * instrumented decoder of Section 4: the N decoders run in the decoding
 * order (steps, coders ascending), and every word one of them reads from its
 * own stream is appended to the multiplexed stream at once.  bits[j] receives
 * coder j's code bits; words[0 .. *nwords) the multiplexed stream. */
static int encode_pfx(const pfx_t *c, uint32_t N, const uint32_t *syms, uint64_t len,
                      uint64_t *bits, uint32_t *words, uint64_t cap, uint64_t *nwords)
{
    uint32_t **st = (uint32_t **)calloc(N, sizeof(uint32_t *));
    uint64_t *nst = (uint64_t *)calloc(N, sizeof(uint64_t)), *rd = (uint64_t *)calloc(N, sizeof(uint64_t));
    bitrd_t *dec = (bitrd_t *)calloc(N, sizeof(bitrd_t));
    uint64_t i, m = 0, per = len / N + 2;
    uint32_t j;
    int rc = ORC_OK;
    if (!st || !nst || !rd || !dec) {
        rc = ORC_ENOMEM;
        goto out;
    }
    /* 1. each coder writes its symbols' codes into its own stream */
    for (j = 0; j < N; j++) {
        uint64_t acc = 0, t;
        uint32_t nacc = 0;
        st[j] = (uint32_t *)calloc(per + 2, sizeof(uint32_t)); /* <= 16 bits per symbol */
        if (!st[j]) {
            rc = ORC_ENOMEM;
            goto out;
        }
        bits[j] = 0;
        for (t = j; t < len; t += N) {
            uint32_t s = syms[t];
            if (s >= c->n || c->len[s] == 0) {
                rc = ORC_ENOSYM;
                goto out;
            }
            acc = (acc << c->len[s]) | c->code[s];
            nacc += c->len[s];
            bits[j] += c->len[s];
            while (nacc >= 16) {
                st[j][nst[j]++] = (uint32_t)(acc >> (nacc - 16)) & 0xFFFF;
                nacc -= 16;
                acc &= ((uint64_t)1 << nacc) - 1;
            }
        }
        if (nacc > 0) /* the last word, zero padded */
            st[j][nst[j]++] = (uint32_t)(acc << (16 - nacc)) & 0xFFFF;
        /* the decoder may read one more word than the bits fill: a word of
         * zeros (st was zero-initialised), present as long as it is read */
        nst[j]++;
    }
    /* 2. the instrumented decoder */
    for (i = 0; i < len; i++) {
        uint32_t s;
        j = (uint32_t)(i % N);
        if (dec[j].nb < 16) {
            uint32_t w;
            if (rd[j] >= nst[j]) {
                rc = ORC_EINVAL;
                goto out;
            }
            w = st[j][rd[j]++];
            if (m >= cap) {
                rc = ORC_ENOSPC;
                goto out;
            }
            words[m++] = w; /* what the decoder reads, in the order it reads it */
            dec[j].buf = (dec[j].buf << 16) | w;
            dec[j].nb += 16;
        }
        rc = pfx_decode_symbol(c, &dec[j], &s);
        if (rc != ORC_OK || s != syms[i]) {
            rc = ORC_EINVAL;
            goto out;
        }
    }
    *nwords = m;
out:
    if (st)
        for (j = 0; j < N; j++)
            free(st[j]);
    free(st);
    free(nst);
    free(rd);
    free(dec);
    return rc;
}

/* Decodes one chunk from the multiplexed stream: the same decoders, reading
 * one shared stream.  End check: every coder consumed exactly bits[j] bits
 * and the stream is exhausted. */
static int decode_pfx(const pfx_t *c, uint32_t N, const uint64_t *bits, const uint32_t *words,
                      uint64_t nwords, uint32_t *syms, uint64_t len)
{
    bitrd_t *dec = (bitrd_t *)calloc(N, sizeof(bitrd_t));
    uint64_t i, rd = 0;
    uint32_t j;
    int rc = ORC_OK;
    if (!dec)
        return ORC_ENOMEM;
    for (i = 0; i < len; i++) {
        j = (uint32_t)(i % N);
        if (dec[j].nb < 16) {
            if (rd >= nwords) {
                rc = ORC_ECORRUPT;
                goto out;
            }
            dec[j].buf = (dec[j].buf << 16) | words[rd++];
            dec[j].nb += 16;
        }
        rc = pfx_decode_symbol(c, &dec[j], &syms[i]);
        if (rc != ORC_OK)
            goto out;
    }
    for (j = 0; j < N; j++)
        if (dec[j].used != bits[j])
            rc = ORC_ECORRUPT;
    if (rd != nwords)
        rc = ORC_ECORRUPT;
out:
    free(dec);
    return rc;
}

/* Code lengths and code values of the prefix code (tests). */
int orc_pfx_code(const uint32_t *f, uint32_t n, uint32_t k, uint32_t *len, uint32_t *code)
{
    pfx_t c;
    int rc = pfx_init(&c, f, n, k);
    if (rc != ORC_OK)
        return rc;
    memcpy(len, c.len, sizeof(uint32_t) * n);
    memcpy(code, c.code, sizeof(uint32_t) * n);
    pfx_free(&c);
    return ORC_OK;
}

/* Digit-level entry points (tests).  order: 0 = depth-first, 1 = breadth-
 * first.  digits: caller buffer of cap entries; on success the stream is
 * moved to digits[0 .. *ndigits).  trace (optional, len entries): state of
 * the owning coder after symbol i was coded. */
int orc_encode_digits(const uint32_t *f, uint32_t n, uint32_t k, uint32_t r, uint32_t l,
                      uint32_t N, int order, const uint32_t *syms, uint64_t len,
                      uint64_t *states, uint32_t *digits, uint64_t cap, uint64_t *ndigits,
                      uint64_t *trace)
{
    model_t m;
    geom_t g;
    uint64_t start = 0;
    int rc = check_geometry(k, r, l, N);
    if (rc != ORC_OK)
        return rc;
    rc = model_init(&m, f, n, k);
    if (rc != ORC_OK)
        return rc;
    g.b = (uint64_t)1 << r;
    g.L = (uint64_t)1 << l;
    g.N = N;
    rc = order ? encode_bf(&m, &g, syms, len, states, digits, cap, &start, trace)
               : encode_df(&m, &g, syms, len, states, digits, cap, &start, trace);
    if (rc == ORC_OK) {
        *ndigits = cap - start;
        memmove(digits, digits + start, sizeof(uint32_t) * (cap - start));
    }
    model_free(&m);
    return rc;
}

int orc_decode_digits(const uint32_t *f, uint32_t n, uint32_t k, uint32_t r, uint32_t l,
                      uint32_t N, int order, const uint64_t *states, const uint32_t *digits,
                      uint64_t ndigits, uint32_t *syms, uint64_t len, uint64_t *trace)
{
    model_t m;
    geom_t g;
    int rc = check_geometry(k, r, l, N);
    if (rc != ORC_OK)
        return rc;
    rc = model_init(&m, f, n, k);
    if (rc != ORC_OK)
        return rc;
    g.b = (uint64_t)1 << r;
    g.L = (uint64_t)1 << l;
    g.N = N;
    rc = order ? decode_bf(&m, &g, states, digits, ndigits, syms, len, trace)
               : decode_df(&m, &g, states, digits, ndigits, syms, len, trace);
    model_free(&m);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Container (reading Q8), all fields little-endian:
 *   header, 32 bytes:
 *     0: u32 magic   4: u8 version=1   5: u8 k   6: u8 r   7: u8 l
 *     8: u8 w (symbol bytes)   9: u8 flags (bit 0 breadth-first digit order,
 *     bit 1 escape coding, not both; reading Q16)   10: u16 N   12: u32 C (symbols per
 *     chunk)   16: u64 n (symbols)   24: u32 n_chunks = ceil(n/C)   28: u32 0
 *   directory at 32: n_chunks entries {u64 offset, u32 length, u32 0}
 *   chunk streams at 16-byte aligned offsets, zero padding in between;
 *   the first one at align16(32 + 16*n_chunks).
 *   chunk stream: N x u32 final states, then the digits (u16 words for
 *   r = 16, bytes for r = 8) in decoder order.                            */

static void put_u16(uint8_t *p, uint32_t v) { p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); }
static void put_u32(uint8_t *p, uint32_t v)
{
    put_u16(p, v & 0xFFFF);
    put_u16(p + 2, v >> 16);
}
static void put_u64(uint8_t *p, uint64_t v)
{
    put_u32(p, (uint32_t)v);
    put_u32(p + 4, (uint32_t)(v >> 32));
}
static uint32_t get_u16(const uint8_t *p) { return (uint32_t)p[0] | ((uint32_t)p[1] << 8); }
static uint32_t get_u32(const uint8_t *p) { return get_u16(p) | (get_u16(p + 2) << 16); }
static uint64_t get_u64(const uint8_t *p) { return get_u32(p) | ((uint64_t)get_u32(p + 4) << 32); }
static uint64_t align16(uint64_t v) { return (v + 15) & ~(uint64_t)15; }

static uint32_t get_sym(const uint8_t *p, uint32_t w, uint64_t i)
{
    return w == 1 ? p[i] : get_u16(p + 2 * i);
}
static void put_sym(uint8_t *p, uint32_t w, uint64_t i, uint32_t s)
{
    if (w == 1)
        p[i] = (uint8_t)s;
    else
        put_u16(p + 2 * i, s);
}

static int check_container_params(uint32_t k, uint32_t r, uint32_t l, uint32_t w, uint32_t N)
{
    if (check_geometry(k, r, l, N) != ORC_OK)
        return ORC_EINVAL;
    if ((r != 8 && r != 16) || (w != 1 && w != 2) || N > 65535)
        return ORC_EINVAL;
    return ORC_OK;
}

/* digits a single symbol can emit: the state shrinks below b*f_s*L/M after
 * at most ceil(k/r) divisions by b. */
static uint64_t max_digits_per_symbol(uint32_t k, uint32_t r) { return (k + r - 1) / r; }

/* nraw: raw digits an escaped symbol adds (0 without escape coding). */
uint64_t orc_encode_bound_raw(uint64_t nsyms, uint32_t k, uint32_t r, uint32_t N, uint32_t C,
                              uint32_t nraw)
{
    uint64_t nch, c, total, per;
    if (C == 0)
        C = nsyms > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)nsyms;
    if (nsyms == 0 || C == 0)
        return 32;
    nch = (nsyms + C - 1) / C;
    total = align16(32 + 16 * nch);
    per = (max_digits_per_symbol(k, r) + nraw) * (r / 8);
    for (c = 0; c < nch; c++) {
        uint64_t len = (c + 1 == nch) ? nsyms - c * (uint64_t)C : C;
        total += align16(4ull * N + per * len);
    }
    return total;
}

uint64_t orc_encode_bound(uint64_t nsyms, uint32_t k, uint32_t r, uint32_t N, uint32_t C)
{
    return orc_encode_bound_raw(nsyms, k, r, N, C, 0);
}

typedef struct {
    const model_t *m;
    geom_t g;
    uint32_t r, w, C;
    int order;     /* 0 depth-first, 1 breadth-first */
    uint32_t nraw; /* escape coding: raw digits per escaped value; 0 = off */
    const pfx_t *pc; /* prefix-code family (Section 4 multiplexer), or NULL */
    const uint8_t *syms;
    uint64_t nsyms, nch;
    uint8_t **chunk_bytes;
    uint64_t *chunk_len;
    const uint8_t *in;
    uint64_t in_len;
    uint8_t *out_syms;
    const void *hdr;
    int tid, nthreads;
    int rc;
} job_t;

static void *encode_worker(void *arg)
{
    job_t *jb = (job_t *)arg;
    uint64_t c;
    uint32_t *syms = (uint32_t *)malloc(sizeof(uint32_t) * (jb->C ? jb->C : 1));
    uint64_t cap = (max_digits_per_symbol(jb->m->k, jb->r) + jb->nraw) * jb->C + jb->g.N + 1;
    uint32_t *dig = (uint32_t *)malloc(sizeof(uint32_t) * cap);
    uint64_t *states = (uint64_t *)malloc(sizeof(uint64_t) * jb->g.N);
    jb->rc = ORC_OK;
    if (!syms || !dig || !states) {
        jb->rc = ORC_ENOMEM;
        goto out;
    }
    for (c = (uint64_t)jb->tid; c < jb->nch; c += (uint64_t)jb->nthreads) {
        uint64_t base = c * jb->C, len = jb->nsyms - base < jb->C ? jb->nsyms - base : jb->C;
        uint64_t i, start, nd, bytes;
        uint8_t *p;
        uint32_t j;
        int rc;
        for (i = 0; i < len; i++)
            syms[i] = get_sym(jb->syms, jb->w, base + i);
        if (jb->pc) {
            /* multiplexed words go to the front of dig: at most one per
             * symbol plus one per coder */
            uint64_t nw = 0;
            if (cap < len + jb->g.N) {
                jb->rc = ORC_EINVAL;
                goto out;
            }
            rc = encode_pfx(jb->pc, jb->g.N, syms, len, states, dig, cap, &nw);
            if (rc == ORC_OK) {
                memmove(dig + (cap - nw), dig, sizeof(uint32_t) * nw);
                start = cap - nw;
            }
        } else if (jb->nraw)
            rc = encode_esc(jb->m, &jb->g, jb->nraw, syms, len, states, dig, cap, &start);
        else if (jb->order)
            rc = encode_bf(jb->m, &jb->g, syms, len, states, dig, cap, &start, NULL);
        else
            rc = encode_df(jb->m, &jb->g, syms, len, states, dig, cap, &start, NULL);
        if (rc != ORC_OK) {
            jb->rc = rc;
            goto out;
        }
        nd = cap - start;
        bytes = 4ull * jb->g.N + nd * (jb->r / 8);
        p = (uint8_t *)malloc(bytes ? bytes : 1);
        if (!p) {
            jb->rc = ORC_ENOMEM;
            goto out;
        }
        for (j = 0; j < jb->g.N; j++)
            put_u32(p + 4ull * j, (uint32_t)states[j]);
        for (i = 0; i < nd; i++) {
            if (jb->r == 16)
                put_u16(p + 4ull * jb->g.N + 2 * i, dig[start + i]);
            else
                p[4ull * jb->g.N + i] = (uint8_t)dig[start + i];
        }
        jb->chunk_bytes[c] = p;
        jb->chunk_len[c] = bytes;
    }
out:
    free(syms);
    free(dig);
    free(states);
    return NULL;
}

static int run_workers(job_t *proto, int nthreads, void *(*fn)(void *))
{
    job_t *jobs;
    pthread_t *th;
    int t, rc = ORC_OK;
    if (nthreads < 1)
        nthreads = 1;
    jobs = (job_t *)malloc(sizeof(job_t) * nthreads);
    th = (pthread_t *)malloc(sizeof(pthread_t) * nthreads);
    if (!jobs || !th) {
        free(jobs);
        free(th);
        return ORC_ENOMEM;
    }
    for (t = 0; t < nthreads; t++) {
        jobs[t] = *proto;
        jobs[t].tid = t;
        jobs[t].nthreads = nthreads;
    }
    if (nthreads == 1) {
        fn(&jobs[0]);
    } else {
        for (t = 0; t < nthreads; t++)
            pthread_create(&th[t], NULL, fn, &jobs[t]);
        for (t = 0; t < nthreads; t++)
            pthread_join(th[t], NULL);
    }
    for (t = 0; t < nthreads; t++)
        if (jobs[t].rc != ORC_OK)
            rc = jobs[t].rc;
    free(jobs);
    free(th);
    return rc;
}

/* Raw digits an escaped w-byte value takes (all 8w bits). */
static uint32_t raw_digits(uint32_t w, uint32_t r) { return (8 * w + r - 1) / r; }

/* Encodes nsyms symbols (w bytes each, little-endian) into a container.
 * flags (header byte 9): bit 0 breadth-first digit order, bit 1 escape
 * coding (16-bit symbols, depth-first only), bit 2 the prefix-code family
 * multiplexed by the instrumented decoder (r = 16; alone). */
int orc_encode_flags(const uint32_t *f, uint32_t n_alpha, uint32_t k, uint32_t r, uint32_t l,
                     uint32_t w, uint32_t N, uint32_t C, int flags, const uint8_t *syms,
                     uint64_t nsyms, uint8_t *out, uint64_t cap, uint64_t *out_len, int nthreads)
{
    model_t m;
    pfx_t pc;
    job_t jb;
    uint64_t nch, c, off, total;
    int rc = check_container_params(k, r, l, w, N);
    if (rc != ORC_OK)
        return rc;
    if (flags != 0 && flags != 1 && flags != 2 && flags != 4)
        return ORC_EINVAL;
    if ((flags == 2 && w != 2) || (flags == 4 && r != 16))
        return ORC_EINVAL;
    if (C == 0) {
        if (nsyms > 0xFFFFFFFFull)
            return ORC_EINVAL;
        C = (uint32_t)nsyms;
    }
    nch = (nsyms == 0) ? 0 : (nsyms + C - 1) / C;
    if (nch > 0xFFFFFFFFull)
        return ORC_EINVAL;
    rc = model_init(&m, f, n_alpha, k);
    if (rc != ORC_OK)
        return rc;
    memset(&jb, 0, sizeof(jb));
    if (flags == 4) {
        rc = pfx_init(&pc, f, n_alpha, k);
        if (rc != ORC_OK) {
            model_free(&m);
            return rc;
        }
        jb.pc = &pc;
    }
    jb.m = &m;
    jb.g.b = (uint64_t)1 << r;
    jb.g.L = (uint64_t)1 << l;
    jb.g.N = N;
    jb.r = r;
    jb.w = w;
    jb.C = C;
    jb.order = flags & 1;
    jb.nraw = (flags & 2) ? raw_digits(w, r) : 0;
    jb.syms = syms;
    jb.nsyms = nsyms;
    jb.nch = nch;
    jb.chunk_bytes = (uint8_t **)calloc(nch ? nch : 1, sizeof(uint8_t *));
    jb.chunk_len = (uint64_t *)calloc(nch ? nch : 1, sizeof(uint64_t));
    if (!jb.chunk_bytes || !jb.chunk_len) {
        rc = ORC_ENOMEM;
        goto out;
    }
    if (nch > 0) {
        rc = run_workers(&jb, nthreads, encode_worker);
        if (rc != ORC_OK)
            goto out;
    }
    total = align16(32 + 16 * nch);
    for (c = 0; c < nch; c++)
        total = align16(total + jb.chunk_len[c]);
    if (nch == 0)
        total = 32;
    *out_len = total;
    if (total > cap) {
        rc = ORC_ENOSPC;
        goto out;
    }
    memset(out, 0, total);
    put_u32(out + 0, ORC_MAGIC);
    out[4] = 1;
    out[5] = (uint8_t)k;
    out[6] = (uint8_t)r;
    out[7] = (uint8_t)l;
    out[8] = (uint8_t)w;
    out[9] = (uint8_t)flags;
    put_u16(out + 10, N);
    put_u32(out + 12, C);
    put_u64(out + 16, nsyms);
    put_u32(out + 24, (uint32_t)nch);
    put_u32(out + 28, 0);
    off = align16(32 + 16 * nch);
    for (c = 0; c < nch; c++) {
        put_u64(out + 32 + 16 * c, off);
        put_u32(out + 32 + 16 * c + 8, (uint32_t)jb.chunk_len[c]);
        put_u32(out + 32 + 16 * c + 12, 0);
        memcpy(out + off, jb.chunk_bytes[c], jb.chunk_len[c]);
        off = align16(off + jb.chunk_len[c]);
    }
out:
    if (jb.chunk_bytes)
        for (c = 0; c < nch; c++)
            free(jb.chunk_bytes[c]);
    free(jb.chunk_bytes);
    free(jb.chunk_len);
    if (jb.pc)
        pfx_free(&pc);
    model_free(&m);
    return rc;
}

/* Container with digit order `order` (0 depth-first, 1 breadth-first). */
int orc_encode_order(const uint32_t *f, uint32_t n_alpha, uint32_t k, uint32_t r, uint32_t l,
                     uint32_t w, uint32_t N, uint32_t C, int order, const uint8_t *syms,
                     uint64_t nsyms, uint8_t *out, uint64_t cap, uint64_t *out_len, int nthreads)
{
    if (order != 0 && order != 1)
        return ORC_EINVAL;
    return orc_encode_flags(f, n_alpha, k, r, l, w, N, C, order, syms, nsyms, out, cap, out_len,
                            nthreads);
}

/* Depth-first container (the digit order every caller used before the order
 * byte existed). */
int orc_encode(const uint32_t *f, uint32_t n_alpha, uint32_t k, uint32_t r, uint32_t l,
               uint32_t w, uint32_t N, uint32_t C, const uint8_t *syms, uint64_t nsyms,
               uint8_t *out, uint64_t cap, uint64_t *out_len, int nthreads)
{
    return orc_encode_order(f, n_alpha, k, r, l, w, N, C, 0, syms, nsyms, out, cap, out_len,
                            nthreads);
}

typedef struct {
    uint32_t k, r, l, w, N, C, order, nraw, pfx;
    uint64_t n, nch;
} hdr_t;

static int parse_header(const uint8_t *in, uint64_t in_len, hdr_t *h)
{
    if (in_len < 32 || get_u32(in) != ORC_MAGIC || in[4] != 1 ||
        (in[9] != 0 && in[9] != 1 && in[9] != 2 && in[9] != 4) || (in[9] == 2 && in[8] != 2) ||
        (in[9] == 4 && in[6] != 16))
        return ORC_ECORRUPT;
    h->order = in[9] & 1;
    h->pfx = in[9] == 4;
    h->k = in[5];
    h->r = in[6];
    h->l = in[7];
    h->w = in[8];
    h->N = get_u16(in + 10);
    h->C = get_u32(in + 12);
    h->n = get_u64(in + 16);
    h->nch = get_u32(in + 24);
    if (check_container_params(h->k, h->r, h->l, h->w, h->N) != ORC_OK)
        return ORC_ECORRUPT;
    h->nraw = (in[9] & 2) ? raw_digits(h->w, h->r) : 0;
    if (h->n == 0 ? h->nch != 0 : (h->C == 0 || h->nch != (h->n + h->C - 1) / h->C))
        return ORC_ECORRUPT;
    if (32 + 16 * h->nch > in_len)
        return ORC_ECORRUPT;
    return ORC_OK;
}

/* Reads the header fields: out[0..10] = k, r, l, w, N, C, n, n_chunks, digit
 * order, raw digits per escaped value (0: no escape coding), prefix-code
 * family (0/1). */
int orc_header(const uint8_t *in, uint64_t in_len, uint64_t *out)
{
    hdr_t h;
    int rc = parse_header(in, in_len, &h);
    if (rc != ORC_OK)
        return rc;
    out[0] = h.k;
    out[1] = h.r;
    out[2] = h.l;
    out[3] = h.w;
    out[4] = h.N;
    out[5] = h.C;
    out[6] = h.n;
    out[7] = h.nch;
    out[8] = h.order;
    out[9] = h.nraw;
    out[10] = h.pfx;
    return ORC_OK;
}

static void *decode_worker(void *arg)
{
    job_t *jb = (job_t *)arg;
    const hdr_t *h = (const hdr_t *)jb->hdr;
    uint64_t c;
    uint32_t *syms = (uint32_t *)malloc(sizeof(uint32_t) * (h->C ? h->C : 1));
    uint64_t cap = (max_digits_per_symbol(h->k, h->r) + h->nraw) * h->C + h->N + 1;
    uint32_t *dig = (uint32_t *)malloc(sizeof(uint32_t) * cap);
    uint64_t *states = (uint64_t *)malloc(sizeof(uint64_t) * h->N);
    jb->rc = ORC_OK;
    if (!syms || !dig || !states) {
        jb->rc = ORC_ENOMEM;
        goto out;
    }
    for (c = (uint64_t)jb->tid; c < h->nch; c += (uint64_t)jb->nthreads) {
        uint64_t off = get_u64(jb->in + 32 + 16 * c);
        uint64_t len = get_u32(jb->in + 32 + 16 * c + 8);
        uint64_t base = c * h->C, nsy = h->n - base < h->C ? h->n - base : h->C;
        uint64_t nd, i;
        uint32_t j;
        int rc;
        if (off > jb->in_len || len > jb->in_len - off || len < 4ull * h->N ||
            (len - 4ull * h->N) % (h->r / 8) != 0) {
            jb->rc = ORC_ECORRUPT;
            goto out;
        }
        nd = (len - 4ull * h->N) / (h->r / 8);
        if (nd > cap) {
            jb->rc = ORC_ECORRUPT;
            goto out;
        }
        for (j = 0; j < h->N; j++)
            states[j] = get_u32(jb->in + off + 4ull * j);
        for (i = 0; i < nd; i++)
            dig[i] = h->r == 16 ? get_u16(jb->in + off + 4ull * h->N + 2 * i)
                                : jb->in[off + 4ull * h->N + i];
        if (h->pfx)
            rc = decode_pfx(jb->pc, h->N, states, dig, nd, syms, nsy);
        else if (h->nraw)
            rc = decode_esc(jb->m, &jb->g, h->nraw, states, dig, nd, syms, nsy);
        else if (h->order)
            rc = decode_bf(jb->m, &jb->g, states, dig, nd, syms, nsy, NULL);
        else
            rc = decode_df(jb->m, &jb->g, states, dig, nd, syms, nsy, NULL);
        if (rc != ORC_OK) {
            jb->rc = rc;
            goto out;
        }
        for (i = 0; i < nsy; i++)
            put_sym(jb->out_syms, h->w, base + i, syms[i]);
    }
out:
    free(syms);
    free(dig);
    free(states);
    return NULL;
}

/* Decodes a container; symbols are written as w-byte little-endian values. */
int orc_decode(const uint32_t *f, uint32_t n_alpha, const uint8_t *in, uint64_t in_len,
               uint8_t *out_syms, uint64_t cap_syms, uint64_t *nsyms, int nthreads)
{
    model_t m;
    pfx_t pc;
    job_t jb;
    hdr_t h;
    uint64_t s;
    int rc = parse_header(in, in_len, &h);
    if (rc != ORC_OK)
        return rc;
    *nsyms = h.n;
    if (h.n > cap_syms)
        return ORC_ENOSPC;
    if (h.nch == 0)
        return ORC_OK;
    for (s = 0; s < n_alpha; s++)
        if (h.w == 1 && s >= 256 && f[s] != 0)
            return ORC_EINVAL;
    rc = model_init(&m, f, n_alpha, h.k);
    if (rc != ORC_OK)
        return rc;
    memset(&jb, 0, sizeof(jb));
    if (h.pfx) {
        rc = pfx_init(&pc, f, n_alpha, h.k);
        if (rc != ORC_OK) {
            model_free(&m);
            return rc;
        }
        jb.pc = &pc;
    }
    jb.m = &m;
    jb.g.b = (uint64_t)1 << h.r;
    jb.g.L = (uint64_t)1 << h.l;
    jb.g.N = h.N;
    jb.r = h.r;
    jb.w = h.w;
    jb.C = h.C;
    jb.in = in;
    jb.in_len = in_len;
    jb.out_syms = out_syms;
    jb.hdr = &h;
    rc = run_workers(&jb, nthreads, decode_worker);
    if (jb.pc)
        pfx_free(&pc);
    model_free(&m);
    return rc;
}
