/*
 * Oracle for windowed GenASM alignment (Scrooge, arXiv 2208.09985).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code with the GPU library.
 *
 * It is the plainest form of the method, written for checking by eye:
 *   - GenASM-DC exactly as Algorithm 1 (Section 2.2.1): the full
 *     (n_w+1) x (k_w+1) table R of m_w-bit bitvectors, no early termination,
 *     no discarded entries.  Bit j of a pattern-indexed bitvector is stored at
 *     machine bit (m_w-1-j), so j = 0 is the most significant bit, as in the
 *     paper ("msb", "first bit (j=0)").  A shift "<< 1" moves bit j+1 into
 *     bit j and brings a 0 into bit m_w-1.
 *   - pattern masks as defined in Section 2.2.1: PM[X] has a 0 at bit j iff
 *     pattern[j] == X.
 *   - GenASM-TB (Section 2.2.2): from the 0 in the msb of R[0][d_w], follow a
 *     0 through the update terms M, S, I, D (first available in that order)
 *     toward the north-east, recording each crossed term as an operation.
 *     The four terms are regenerated from stored entries with the update
 *     rules of Algorithm 1 (the SENE idea, Section 2.4.1), which is the same
 *     information GenASM stores as edges.
 *   - the windowing heuristic (Section 2.2.3): each window aligns a prefix of
 *     at most W characters of both sequences; traceback stops once W-O
 *     characters of text or of pattern are consumed (Section 2.4.2, Fig. DENT)
 *     or the window's pattern is exhausted; the next window starts after the
 *     consumed characters.
 *
 * Readings where the paper is silent (listed with reasons in the design notes):
 *   k_w = min(k, m_w); a window with no msb 0 in rows 0..k_w makes the pair
 *   NOT_ALIGNED; traceback priority M > S > I > D; the cap applies in every
 *   window including the last; edits = number of non-M operations emitted;
 *   trailing text is free (text_end reports how much text was consumed).
 *
 * Window widths: W up to 128.  A pattern-indexed bitvector is a uint64_t for
 * W <= 64 and an unsigned __int128 above; the algorithm is written once, in
 * oracle_width.inc, and instantiated for both types.
 *
 * Operation codes: 0 = M (match), 1 = S (substitution), 2 = I (pattern
 * character not in text), 3 = D (text character not in pattern).
 *
 * Work counters follow the supplementary Section 8.2 accounting: one op per
 * right-column entry, two per top-row entry, seven per inner entry.
 */
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_NOT_ALIGNED 1
#define OR_EINVAL (-1)
#define OR_EALPHABET (-2)
#define OR_ERANGE (-3)
#define OR_ENOMEM (-4)
#define OR_EINTERNAL (-7)

enum { OP_M = 0, OP_S = 1, OP_I = 2, OP_D = 3 };

typedef struct {
    int64_t windows;
    int64_t ops_alg;        /* sum over windows of (d_w+1) + 2 n_w + 7 n_w d_w  */
    int64_t ops_genasm;     /* same with k_w in place of d_w (full-k GenASM)     */
    int64_t tb_steps;
    /* instrumentation of the traceback's reads (DENT / ET claims) */
    int32_t max_col_read;          /* largest column i of R read by traceback    */
    int32_t max_bit_read;          /* largest pattern bit j read by traceback    */
    int32_t max_row_above_dw;      /* max over windows of (row read - d_w)       */
    int32_t max_rows_below_dw;     /* max over windows of (d_w - lowest row read) */
} or_stats;

typedef struct {
    int32_t pair, p0, t0, m_w, n_w, k_w, d_w, adv_p, adv_t, edits;
} or_window;

static int encode_base(uint8_t c) {
    switch (c) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return -1;
    }
}

typedef struct {
    int max_col, max_bit, max_row, min_row;
} tb_reads;

#define BV uint64_t
#define BVBITS 64
#define SFX(x) x##_64
#include "oracle_width.inc"
#undef BV
#undef BVBITS
#undef SFX

#define BV unsigned __int128
#define BVBITS 128
#define SFX(x) x##_128
#include "oracle_width.inc"
#undef BV
#undef BVBITS
#undef SFX

/* Public: run Algorithm 1 on one window given as ASCII and return the table. */
int or_dc_table(const uint8_t* pat, int32_t mw, const uint8_t* txt, int32_t nw, int32_t kw,
                uint64_t* R, int32_t* dw) {
    if (mw < 1 || mw > 64 || nw < 0 || nw > 64 || kw < 0 || kw > mw) return OR_EINVAL;
    int8_t p[64], t[64];
    for (int j = 0; j < mw; j++) { int c = encode_base(pat[j]); if (c < 0) return OR_EALPHABET; p[j] = (int8_t)c; }
    for (int i = 0; i < nw; i++) { int c = encode_base(txt[i]); if (c < 0) return OR_EALPHABET; t[i] = (int8_t)c; }
    *dw = genasm_dc_64(p, mw, t, nw, kw, R);
    return OR_OK;
}

/* Public: the same for windows of up to 128 characters; entry (i, d) is
 * returned as two words, R2[2*(i*(kw+1)+d)] = low 64 bits, [+1] = high. */
int or_dc_table_wide(const uint8_t* pat, int32_t mw, const uint8_t* txt, int32_t nw, int32_t kw,
                     uint64_t* R2, int32_t* dw) {
    if (mw < 1 || mw > 128 || nw < 0 || nw > 128 || kw < 0 || kw > mw) return OR_EINVAL;
    int8_t p[128], t[128];
    for (int j = 0; j < mw; j++) { int c = encode_base(pat[j]); if (c < 0) return OR_EALPHABET; p[j] = (int8_t)c; }
    for (int i = 0; i < nw; i++) { int c = encode_base(txt[i]); if (c < 0) return OR_EALPHABET; t[i] = (int8_t)c; }
    const size_t cells = (size_t)(nw + 1) * (size_t)(kw + 1);
    unsigned __int128* R = (unsigned __int128*)malloc(sizeof(unsigned __int128) * cells);
    if (!R) return OR_ENOMEM;
    *dw = genasm_dc_128(p, mw, t, nw, kw, R);
    for (size_t x = 0; x < cells; x++) {
        R2[2 * x] = (uint64_t)R[x];
        R2[2 * x + 1] = (uint64_t)(R[x] >> 64);
    }
    free(R);
    return OR_OK;
}

/* Public: the four pattern masks of a window (ASCII pattern, 1..64 chars). */
int or_pattern_masks(const uint8_t* pat, int32_t mw, uint64_t* PM) {
    if (mw < 1 || mw > 64) return OR_EINVAL;
    int8_t p[64];
    for (int j = 0; j < mw; j++) { int c = encode_base(pat[j]); if (c < 0) return OR_EALPHABET; p[j] = (int8_t)c; }
    build_pattern_masks_64(p, mw, PM);
    return OR_OK;
}


/* Align one pair with window W (1..128), overlap O and edit budget k: the
 * 64-bit instantiation for W <= 64, the 128-bit one above.  Returns OR_OK,
 * OR_NOT_ALIGNED or a negative error. */
int or_align_pair(const uint8_t* pat, int32_t m, const uint8_t* txt, int32_t n,
                  int32_t W, int32_t O, int32_t k,
                  int32_t* edits_out, int32_t* text_end_out,
                  uint8_t* ops, int64_t ops_cap, int64_t* n_ops_out,
                  or_stats* st, or_window* wrec, int64_t wrec_cap, int64_t* n_wrec, int32_t pair_id) {
    if (W < 1 || W > 128 || O < 0 || O >= W || k < 0 || k > W || m < 0 || n < 0) return OR_EINVAL;
    if (W <= 64)
        return align_pair_64(pat, m, txt, n, W, O, k, edits_out, text_end_out, ops, ops_cap, n_ops_out, st, wrec,
                             wrec_cap, n_wrec, pair_id);
    return align_pair_128(pat, m, txt, n, W, O, k, edits_out, text_end_out, ops, ops_cap, n_ops_out, st, wrec,
                          wrec_cap, n_wrec, pair_id);
}

typedef struct {
    int32_t npairs;
    const uint8_t *pat, *txt;
    const int64_t *pat_off, *txt_off, *ops_off;
    int32_t W, O, k;
    int32_t *edits, *text_end, *status;
    uint8_t* ops;
    int64_t* n_ops;
    atomic_long next;
    atomic_int err;
    pthread_mutex_t lock;
    or_stats total;
} batch_job;

static void* batch_worker(void* arg) {
    batch_job* J = (batch_job*)arg;
    or_stats st;
    memset(&st, 0, sizeof st);
    st.max_col_read = st.max_bit_read = -1;
    for (;;) {
        long idx = atomic_fetch_add(&J->next, 1);
        if (idx >= J->npairs) break;
        const int64_t ps = J->pat_off[idx], pe = J->pat_off[idx + 1];
        const int64_t ts = J->txt_off[idx], te = J->txt_off[idx + 1];
        const int64_t os = J->ops_off[idx], oe = J->ops_off[idx + 1];
        int rc = or_align_pair(J->pat + ps, (int32_t)(pe - ps), J->txt + ts, (int32_t)(te - ts),
                               J->W, J->O, J->k, &J->edits[idx], &J->text_end[idx],
                               J->ops + os, oe - os, &J->n_ops[idx], &st, NULL, 0, NULL, (int32_t)idx);
        J->status[idx] = rc;
        if (rc < 0) atomic_store(&J->err, rc);
    }
    pthread_mutex_lock(&J->lock);
    J->total.windows += st.windows;
    J->total.ops_alg += st.ops_alg;
    J->total.ops_genasm += st.ops_genasm;
    J->total.tb_steps += st.tb_steps;
    if (st.max_col_read > J->total.max_col_read) J->total.max_col_read = st.max_col_read;
    if (st.max_bit_read > J->total.max_bit_read) J->total.max_bit_read = st.max_bit_read;
    if (st.max_row_above_dw > J->total.max_row_above_dw) J->total.max_row_above_dw = st.max_row_above_dw;
    if (st.max_rows_below_dw > J->total.max_rows_below_dw) J->total.max_rows_below_dw = st.max_rows_below_dw;
    pthread_mutex_unlock(&J->lock);
    return NULL;
}

/* Align a CSR batch on nthreads host threads (a shared atomic pair index).
 * Per-pair status goes to status[] (OR_OK / OR_NOT_ALIGNED / negative).
 * Returns the first negative per-pair error, else OR_OK. */
int or_align_batch(int32_t npairs, const uint8_t* pat, const int64_t* pat_off,
                   const uint8_t* txt, const int64_t* txt_off,
                   int32_t W, int32_t O, int32_t k, int32_t nthreads,
                   int32_t* edits, int32_t* text_end, int32_t* status,
                   uint8_t* ops, const int64_t* ops_off, int64_t* n_ops, or_stats* total) {
    if (npairs < 0 || nthreads < 1 || nthreads > 1024) return OR_EINVAL;
    if (W < 1 || W > 128 || O < 0 || O >= W || k < 0 || k > W) return OR_EINVAL;
    batch_job J;
    memset(&J, 0, sizeof J);
    J.npairs = npairs; J.pat = pat; J.txt = txt; J.pat_off = pat_off; J.txt_off = txt_off; J.ops_off = ops_off;
    J.W = W; J.O = O; J.k = k; J.edits = edits; J.text_end = text_end; J.status = status; J.ops = ops; J.n_ops = n_ops;
    atomic_init(&J.next, 0);
    atomic_init(&J.err, 0);
    pthread_mutex_init(&J.lock, NULL);
    J.total.max_col_read = J.total.max_bit_read = -1;
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nthreads);
    if (!th) return OR_ENOMEM;
    int started = 0;
    for (int x = 0; x < nthreads; x++)
        if (pthread_create(&th[x], NULL, batch_worker, &J) == 0) started++;
    if (started == 0) batch_worker(&J);
    for (int x = 0; x < started; x++) pthread_join(th[x], NULL);
    free(th);
    pthread_mutex_destroy(&J.lock);
    if (total) *total = J.total;
    return atomic_load(&J.err);
}
