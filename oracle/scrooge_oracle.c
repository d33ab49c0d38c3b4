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

/* all-ones over the m_w low machine bits */
static uint64_t width_mask(int mw) { return mw >= 64 ? ~0ULL : ((1ULL << mw) - 1ULL); }

/* paper bit j of an m_w-bit vector; bit index m_w (one past the last pattern
 * character) reads as 0: the empty pattern suffix is always within distance. */
static int pbit(uint64_t v, int j, int mw) {
    if (j >= mw) return 0;
    return (int)((v >> (mw - 1 - j)) & 1ULL);
}

/* buildPatternMasks (Section 2.2.1): PM[X] has a 0 at bit j iff p[j] == X. */
static void build_pattern_masks(const int8_t* p, int mw, uint64_t PM[4]) {
    const uint64_t mask = width_mask(mw);
    for (int x = 0; x < 4; x++) {
        PM[x] = mask;
        for (int j = 0; j < mw; j++)
            if (p[j] == x) PM[x] &= ~(1ULL << (mw - 1 - j));
    }
}

/* Algorithm 1 on one window.  p, t hold base codes.  R must hold
 * (nw+1)*(kw+1) words, R[i*(kw+1)+d].  Returns d_w, or -1 when no row
 * 0..kw has a 0 in the msb of its leftmost entry. */
static int genasm_dc(const int8_t* p, int mw, const int8_t* t, int nw, int kw, uint64_t* R) {
    const uint64_t mask = width_mask(mw);
    const int K = kw + 1;
    uint64_t PM[4];
    build_pattern_masks(p, mw, PM);
    /* right column: R[n][d] = 11...1 << d, restricted to m_w bits */
    for (int d = 0; d <= kw; d++)
        R[nw * K + d] = d >= 64 ? 0ULL : ((mask << d) & mask);
    for (int i = nw - 1; i >= 0; i--) {
        const uint64_t cur = PM[(int)t[i]];
        R[i * K + 0] = ((R[(i + 1) * K + 0] << 1) | cur) & mask;
        for (int d = 1; d <= kw; d++) {
            const uint64_t I = (R[i * K + d - 1] << 1) & mask;
            const uint64_t D = R[(i + 1) * K + d - 1];
            const uint64_t S = (R[(i + 1) * K + d - 1] << 1) & mask;
            const uint64_t M = ((R[(i + 1) * K + d] << 1) | cur) & mask;
            R[i * K + d] = I & D & S & M;
        }
    }
    for (int d = 0; d <= kw; d++)
        if (pbit(R[d], 0, mw) == 0) return d;
    return -1;
}

/* Public: run Algorithm 1 on one window given as ASCII and return the table. */
int or_dc_table(const uint8_t* pat, int32_t mw, const uint8_t* txt, int32_t nw, int32_t kw,
                uint64_t* R, int32_t* dw) {
    if (mw < 1 || mw > 64 || nw < 0 || nw > 64 || kw < 0 || kw > mw) return OR_EINVAL;
    int8_t p[64], t[64];
    for (int j = 0; j < mw; j++) { int c = encode_base(pat[j]); if (c < 0) return OR_EALPHABET; p[j] = (int8_t)c; }
    for (int i = 0; i < nw; i++) { int c = encode_base(txt[i]); if (c < 0) return OR_EALPHABET; t[i] = (int8_t)c; }
    *dw = genasm_dc(p, mw, t, nw, kw, R);
    return OR_OK;
}

/* Public: the four pattern masks of a window (ASCII pattern, 1..64 chars). */
int or_pattern_masks(const uint8_t* pat, int32_t mw, uint64_t* PM) {
    if (mw < 1 || mw > 64) return OR_EINVAL;
    int8_t p[64];
    for (int j = 0; j < mw; j++) { int c = encode_base(pat[j]); if (c < 0) return OR_EALPHABET; p[j] = (int8_t)c; }
    build_pattern_masks(p, mw, PM);
    return OR_OK;
}

typedef struct {
    int max_col, max_bit, max_row, min_row;
} tb_reads;

static uint64_t tb_entry(const uint64_t* R, int K, int i, int d, int j, tb_reads* rd) {
    if (i > rd->max_col) rd->max_col = i;
    if (j > rd->max_bit) rd->max_bit = j;
    if (d > rd->max_row) rd->max_row = d;
    if (d < rd->min_row) rd->min_row = d;
    return R[i * K + d];
}

/* Align one pair.  ops receives one byte per operation.  Returns OR_OK,
 * OR_NOT_ALIGNED or a negative error.  wrec (optional) receives one record
 * per window. */
int or_align_pair(const uint8_t* pat, int32_t m, const uint8_t* txt, int32_t n,
                  int32_t W, int32_t O, int32_t k,
                  int32_t* edits_out, int32_t* text_end_out,
                  uint8_t* ops, int64_t ops_cap, int64_t* n_ops_out,
                  or_stats* st, or_window* wrec, int64_t wrec_cap, int64_t* n_wrec, int32_t pair_id) {
    if (W < 1 || W > 64 || O < 0 || O >= W || k < 0 || k > W || m < 0 || n < 0) return OR_EINVAL;
    int8_t* P = (int8_t*)malloc((size_t)m + 1);
    int8_t* T = (int8_t*)malloc((size_t)n + 1);
    uint64_t* R = (uint64_t*)malloc(sizeof(uint64_t) * 65 * 65);
    if (!P || !T || !R) { free(P); free(T); free(R); return OR_ENOMEM; }
    int rc = OR_OK;
    for (int32_t x = 0; x < m && rc == OR_OK; x++) { int c = encode_base(pat[x]); if (c < 0) rc = OR_EALPHABET; else P[x] = (int8_t)c; }
    for (int32_t x = 0; x < n && rc == OR_OK; x++) { int c = encode_base(txt[x]); if (c < 0) rc = OR_EALPHABET; else T[x] = (int8_t)c; }
    int64_t nops = 0, nw_rec = 0;
    int32_t edits = 0, p0 = 0, t0 = 0;
    const int cap = W - O;
    while (rc == OR_OK && p0 < m) {
        const int mw = (m - p0) < W ? (m - p0) : W;
        const int nw = (n - t0) < W ? (n - t0) : W;
        const int kw = k < mw ? k : mw;
        const int K = kw + 1;
        const int8_t* p = P + p0;
        const int8_t* t = T + t0;
        const int dw = genasm_dc(p, mw, t, nw, kw, R);
        const int drows = dw < 0 ? kw : dw;
        if (st) {
            st->windows++;
            st->ops_alg += (int64_t)(drows + 1) + 2LL * nw + 7LL * nw * drows;
            st->ops_genasm += (int64_t)(kw + 1) + 2LL * nw + 7LL * nw * kw;
        }
        if (dw < 0) { rc = OR_NOT_ALIGNED; break; }
        /* GenASM-TB */
        int i = 0, j = 0, d = dw, wedits = 0;
        tb_reads rd = {-1, -1, -1, 1 << 30};
        while (j < mw && i < cap && j < cap) {
            int m_ok = 0, s_ok = 0, i_ok = 0, d_ok = 0;
            if (i < nw && t[i] == p[j])
                m_ok = pbit(tb_entry(R, K, i + 1, d, j + 1, &rd), j + 1, mw) == 0;
            if (!m_ok && d > 0) {
                if (i < nw) s_ok = pbit(tb_entry(R, K, i + 1, d - 1, j + 1, &rd), j + 1, mw) == 0;
                if (!s_ok) i_ok = pbit(tb_entry(R, K, i, d - 1, j + 1, &rd), j + 1, mw) == 0;
                if (!s_ok && !i_ok && i < nw) d_ok = pbit(tb_entry(R, K, i + 1, d - 1, j, &rd), j, mw) == 0;
            }
            int op;
            if (m_ok) { op = OP_M; i++; j++; }
            else if (s_ok) { op = OP_S; i++; j++; d--; }
            else if (i_ok) { op = OP_I; j++; d--; }
            else if (d_ok) { op = OP_D; i++; d--; }
            else { rc = OR_EINTERNAL; break; }
            if (op != OP_M) wedits++;
            if (nops >= ops_cap) { rc = OR_ERANGE; break; }
            ops[nops++] = (uint8_t)op;
            if (st) st->tb_steps++;
        }
        if (rc != OR_OK) break;
        if (st) {
            if (rd.max_col > st->max_col_read) st->max_col_read = rd.max_col;
            if (rd.max_bit > st->max_bit_read) st->max_bit_read = rd.max_bit;
            if (rd.max_row >= 0 && rd.max_row - dw > st->max_row_above_dw) st->max_row_above_dw = rd.max_row - dw;
            if (rd.min_row <= 64 && dw - rd.min_row > st->max_rows_below_dw) st->max_rows_below_dw = dw - rd.min_row;
        }
        if (wrec && nw_rec < wrec_cap) {
            or_window* w = &wrec[nw_rec];
            w->pair = pair_id; w->p0 = p0; w->t0 = t0; w->m_w = mw; w->n_w = nw; w->k_w = kw;
            w->d_w = dw; w->adv_p = j; w->adv_t = i; w->edits = wedits;
        }
        nw_rec++;
        edits += wedits;
        p0 += j;
        t0 += i;
    }
    if (n_wrec) *n_wrec = nw_rec;
    if (rc == OR_OK) {
        *edits_out = edits; *text_end_out = t0; *n_ops_out = nops;
    } else {
        *edits_out = -1; *text_end_out = -1; *n_ops_out = 0;
    }
    free(P); free(T); free(R);
    return rc;
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
    if (W < 1 || W > 64 || O < 0 || O >= W || k < 0 || k > W) return OR_EINVAL;
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
