/*
 * scrooge.h -- C ABI of libscrooge_hip.so: windowed GenASM pairwise alignment
 * (Scrooge, arXiv 2208.09985) on AMD Instinct MI355X (gfx950).
 *
 * Problem (Section 2.1): given a text and a pattern over {A,C,G,T}, find the
 * smallest number of substitutions, insertions and deletions turning the text
 * into the pattern, and the edit sequence (CIGAR).  The method is GenASM-DC
 * (Algorithm 1, Section 2.2.1) and GenASM-TB (Section 2.2.2) applied window
 * by window (Section 2.2.3) with the three Scrooge improvements: stored
 * entries instead of edges (Section 2.4.1), discarded entries that traceback
 * never reads (Section 2.4.2) and early termination (Section 2.4.3).
 *
 * Conventions common to every call:
 *   - Every function returns an int status (SCG_OK or a negative SCG_E*);
 *     nothing aborts or throws across this boundary.  scg_strerror() names it.
 *   - Sequences are ASCII A/C/G/T (either case).  Anything else is an input
 *     error: host input is rejected at batch creation (SCG_EALPHABET); device
 *     input marks the offending pair with SCG_PAIR_BAD_INPUT.
 *   - Windows: 1 <= W <= 64, 0 <= O < W, 0 <= k <= W (else SCG_EINVAL);
 *     plain mode also takes 64 < W <= 128 (128-bit bitvectors, column
 *     blocks, no yields or ablation flags; anything else with W > 64 is
 *     SCG_EINVAL).
 *     Window w aligns pattern[p0, p0+m_w) with text[t0, t0+n_w), m_w =
 *     min(W, m-p0), n_w = min(W, n-t0), allowing k_w = min(k, m_w) edits.
 *     Traceback stops once W-O characters of text or pattern are consumed
 *     (or the window's pattern is used up); the next window starts there.
 *     Traceback prefers M, then S, then I, then D.  The text tail after the
 *     last aligned character is free; text_end reports how much was consumed.
 *   - Operations: SCG_OP_M '=' match, SCG_OP_S 'X' substitution, SCG_OP_I 'I'
 *     a pattern character absent from the text, SCG_OP_D 'D' a text character
 *     absent from the pattern.  edits = number of non-M operations.
 *   - CIGAR output is run-length encoded as uint32 words (len << 2) | op,
 *     runs merged across windows.  A pair of lengths (m, n) never needs more
 *     than m + n + 1 words.
 *   - Device pointers are used as-is on the caller's HIP stream (a
 *     hipStream_t passed as void*; NULL = the null stream).  The library
 *     owns only its own workspace; every caller buffer stays the caller's.
 */
#ifndef SCROOGE_H
#define SCROOGE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SCG_OK = 0,
    SCG_EINVAL = -1,      /* bad argument (NULL, size or W/O/k range)          */
    SCG_EALPHABET = -2,   /* a character outside A/C/G/T (host input)          */
    SCG_ERANGE = -3,      /* caller buffer too small                           */
    SCG_ENOMEM = -4,      /* device or host allocation failed                  */
    SCG_EDEVICE = -5,     /* a HIP runtime call failed                         */
    SCG_ENOMODEL = -6,    /* learned mode requested without a loaded predictor */
    SCG_EINTERNAL = -7,   /* the device reported an inconsistent state         */
    SCG_ELIMIT = -8       /* batch larger than the allocation-free workspace   */
};

/* per-pair status values */
enum {
    SCG_PAIR_OK = 0,
    SCG_PAIR_NOT_ALIGNED = 1,  /* some window had no distance <= k_w; edits = -1 */
    SCG_PAIR_BAD_INPUT = 2,    /* non-ACGT character in device input             */
    SCG_PAIR_ERROR = 3         /* internal inconsistency or run buffer overflow  */
};

enum { SCG_OP_M = 0, SCG_OP_S = 1, SCG_OP_I = 2, SCG_OP_D = 3 };

/* how many error rows each window computes before falling back */
enum {
    SCG_MODE_PLAIN = 0,    /* every window computes all rows 0..k_w (with early termination)  */
    SCG_MODE_LEARNED = 1,  /* the loaded predictor picks a row budget k' per window;           */
                           /* a window with no distance <= k' is recomputed with all rows      */
    SCG_MODE_FIXED = 2     /* constant budget (fixed_rows) per window, same fallback           */
};

/* queue order of the pairs (results do not depend on it): input order, longest
 * (pattern + text) first, or automatic (the default of scg_params_default:
 * longest first when the lengths' coefficient of variation exceeds 0.1) */
enum { SCG_ORDER_INPUT = 0, SCG_ORDER_LONGEST_FIRST = 1, SCG_ORDER_AUTO = 2 };
enum { SCG_WHERE_HOST = 0, SCG_WHERE_DEVICE = 1 };
/* input_kind of the batch calls: how pattern and text bytes are encoded */
enum {
    SCG_INPUT_ASCII = 0,   /* one ASCII byte per base (A/C/G/T, either case); offsets count bytes    */
    SCG_INPUT_PACKED2 = 1  /* two bits per base (the paper's 2-bit encoding, Section 2.5): 32 bases */
                           /* per uint64, base t of a word in bits 2t and 2t+1; offsets count bases; */
                           /* sequence i starts at uint64 word sum over j < i of ceil(len_j / 32).   */
                           /* Any code assignment works as long as patterns and texts share it       */
};
enum {
    SCG_FLAG_GRAPH = 1,              /* replay the batch's launches from a captured hipGraph   */
                                     /* (ignored when the batch runs off-track helpers: their */
                                     /* launch runs beside the main one on the context's      */
                                     /* helper stream, which a graph would not keep)          */
    /* Ablations of the paper's improvements (Section 2.4), plain mode in the column-block     */
    /* kernel only (SCG_EINVAL otherwise); results are unchanged, only the work grows:         */
    SCG_FLAG_NO_EARLY_TERMINATION = 2,  /* every window computes all k_w+1 rows (no ET)        */
    SCG_FLAG_STORE_ALL_COLUMNS = 4,     /* store every column of a row, not only 0..W-O (no    */
                                        /* DENT)                                               */
    SCG_FLAG_ROWS_LDS = 8,              /* keep the lowest stored rows of each window in LDS   */
                                        /* (as many as fit with the wavefronts the batch       */
                                        /* needs; 4, 8 or 16 windows per wavefront), the rest  */
                                        /* in global memory; by default all rows are global    */
                                        /* in the main launch (the off-track helper launch     */
                                        /* always keeps its lowest rows in LDS)                */
    SCG_FLAG_STORE_EDGES = 16,          /* store each entry's edge bitvectors (I, S, D of the  */
                                        /* row above and M, 32 bytes) instead of the entry (no */
                                        /* SENE); 4, 8 or 16 windows per wavefront, rows in    */
                                        /* global memory                                       */
    SCG_FLAG_ROW_RING = 32              /* DENT extended to rows (supplementary Section 1):    */
                                        /* stored rows in a ring of W-O+1+64/slots slots, the  */
                                        /* rows traceback can read below d_w plus those the    */
                                        /* lanes compute past it; needs early termination; 4,  */
                                        /* 8 or 16 windows per wavefront                       */
};

/* which fused kernel aligns the batch (same results, different mappings) */
enum {
    SCG_KERNEL_AUTO = 0,     /* column blocks in plain mode, error rows with a row budget     */
    SCG_KERNEL_ROWS = 1,     /* lanes are error rows; windows packed as lane segments          */
    SCG_KERNEL_COLUMNS = 2,  /* 4/8/16 windows per wavefront (32 without a learned budget),   */
                             /* lanes own text columns; a pass of row steps, then tracebacks   */
    SCG_KERNEL_LANES = 3     /* one lane per pair, rows computed in order over all columns,  */
                             /* the latest W-O+1 rows kept (the paper's row-wise CPU mapping; */
                             /* plain mode, W <= 64, no yields or ablation flags)             */
};

typedef struct {
    int32_t W, O, k;        /* window size, overlap, edit budget per window            */
    int32_t mode;           /* SCG_MODE_*                                              */
    int32_t slots;          /* windows in flight per wavefront, 1..16 (0 = automatic); */
                            /* column blocks round up to 4, 8, 16 or, in plain and     */
                            /* fixed modes, 10 (slots 9..10: six lanes of 12 columns)  */
                            /* or 32 (slots 17..32).  Automatic, column blocks: short  */
                            /* reads (16 windows or fewer per pattern on average, plain */
                            /* mode) 16 once those fill the SIMDs, else 8; fewer than  */
                            /* 8 pairs per CU 4; lengths that vary, longest first      */
                            /* (plain mode, rows in global memory) 4, with just enough */
                            /* wavefronts per CU to keep (all windows / the longest    */
                            /* pair's windows) windows in flight, when that is at most */
                            /* one per SIMD, and 16 beside helpers that hold the       */
                            /* longest pairs when it is more but below the occupancy   */
                            /* maximum; otherwise 8 (10 when those fit one per SIMD    */
                            /* and 8 do not); 16 with the off-track helpers            */
    int32_t waves_per_cu;   /* persistent wavefronts per CU (0 = occupancy maximum, or */
                            /* the count the automatic rule for varying lengths picks) */
    int32_t order;          /* SCG_ORDER_* : queue order of pairs                      */
    int32_t fixed_rows;     /* SCG_MODE_FIXED: rows computed before falling back       */
    float tau;              /* SCG_MODE_LEARNED: confidence needed for a smaller budget */
    int32_t flags;          /* SCG_FLAG_*                                              */
    int32_t yield_chars;    /* a pair returns to the queue after advancing this many   */
                            /* pattern characters (0 = never; > 0: at least W-O;       */
                            /* < 0: automatic, 1280 for error-row lanes, 0 for column  */
                            /* blocks)                                                 */
    int32_t kernel;         /* SCG_KERNEL_*                                            */
    int32_t one_per_simd;   /* column blocks, plain mode, rows in global memory, 4, 8, */
                            /* 10 or 16 windows per wavefront: 1 = the form that holds a */
                            /* whole SIMD per wavefront (the grid is then at most one  */
                            /* wavefront per SIMD); 0 = automatic, that form whenever  */
                            /* the batch's wavefronts fit one per SIMD (10 windows per */
                            /* wavefront are then picked when 8 would not fit); -1 =   */
                            /* never.  Results are the same either way                 */
    int32_t offtrack_helpers;  /* column blocks, plain mode, no yields or ablations     */
                            /* (SCG_FLAG_ROWS_LDS allowed, with 16 windows per main    */
                            /* wavefront; the graph flag too, which is then ignored): */
                            /* a pair whose last three                                 */
                            /* windows each had d_w >= 3(W-O)/5 (it has lost the      */
                            /* diagonal) is handed to a second launch of wavefronts    */
                            /* with 4 windows of 16 lanes each, on the SIMDs the main  */
                            /* launch (16 windows per wavefront, one per SIMD) leaves  */
                            /* free, which keeps its windows' lowest rows in LDS; its  */
                            /* windows then take fewer instructions.  1 = always when  */
                            /* the main launch fits, 0 = automatic (W-O at least 30,   */
                            /* pairs longer than 32 windows on average, at least as    */
                            /* many pairs as 4-window wavefronts one per SIMD hold,    */
                            /* and 16-window wavefronts that fit while leaving at      */
                            /* least 128 SIMDs), -1 = never.  Results are the same     */
                            /* either way.  Automatic also for lengths that vary, when */
                            /* the batch needs more than one 4-window wavefront per    */
                            /* SIMD (W-O at least 30): one helper wavefront per CU     */
                            /* holds the longest pairs from the start, and 16-window   */
                            /* wavefronts one per SIMD take the others from the queue. */
                            /* A helper that sees no progress of the main              */
                            /* launch for some 55 ms (environment variable             */
                            /* SCG_HELPER_IDLE_POLLS, read at batch creation, sets the */
                            /* polls) stops taking pairs; the main launch then keeps   */
                            /* the pairs it would have handed over.  The helper launch */
                            /* runs on one stream per context, created on first use    */
                            /* and shared by the context's batches: runs of two such   */
                            /* batches of one context on different streams at once    */
                            /* are correct, but their helper launches take turns; a    */
                            /* caller that captures such a run into a graph of its own */
                            /* captures the helper stream with it, so no other batch  */
                            /* of the context may run until the capture ends           */
} scg_params;

typedef struct {
    double kernel_ms;          /* alignment kernel time of the last run (HIP events)     */
    double pack_ms;            /* encode/pack kernels of the last run                    */
    double kernel_ms_avg;      /* mean alignment kernel time over the runs since the     */
    double pack_ms_avg;        /*   previous scg_batch_stats call (at most 256 runs)     */
    int64_t timed_runs;        /* number of runs in those means                          */
    int64_t windows;           /* windows aligned (last run)                             */
    int64_t ops_alg;           /* sum over windows of (d_w+1) + 2 n_w + 7 n_w d_w        */
    int64_t fallback_windows;  /* windows recomputed after missing their budget          */
    int64_t lane_steps;        /* sum over passes of lanes x diagonal steps (work issued) */
    int64_t rounds;            /* wavefront rounds (one DC pass each)                    */
    int64_t rows_budgeted;     /* sum over window attempts of rows computed              */
    int64_t yields;            /* times a pair went back to the queue                    */
} scg_stats;

typedef struct scg_ctx scg_ctx;
typedef struct scg_batch scg_batch;

/* Name of a status code (static string). */
const char* scg_strerror(int code);

/* Text of the last failing HIP runtime call on this thread ("" if none):
 * the call and the runtime's message.  Static per-thread storage. */
const char* scg_last_hip_error(void);

/* Default parameters: W=64, O=24, k=64, plain mode, automatic launch shape
 * (column blocks in plain mode, windows per wavefront as described at
 * scg_params.slots; error-row lanes with 4 slots when windows start with a
 * row budget), automatic queue order, one_per_simd and offtrack_helpers,
 * fixed_rows = 15, tau = 0.8, yield_chars = -1 (automatic). */
void scg_params_default(scg_params* p);

/* Create a context on HIP device `device`.  *out receives the context; the
 * caller releases it with scg_destroy.  weights_path names a predictor file
 * for SCG_MODE_LEARNED (NULL: plain and fixed modes only, or a later
 * scg_set_model).  The file is little-endian: the bytes "SCGW", uint32
 * version 1, int32 F, H, C, int32 budget_rows[C], then FP16 w1[F*H], b1[H],
 * w2[H*C], b2[C] (as scg_set_model), nothing after.
 * Errors: SCG_EINVAL (also a missing or malformed file), SCG_EDEVICE. */
int scg_create(scg_ctx** out, int device, const char* weights_path);
/* Release the context and its helper stream: destroy its batches first, once
 * their runs have finished. */
void scg_destroy(scg_ctx* ctx);

/* Number of compute units of the context's device (for launch planning). */
int scg_device_cus(const scg_ctx* ctx);

/* Load the row-budget predictor used by SCG_MODE_LEARNED: a 2-layer MLP
 * F -> H (ReLU) -> C over per-window features (scg_features), all FP16,
 * host arrays, row-major: w1[F*H], b1[H], w2[H*C], b2[C].  Class c predicts
 * "d_w fits in budget_rows[c] rows" (budget_rows: C increasing int32,
 * the last >= 64).  F must be SCG_NFEATURES, H <= 64, C <= 4.
 * Copied to the device; the host arrays stay the caller's. */
enum { SCG_NFEATURES = 16 };
int scg_set_model(scg_ctx* ctx, int32_t F, int32_t H, int32_t C,
                  const uint16_t* w1, const uint16_t* b1, const uint16_t* w2, const uint16_t* b2,
                  const int32_t* budget_rows);

/* Prepare a batch of npairs (pattern, text) pairs for repeated alignment.
 * pat/txt: concatenated sequences encoded as input_kind says (SCG_INPUT_*);
 * pat_off/txt_off: npairs+1 int64 offsets (bytes for ASCII, bases for packed
 * input), always in HOST memory.  where = SCG_WHERE_HOST (bytes in host
 * memory, validated and copied to the device) or SCG_WHERE_DEVICE (bytes
 * already in device memory, used in place: they must outlive the batch).
 * The batch owns its workspace (2-bit planes, queue, counters); free it
 * with scg_batch_destroy.  Errors: SCG_EINVAL, SCG_EALPHABET, SCG_ENOMEM,
 * SCG_EDEVICE, SCG_ENOMODEL (learned mode without scg_set_model). */
int scg_batch_create(scg_ctx* ctx, const scg_params* params, int32_t npairs,
                     const void* pat, const int64_t* pat_off, const void* txt, const int64_t* txt_off,
                     int32_t input_kind, int32_t where, void* stream, scg_batch** out);
void scg_batch_destroy(scg_batch* b);

/* uint32 words the runs buffer of scg_batch_run needs, and the per-pair
 * start offsets into it (npairs+1 int64, host memory). */
int64_t scg_batch_runs_capacity(const scg_batch* b);
int scg_batch_runs_offsets(const scg_batch* b, int64_t* out);

/* The launch shape the batch was created with (a query; no device work).
 * out[0] kernel: SCG_KERNEL_ROWS, SCG_KERNEL_COLUMNS, SCG_KERNEL_LANES, or 4
 * for the wide-window column form (W > 64); out[1] windows per wavefront;
 * out[2] wavefronts in the grid; out[3] dynamic LDS bytes per wavefront;
 * out[4] 1 for the form holding a whole SIMD per wavefront; out[5] stored
 * entry bits (32, 48 or 64; 96 or 128 for wide windows; 0 for error-row
 * lanes); out[6] wavefronts of the off-track helper launch (0: none);
 * out[7] its windows per wavefront; out[8] its dynamic LDS bytes per
 * wavefront; out[9] the longest pairs it holds from the start (0: only
 * pairs handed over).  out: 10 int32 in host memory.
 * Errors: SCG_EINVAL. */
int scg_batch_launch_shape(const scg_batch* b, int32_t* out);

/* Align the batch: encode+pack (Section 2.5's 2-bit encoding), then the
 * persistent fused DC+TB kernel.  All outputs are DEVICE pointers of npairs
 * int32 each, except runs (scg_batch_runs_capacity uint32 words, pair p at
 * offset runs_offsets[p]).  Asynchronous on `stream`; the caller
 * synchronises before reading.  Pairs with status != SCG_PAIR_OK have
 * edits = text_end = -1 and n_runs = 0. */
int scg_batch_run(scg_batch* b, void* stream, int32_t* edits, int32_t* text_end, int32_t* status,
                  uint32_t* runs, int32_t* n_runs);

/* Synchronise the batch's last run and read its counters and timings.
 * Timings come from HIP events recorded on the run's stream around the
 * pack kernels and around the alignment kernel (graph replays: around the
 * whole replay, reported as kernel time). */
int scg_batch_stats(scg_batch* b, scg_stats* out);

/* One pair in host memory (convenience; allocates and synchronises).
 * cigar receives a NUL-terminated string ("12=1X3I..."); cap must cover it
 * (SCG_ERANGE with *cigar_len = needed length otherwise). */
int scg_align(scg_ctx* ctx, const char* pattern, int32_t m, const char* text, int32_t n,
              int32_t W, int32_t O, int32_t k, int32_t* edits, int32_t* text_end,
              char* cigar, int32_t cigar_cap, int32_t* cigar_len);

/* A whole batch in one call (the align-all call of supplementary Section 7,
 * tool function calls; the problem statement of Section 2.1 per pair: edit
 * count and edit sequence): scg_batch_create + scg_batch_run + expansion of
 * the runs into operation streams + synchronise + destroy.
 * Inputs as in scg_batch_create.  Outputs live where the inputs do: with
 * SCG_WHERE_HOST they are host arrays (the library allocates device
 * buffers for the run and copies back), with SCG_WHERE_DEVICE device arrays
 * written in place.  edits, text_end, status, n_ops: npairs int32 each.
 * ops: each pair's operations at two bits each (SCG_OP_*), operation t of
 * pair p in byte ops_off[p] + t / 4, bits 2 (t % 4) and 2 (t % 4) + 1;
 * ops_off: npairs+1 int64 byte offsets, always in HOST memory; pair p needs
 * ceil((m_p + n_p) / 4) bytes (SCG_ERANGE otherwise, nothing run);
 * n_ops[p] operations are written (0 for pairs with status != SCG_PAIR_OK).
 * Returns when the outputs are complete.  The counters and timings of the
 * run are kept for scg_last_stats.
 * Errors: as scg_batch_create and scg_batch_run, and SCG_ERANGE. */
int scg_align_batch(scg_ctx* ctx, const scg_params* params, int32_t npairs,
                    const void* pat, const int64_t* pat_off, const void* txt, const int64_t* txt_off,
                    int32_t input_kind, int32_t where, void* stream,
                    int32_t* edits, int32_t* text_end, int32_t* status,
                    uint8_t* ops, const int64_t* ops_off, int32_t* n_ops);

/* Render a 2-bit operation stream (as written by scg_align_batch) as a
 * NUL-terminated CIGAR string, runs of equal operations merged ("12=1X3I");
 * cap must cover it (SCG_ERANGE with *len = needed length otherwise). */
int scg_ops_to_cigar(const uint8_t* ops, int32_t n_ops, char* cigar, int32_t cap, int32_t* len);

/* ---- allocation-free batch call ----
 *
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * alignment and run-word output as scg_batch_create + scg_batch_run in plain
 * mode (column-block kernel, input order: order SCG_ORDER_INPUT or SCG_ORDER_AUTO,
 * W <= 64, no yields, flags 0) on
 * device input, in one call, with every buffer besides the caller's
 * inputs and outputs taken from a static device workspace of fixed size that
 * each device holds for the life of the process (SCG_NOALLOC_DENT_MIB MiB of
 * stored rows plus planes and per-pair tables for the limits below, about
 * 105 MB).  The call enqueues its kernels on `stream` and returns without
 * synchronising; it calls no hipMalloc, hipFree or other allocating routine.
 *
 * All pointers are DEVICE pointers: pat/txt ASCII bytes (pat_total and
 * txt_total bytes, stated by the caller in host ints), pat_off/txt_off
 * npairs+1 int64 byte offsets each, outputs as for scg_batch_run (edits,
 * text_end, status, n_runs: npairs int32; runs: sum over pairs of
 * (m + n + 1) uint32 words, pair p at sum over i < p of (m_i + n_i + 1)).
 * Offsets out of order or beyond the stated totals make every pair
 * SCG_PAIR_BAD_INPUT (checked on the device).
 *
 * Limits: npairs <= SCG_NOALLOC_MAX_PAIRS, pat_total and txt_total <=
 * SCG_NOALLOC_MAX_BASES (else SCG_ELIMIT, nothing enqueued); the number of
 * wavefronts is capped by the stored-row region, so very large batches run
 * with fewer windows in flight than scg_align_batch would use.
 * Every call on a device shares that device's workspace and leaves its
 * contents behind: calls that overlap on one device (different streams or
 * host threads without ordering) race and must not be issued.
 * Errors: SCG_EINVAL, SCG_ELIMIT, SCG_EDEVICE. */
enum {
    SCG_NOALLOC_MAX_PAIRS = 65536,
    SCG_NOALLOC_MAX_BASES = 67108864,
    SCG_NOALLOC_DENT_MIB = 64
};
int scg_align_batch_noalloc(scg_ctx* ctx, const scg_params* params, int32_t npairs,
                            const void* pat, const int64_t* pat_off, int64_t pat_total,
                            const void* txt, const int64_t* txt_off, int64_t txt_total, void* stream,
                            int32_t* edits, int32_t* text_end, int32_t* status, uint32_t* runs, int32_t* n_runs);

/* Counters and timings of the context's last scg_align_batch (zeros before
 * the first): its alignment kernel time, its algorithmic work (sum over
 * windows of (d_w+1) + 2 n_w + 7 n_w d_w, supplementary Section 8's work
 * model) and the windows recomputed after missing a row budget.  Any output
 * pointer may be NULL.  scg_last_stats_all returns every counter.
 * Errors: SCG_EINVAL. */
int scg_last_stats(const scg_ctx* ctx, double* kernel_ms, int64_t* ops_alg, int64_t* fallback_windows);
int scg_last_stats_all(const scg_ctx* ctx, scg_stats* out);

/* Render run words as a CIGAR string (host memory). */
int scg_runs_to_cigar(const uint32_t* runs, int32_t n_runs, char* cigar, int32_t cap, int32_t* len);

/* ---- learned row budget: features and predictor training (device pointers) ----
 *
 * scg_features: for nwin windows given as (pair, p0, t0) int32 triples (device,
 * 3*nwin) of a prepared batch, write SCG_NFEATURES uint16 counts per window
 * (device, row-major nwin x 16): the number of aligned 4-mer matches between
 * pattern[p0, p0+m_w) and text[t0+delta, ...) on each diagonal delta = -3..3
 * (7 counts), the number of single-character matches on the same diagonals
 * (7 counts), m_w and n_w.  prev_dw is not a feature: windows are scored
 * independently so the same features serve training and inference. */
int scg_features(scg_batch* b, int32_t nwin, const int32_t* windows, uint16_t* features, void* stream);

/* Forward pass of the predictor on a batch (device pointers, FP16 storage,
 * FP32 accumulation): x[B*F] features scaled to [0,1] as fp16, weights as in
 * scg_set_model, logits[B*C] fp32 out, hidden[B*H] fp16 (post-ReLU) out.
 * With labels (int32[B], class index) also per-sample softmax cross-entropy
 * loss[B] fp32 and dlogits[B*C] fp32 = (softmax - onehot) / B. */
int scg_mlp_forward(int32_t B, int32_t F, int32_t H, int32_t C, const uint16_t* x,
                    const uint16_t* w1, const uint16_t* b1, const uint16_t* w2, const uint16_t* b2,
                    float* logits, uint16_t* hidden, const int32_t* labels, float* loss, float* dlogits,
                    void* stream);

/* Backward pass: given x, hidden (from forward), w2 and dlogits, accumulate
 * FP32 gradients gw1[F*H], gb1[H], gw2[H*C], gb2[C] (overwritten, not added).
 * workspace: a caller-owned device buffer of at least
 * scg_mlp_backward_workspace(B, H, C) floats for the per-block partial sums
 * (SCG_ERANGE if smaller); calls that share one workspace must not overlap. */
int64_t scg_mlp_backward_workspace(int32_t B, int32_t H, int32_t C);
int scg_mlp_backward(int32_t B, int32_t F, int32_t H, int32_t C, const uint16_t* x, const uint16_t* hidden,
                     const uint16_t* w2, const float* dlogits,
                     float* gw1, float* gb1, float* gw2, float* gb2,
                     float* workspace, int64_t workspace_floats, void* stream);

/* Adam step on FP32 master weights p[n] with gradient g[n] and moments m, v
 * (all device), writing the FP16 copy p16[n].  step is 1-based. */
int scg_adam_step(int32_t n, float* p, const float* g, float* m, float* v, uint16_t* p16,
                  float lr, float beta1, float beta2, float eps, int32_t step, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SCROOGE_H */
