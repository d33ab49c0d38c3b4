// Internal definitions shared by the HIP kernels and the C-ABI layer of
// libscrooge_hip.so.  Not part of the public interface (include/scrooge.h).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

// 64 bases in planar 2-bit form: bit t of `lo` / `hi` is the low / high bit
// of the code of base t (A=0, C=1, G=2, T=3).  Every sequence starts on a
// Plane2 boundary and is followed by one zero padding Plane2, so a 64-base
// window at any position inside the sequence reads two consecutive Plane2.
struct Plane2 {
    uint64_t lo, hi;
};

enum {
    ST_WINDOWS = 0,
    ST_OPS_ALG,
    ST_FALLBACK,
    ST_LANE_STEPS,
    ST_ROUNDS,
    ST_ROWS,
    ST_ERRORS,
    ST_YIELDS,
    ST_COUNT = 8
};

constexpr int kMaxSlots = 16;     // windows in flight per wavefront
constexpr int kSimdsPerCu = 4;    // SIMDs of a CDNA compute unit
constexpr int kHelperSlots = 4;   // windows per wavefront of the off-track helper launch
// queue-control words of the off-track helpers, 128 bytes apart (helpers poll them
// while the main launch updates the first three)
constexpr int kQcHHead = 32, kQcHTail = 64, kQcHInFlight = 96, kQcBeat = 128, kQcWords = 160;
// set in the in-flight word by a helper that stops waiting: every later hand-over
// then fails (the word exceeds any cap) and the main launch keeps its pairs
constexpr uint32_t kQcGateClosed = 0x80000000u;
constexpr int kMaxClasses = 16;   // predictor classes
constexpr int kMaxHidden = 64;
constexpr int kFeatures = 16;

struct ModelDev {
    const uint4* operands;  // per-lane MFMA operand registers (mlp_load_packed)
    const __half* w1;   // [F][H]
    const __half* b1;   // [H]
    const __half* w2;   // [H][C]
    const __half* b2;   // [C]
    const int32_t* budget_rows;  // [C]
    int32_t H, C;
    float tau;
};

struct AlignArgs {
    const Plane2* pplanes;
    const Plane2* tplanes;
    const int64_t* pword;   // first Plane2 of each pattern
    const int64_t* tword;   // first Plane2 of each text
    const int32_t* plen;
    const int32_t* tlen;
    const uint8_t* bad;     // nonzero: the pair's input held a non-ACGT byte
    const int32_t* order;   // queue order (pair indices)
    int32_t npairs;
    int32_t W, O, k, cap;   // cap = W - O: characters consumed per window
    int32_t mode, fixed_rows;
    int32_t ns;             // slots (windows in flight) per wavefront
    int32_t ccols;          // stored columns of the traceback region = cap + 1
    ModelDev model;
    int32_t* edits;
    int32_t* text_end;
    int32_t* status;
    uint32_t* runs;
    const int64_t* runs_off;
    int32_t* n_runs;
    // Pair queue: ring[q] = pair + 1 once written (0 = reserved, not yet
    // written).  Entries [0, npairs) hold the initial order; a pair that
    // yields is appended at qctl[1] with its state saved in pstate.
    int32_t* ring;
    int64_t qcap;
    uint32_t* qctl;               // [0] head, [1] tail, [2] pairs finished; with off-track
                                  // helpers, each on a cache line of its own: head and tail of
                                  // hring, pairs handed over and not finished, a beat of the
                                  // main launch (kQcHHead.. below)
    int32_t* pstate;              // per pair: p0, t0, edits, nruns, cur_op, cur_len, next_w, 0
    int32_t yield_chars;          // a pair yields after advancing this many pattern chars (<= 0: never)
    unsigned long long* stats;    // ST_COUNT counters
    // column-block kernel: stored rows of every group, [grid][NG][64][dstride] u64
    uint64_t* dent;
    int32_t dstride;
    int32_t lds_rows;             // rows 0..lds_rows-1 of each group's stored region are in LDS
    int32_t edges;                // ablation: stored slots hold edge bitvectors, not entries
    int32_t ring_rows;            // > 0: stored rows kept as a ring of this many slots (extended DENT)
    int32_t no_et;                // ablation: rows continue past d_w up to k_w
    int32_t one_per_simd;         // column blocks: the form that holds a whole SIMD per wavefront
    // Off-track helpers (column blocks, plain mode).  The main launch hands a pair
    // whose last mig_k windows all had d_w >= mig_d to hring (at most mig_cap such
    // pairs unfinished at a time); a helper launch (helper = 1, fewer windows and
    // more lanes per wavefront) takes pairs from hring only and resumes them.
    int32_t* hring;               // npairs entries, pair + 1 once written
    int32_t mig_k, mig_d, mig_cap;
    int32_t helper;
    int32_t idle_limit;           // helper: idle polls without a main-launch pass before it stops
                                  // waiting (closes the hand-over gate and leaves once every pair
                                  // handed over so far is finished)
};

// launchers (defined in the .hip files)
// hring (off-track helpers) is cleared, or, with long_k > 0, holds the first long_k pairs of
// the order from the start (their pstate zeroed) while the main queue starts after them
hipError_t launch_reset(uint32_t* qctl, int32_t* ring, int64_t qcap, const int32_t* order,
                        unsigned long long* stats, uint8_t* bad, int32_t npairs, hipStream_t s,
                        int32_t* hring = nullptr, int32_t long_k = 0, int32_t* pstate = nullptr);
hipError_t launch_pack(const uint8_t* seq, const int64_t* off, const int64_t* wordoff, int32_t npairs,
                       int64_t total_words, int64_t total_bytes, Plane2* out, uint8_t* bad, int num_cu, hipStream_t s);
hipError_t launch_align(const AlignArgs& a, int grid, size_t lds_bytes, hipStream_t s);
size_t align_lds_bytes(int ccols, int ns);
int align_max_blocks_per_cu(size_t lds_bytes, bool learned);
hipError_t launch_align_cols(const AlignArgs& a, int grid, int ng, size_t lds, hipStream_t s);
int cols_dent_stride(int cap, int ng);
size_t cols_lds_row_bytes(bool learned, int cap, int stride);
size_t cols_dent_bytes(int grid, int cap, int ng, bool edges, int ring_rows);
int cols_max_blocks_per_cu(bool learned, int ng, size_t lds, int cap, int sm, bool edges, bool one = false);
bool cols_one_per_simd_ok(bool learned, int ng, int sm, bool edges);
hipError_t launch_align_wide(const AlignArgs& a, int grid, int ng, hipStream_t s);
int wide_dent_stride(int cap, int ng);
size_t wide_dent_bytes(int grid, int cap, int ng);
int wide_max_blocks_per_cu(int ng, int cap);
hipError_t launch_features(const Plane2* pplanes, const Plane2* tplanes, const int64_t* pword,
                           const int64_t* tword, const int32_t* plen, const int32_t* tlen, int32_t npairs,
                           int32_t W, int32_t nwin, const int32_t* windows, uint16_t* features, hipStream_t s);
hipError_t launch_mlp_forward(int32_t B, int32_t F, int32_t H, int32_t C, const __half* x, const __half* w1,
                              const __half* b1, const __half* w2, const __half* b2, float* logits,
                              __half* hidden, const int32_t* labels, float* loss, float* dlogits,
                              hipStream_t s);
hipError_t launch_mlp_backward(int32_t B, int32_t F, int32_t H, int32_t C, const __half* x,
                               const __half* hidden, const __half* w2, const float* dlogits, float* gw1,
                               float* gb1, float* gw2, float* gb2, float* workspace, hipStream_t s);
int64_t mlp_backward_workspace_floats(int32_t B, int32_t H, int32_t C);
hipError_t launch_repack2(const uint64_t* in, const int64_t* inword, const int32_t* len, const int64_t* wordoff,
                          int32_t nseq, int64_t total_words, Plane2* out, int num_cu, hipStream_t s);
hipError_t launch_runs_to_ops(const uint32_t* runs, const int64_t* runs_off, const int32_t* n_runs, int32_t npairs,
                              int32_t* rend, uint8_t* ops, const int64_t* ops_off, int32_t* n_ops, int num_cu,
                              hipStream_t s);
size_t lane_dent_bytes(int grid, int cap);
int lane_max_blocks_per_cu();
hipError_t launch_align_lane(const AlignArgs& a, int grid, hipStream_t s);
int noalloc_init(int device);   // noalloc.hip: device address of its static workspace
hipError_t launch_adam(int32_t n, float* p, const float* g, float* m, float* v, __half* p16, float lr,
                       float b1, float b2, float eps, int32_t step, hipStream_t s);
