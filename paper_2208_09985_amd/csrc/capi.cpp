// C ABI of libscrooge_hip.so (declarations and contracts: include/scrooge.h).
//
// Host responsibilities: argument validation, workspace management (2-bit
// planes, queue, counters), queue order, launch shape, hipGraph capture of a
// batch's launch sequence, and timing with HIP events.  Every step of the
// alignment itself runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/scrooge.h"
#include "internal.h"

struct scg_ctx {
    int device = 0;
    int num_cu = 0;
    size_t lds_per_cu = 0;          // LDS bytes per CU
    size_t lds_per_block = 0;       // LDS bytes one workgroup may use
    bool has_model = false;
    int F = 0, H = 0, C = 0;
    __half* model_d = nullptr;      // w1 | b1 | w2 | b2
    int32_t* budget_d = nullptr;
    uint32_t* operands_d = nullptr; // per-lane MFMA operand blob (64 lanes x 144 B)
    scg_stats last{};               // stats of the last scg_align_batch
    // the stream of the off-track helper launches, shared by the context's batches and
    // created once: the runtime spreads streams over a few hardware queues, and a stream
    // per batch soon lands on the queue of the caller's stream, where the helper launch
    // then waits for the main launch to finish instead of running beside it
    hipStream_t help_stream = nullptr;
    std::mutex help_mu;
};

struct scg_batch {
    scg_ctx* ctx = nullptr;
    bool one = false;   // column blocks: one wavefront per SIMD
    // off-track helpers: a second launch of 4-window wavefronts on the context's helper stream
    int help_grid = 0;
    uint64_t* help_dent_d = nullptr;
    int32_t* hring_d = nullptr;
    int mig_k = 0, mig_d = 0, mig_cap = 0;
    hipStream_t s2 = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    scg_params p{};
    int32_t npairs = 0;
    // sequences (ASCII) on the device
    uint8_t* pat_d = nullptr;
    uint8_t* txt_d = nullptr;
    bool own_seq = false;
    int64_t* pat_off_d = nullptr;
    int64_t* txt_off_d = nullptr;
    // 2-bit planes
    Plane2* pplanes = nullptr;
    Plane2* tplanes = nullptr;
    int64_t pwords = 0, twords = 0;
    int64_t pbytes = 0, tbytes = 0;   // input bytes (the packer reads no further)
    int32_t input_kind = SCG_INPUT_ASCII;
    int64_t* pin_d = nullptr;         // packed input: first uint64 of each sequence (npairs + 1)
    int64_t* tin_d = nullptr;
    int64_t* pword_d = nullptr;
    int64_t* tword_d = nullptr;
    int32_t* plen_d = nullptr;
    int32_t* tlen_d = nullptr;
    uint8_t* bad_d = nullptr;
    int32_t* order_d = nullptr;
    int64_t* runs_off_d = nullptr;
    std::vector<int64_t> runs_off_h;
    uint32_t* qctl_d = nullptr;
    int32_t* ring_d = nullptr;
    int64_t qcap = 0;
    int32_t* pstate_d = nullptr;
    unsigned long long* stats_d = nullptr;
    uint64_t* dent_d = nullptr;     // column-block kernel: stored rows per group
    int dstride = 0;
    int lds_rows = 0;               // column-block kernel: stored rows kept in LDS
    int chain_waves_per_cu = 0;     // column-block kernel: wavefronts per CU for uneven lengths (0: occupancy)
    int long_k = 0;                 // off-track helpers: the longest pairs they hold from the start
    int main_grid = 0;              // > 0: the main launch's wavefronts (the rest of the SIMDs are the helpers')
    int help_lds_rows = 0;          // off-track helpers: stored rows kept in LDS, and the LDS bytes they take
    size_t help_lds = 0;
    // off-track helpers: idle polls (each 16 sleeps of 32 x 64 cycles) without a beat of the
    // main launch before a helper stops waiting; 4096 is some 55 ms.  The environment
    // variable SCG_HELPER_IDLE_POLLS (a count >= 0) replaces it when the batch is created
    int idle_limit = 1 << 12;
    int ring_rows = 0;              // column-block kernel: slots of the stored-row ring (0: 64 rows)
    bool cols = false;              // column-block kernel selected
    bool wide = false;              // windows of 65..128 characters (wide_kernel)
    bool lanes = false;             // one lane per pair, rows computed in order (lane_kernel)
    // launch shape
    int ns = 1;
    int grid = 1;
    size_t lds = 0;
    // timing: a ring of (pack start, align start, align end) events, one per run
    static constexpr int kRing = 256;
    hipEvent_t ev[kRing][3] = {};
    int ring_next = 0;      // slot of the next run
    int ring_pending = 0;   // runs recorded since the last scg_batch_stats
    bool timed = false;
    // captured launch sequence
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    const void* gkey[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
};

namespace {

thread_local char g_last_error[256] = "";

int from_hip(hipError_t e, const char* what = "HIP call") {
    if (e == hipSuccess) return SCG_OK;
    std::snprintf(g_last_error, sizeof g_last_error, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
    if (e == hipErrorOutOfMemory) return SCG_ENOMEM;
    return SCG_EDEVICE;
}

#define HIP_TRY(x)                                       \
    do {                                                 \
        hipError_t _e = (x);                             \
        if (_e != hipSuccess) return from_hip(_e, #x);   \
    } while (0)

// the context's helper stream, created on first use (the device is current)
int ctx_helper_stream(scg_ctx* c, hipStream_t* out) {
    std::lock_guard<std::mutex> lock(c->help_mu);
    if (!c->help_stream) {
        const int rc = from_hip(hipStreamCreateWithFlags(&c->help_stream, hipStreamNonBlocking), "helper stream");
        if (rc) {
            c->help_stream = nullptr;
            return rc;
        }
    }
    *out = c->help_stream;
    return SCG_OK;
}

template <class T>
int dev_alloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return from_hip(hipMalloc((void**)p, count * sizeof(T)));
}

bool valid_base(uint8_t c) {
    switch (c | 0x20) {
    case 'a': case 'c': case 'g': case 't': return true;
    default: return false;
    }
}

int check_params(const scg_params* p) {
    if (!p) return SCG_EINVAL;
    if (p->W < 1 || p->W > 128 || p->O < 0 || p->O >= p->W || p->k < 0 || p->k > p->W) return SCG_EINVAL;
    // windows wider than 64: plain mode in the column-block form only, no yields or ablations
    if (p->W > 64 && (p->mode != SCG_MODE_PLAIN || p->kernel == SCG_KERNEL_ROWS || p->yield_chars > 0 ||
                      (p->flags & (SCG_FLAG_NO_EARLY_TERMINATION | SCG_FLAG_STORE_ALL_COLUMNS | SCG_FLAG_ROWS_LDS |
                                   SCG_FLAG_STORE_EDGES | SCG_FLAG_ROW_RING))))
        return SCG_EINVAL;
    if (p->mode < SCG_MODE_PLAIN || p->mode > SCG_MODE_FIXED) return SCG_EINVAL;
    // column blocks without a learned budget also run 32 windows per wavefront
    const bool cols = p->kernel == SCG_KERNEL_COLUMNS || (p->kernel == SCG_KERNEL_AUTO && p->mode == SCG_MODE_PLAIN);
    const int max_slots = cols && p->mode != SCG_MODE_LEARNED ? 32 : kMaxSlots;
    if (p->slots < 0 || p->slots > max_slots || p->waves_per_cu < 0) return SCG_EINVAL;
    if (p->order != SCG_ORDER_INPUT && p->order != SCG_ORDER_LONGEST_FIRST && p->order != SCG_ORDER_AUTO)
        return SCG_EINVAL;
    if (p->mode == SCG_MODE_FIXED && (p->fixed_rows < 1 || p->fixed_rows > 64)) return SCG_EINVAL;
    if (p->mode == SCG_MODE_LEARNED && !(p->tau > 0.f && p->tau <= 1.f)) return SCG_EINVAL;
    if (p->yield_chars > 0 && p->yield_chars < p->W - p->O) return SCG_EINVAL;
    if (p->kernel < SCG_KERNEL_AUTO || p->kernel > SCG_KERNEL_LANES) return SCG_EINVAL;
    // one lane per pair: plain mode, W <= 64, no yields or flags besides the graph
    if (p->kernel == SCG_KERNEL_LANES &&
        (p->mode != SCG_MODE_PLAIN || p->W > 64 || p->yield_chars > 0 || (p->flags & ~SCG_FLAG_GRAPH)))
        return SCG_EINVAL;
    constexpr int32_t kAblations = SCG_FLAG_NO_EARLY_TERMINATION | SCG_FLAG_STORE_ALL_COLUMNS | SCG_FLAG_ROWS_LDS |
                                   SCG_FLAG_STORE_EDGES | SCG_FLAG_ROW_RING;
    if (p->flags & ~(SCG_FLAG_GRAPH | kAblations)) return SCG_EINVAL;
    if ((p->flags & kAblations) && (p->mode != SCG_MODE_PLAIN || p->kernel == SCG_KERNEL_ROWS)) return SCG_EINVAL;
    // the row ring keeps only the rows ending at d_w: it needs early termination and the
    // global region; 4, 8 or 16 windows per wavefront
    if ((p->flags & SCG_FLAG_ROW_RING) &&
        ((p->flags & (SCG_FLAG_NO_EARLY_TERMINATION | SCG_FLAG_ROWS_LDS)) || (p->slots > 8 && p->slots <= 10) ||
         p->slots > 16))
        return SCG_EINVAL;
    // edges are stored as whole 64-bit words, in global memory, with 4, 8 or 16 windows per wavefront
    if ((p->flags & SCG_FLAG_STORE_EDGES) && ((p->flags & SCG_FLAG_ROWS_LDS) || (p->slots > 16 && p->slots != 0) ||
                                               (p->slots > 8 && p->slots <= 10)))
        return SCG_EINVAL;
    // a whole SIMD per wavefront: plain mode in the column-block kernel, rows in
    // global memory, 4, 8 or 10 windows per wavefront
    if (p->one_per_simd < -1 || p->one_per_simd > 1) return SCG_EINVAL;
    if (p->offtrack_helpers < -1 || p->offtrack_helpers > 1) return SCG_EINVAL;
    // off-track helpers forced: plain mode in the column-block kernel, no yields or
    // ablations, 8, 10 or 16 windows per main wavefront (16 when the main launch
    // keeps rows in LDS)
    if (p->offtrack_helpers == 1 &&
        (p->mode != SCG_MODE_PLAIN || p->W > 64 || p->kernel == SCG_KERNEL_ROWS || p->kernel == SCG_KERNEL_LANES ||
         (p->flags & ~(SCG_FLAG_ROWS_LDS | SCG_FLAG_GRAPH)) != 0 || p->yield_chars > 0 || p->one_per_simd < 0 ||
         (p->slots != 0 && p->slots != 8 && p->slots != 10 && p->slots != 16) ||
         ((p->flags & SCG_FLAG_ROWS_LDS) && p->slots != 0 && p->slots != 16)))
        return SCG_EINVAL;
    if (p->one_per_simd == 1 &&
        (p->mode != SCG_MODE_PLAIN || p->W > 64 || p->kernel == SCG_KERNEL_ROWS || p->kernel == SCG_KERNEL_LANES ||
         (p->flags & (SCG_FLAG_ROWS_LDS | SCG_FLAG_STORE_EDGES | SCG_FLAG_ROW_RING)) || p->slots > 16))
        return SCG_EINVAL;
    return SCG_OK;
}

void free_batch(scg_batch* b) {
    if (!b) return;
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (auto& trip : b->ev)
        for (auto& e : trip)
            if (e) (void)hipEventDestroy(e);
    if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
    if (b->join_ev) (void)hipEventDestroy(b->join_ev);
    void* ptrs[] = {b->own_seq ? b->pat_d : nullptr, b->own_seq ? b->txt_d : nullptr, b->pat_off_d, b->txt_off_d,
                    b->pplanes, b->tplanes, b->pword_d, b->tword_d, b->plen_d, b->tlen_d, b->bad_d, b->order_d,
                    b->runs_off_d, b->qctl_d, b->ring_d, b->pstate_d, b->stats_d, b->dent_d, b->pin_d, b->tin_d,
                    b->help_dent_d, b->hring_d};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    delete b;
}

// ASCII bytes or pre-packed 2-bit words -> the planar layout of the kernels
int enqueue_pack(scg_batch* b, hipStream_t s) {
    const scg_ctx* c = b->ctx;
    if (b->input_kind == SCG_INPUT_PACKED2) {
        HIP_TRY(launch_repack2((const uint64_t*)b->pat_d, b->pin_d, b->plen_d, b->pword_d, b->npairs, b->pwords,
                               b->pplanes, c->num_cu, s));
        HIP_TRY(launch_repack2((const uint64_t*)b->txt_d, b->tin_d, b->tlen_d, b->tword_d, b->npairs, b->twords,
                               b->tplanes, c->num_cu, s));
        return SCG_OK;
    }
    HIP_TRY(launch_pack(b->pat_d, b->pat_off_d, b->pword_d, b->npairs, b->pwords, b->pbytes, b->pplanes, b->bad_d,
                        c->num_cu, s));
    HIP_TRY(launch_pack(b->txt_d, b->txt_off_d, b->tword_d, b->npairs, b->twords, b->tbytes, b->tplanes, b->bad_d,
                        c->num_cu, s));
    return SCG_OK;
}

int enqueue_run(scg_batch* b, hipStream_t s, int32_t* edits, int32_t* text_end, int32_t* status, uint32_t* runs,
                int32_t* n_runs, bool with_events) {
    const scg_ctx* c = b->ctx;
    hipEvent_t* ev = b->ev[b->ring_next];
    if (with_events) {
        for (int i = 0; i < 3; ++i)
            if (!ev[i]) HIP_TRY(hipEventCreate(&ev[i]));
        HIP_TRY(hipEventRecord(ev[0], s));
    }
    HIP_TRY(launch_reset(b->qctl_d, b->ring_d, b->qcap, b->order_d, b->stats_d, b->bad_d, b->npairs, s, b->hring_d,
                         b->long_k, b->pstate_d));
    int prc = enqueue_pack(b, s);
    if (prc) return prc;
    if (with_events) HIP_TRY(hipEventRecord(ev[1], s));
    AlignArgs a{};
    a.pplanes = b->pplanes;
    a.tplanes = b->tplanes;
    a.pword = b->pword_d;
    a.tword = b->tword_d;
    a.plen = b->plen_d;
    a.tlen = b->tlen_d;
    a.bad = b->bad_d;
    a.order = b->order_d;
    a.npairs = b->npairs;
    a.W = b->p.W;
    a.O = b->p.O;
    a.k = b->p.k;
    a.cap = b->p.W - b->p.O;
    a.mode = b->p.mode;
    a.fixed_rows = b->p.fixed_rows;
    a.ns = b->ns;
    a.ccols = a.cap + 1;
    if (b->p.mode == SCG_MODE_LEARNED) {
        const int F = c->F, H = c->H, C = c->C;
        a.model.operands = reinterpret_cast<const uint4*>(c->operands_d);
        a.model.w1 = c->model_d;
        a.model.b1 = c->model_d + F * H;
        a.model.w2 = c->model_d + F * H + H;
        a.model.b2 = c->model_d + F * H + H + H * C;
        a.model.budget_rows = c->budget_d;
        a.model.H = H;
        a.model.C = C;
        a.model.tau = b->p.tau;
    }
    a.edits = edits;
    a.text_end = text_end;
    a.status = status;
    a.runs = runs;
    a.runs_off = b->runs_off_d;
    a.n_runs = n_runs;
    a.ring = b->ring_d;
    a.qcap = b->qcap;
    a.qctl = b->qctl_d;
    a.pstate = b->pstate_d;
    a.yield_chars = b->p.yield_chars;
    a.stats = b->stats_d;
    a.dent = b->dent_d;
    a.dstride = b->dstride;
    a.lds_rows = b->lds_rows;
    a.edges = (b->p.flags & SCG_FLAG_STORE_EDGES) ? 1 : 0;
    a.ring_rows = b->ring_rows;
    a.no_et = (b->p.flags & SCG_FLAG_NO_EARLY_TERMINATION) ? 1 : 0;
    a.one_per_simd = b->one ? 1 : 0;
    a.hring = b->hring_d;
    a.mig_k = b->help_grid > 0 ? b->mig_k : 0;
    a.mig_d = b->mig_d;
    a.mig_cap = b->mig_cap;
    a.helper = 0;
    a.idle_limit = b->idle_limit;
    if (b->npairs > 0) {
        if (b->lanes) HIP_TRY(launch_align_lane(a, b->grid, s));
        else if (b->wide) HIP_TRY(launch_align_wide(a, b->grid, b->ns, s));
        else if (b->cols && b->help_grid > 0) {
            // main launch on s, helper launch on s2 after the queues are reset, joined back into s
            HIP_TRY(hipEventRecord(b->fork_ev, s));
            HIP_TRY(launch_align_cols(a, b->grid, b->ns, b->lds, s));
            HIP_TRY(hipStreamWaitEvent(b->s2, b->fork_ev, 0));
            AlignArgs h = a;
            h.helper = 1;
            h.mig_k = 0;
            h.yield_chars = 0;
            h.ns = kHelperSlots;
            h.dent = b->help_dent_d;
            h.dstride = cols_dent_stride(a.cap, kHelperSlots);
            h.lds_rows = b->help_lds_rows;
            HIP_TRY(launch_align_cols(h, b->help_grid, kHelperSlots, b->help_lds, b->s2));
            HIP_TRY(hipEventRecord(b->join_ev, b->s2));
            HIP_TRY(hipStreamWaitEvent(s, b->join_ev, 0));
        } else if (b->cols) HIP_TRY(launch_align_cols(a, b->grid, b->ns, b->lds, s));
        else HIP_TRY(launch_align(a, b->grid, b->lds, s));
    }
    if (with_events) {
        HIP_TRY(hipEventRecord(ev[2], s));
        b->ring_next = (b->ring_next + 1) % scg_batch::kRing;
        b->ring_pending = std::min(b->ring_pending + 1, scg_batch::kRing);
    }
    return SCG_OK;
}

}  // namespace

// Predictor file (little-endian): "SCGW", uint32 version 1, int32 F, H, C,
// int32 budget_rows[C], then FP16 w1[F*H], b1[H], w2[H*C], b2[C], row-major,
// and nothing after.
static int load_weights_file(scg_ctx* c, const char* path) {
    FILE* f = std::fopen(path, "rb");
    if (!f) {
        std::snprintf(g_last_error, sizeof g_last_error, "cannot open predictor file %s", path);
        return SCG_EINVAL;
    }
    std::vector<unsigned char> buf;
    unsigned char tmp[4096];
    size_t got;
    while ((got = std::fread(tmp, 1, sizeof tmp, f)) > 0) buf.insert(buf.end(), tmp, tmp + got);
    std::fclose(f);
    auto bad = [&](const char* why) {
        std::snprintf(g_last_error, sizeof g_last_error, "predictor file %s: %s", path, why);
        return SCG_EINVAL;
    };
    if (buf.size() < 20 || std::memcmp(buf.data(), "SCGW", 4) != 0) return bad("not a predictor file");
    int32_t hdr[4];
    std::memcpy(hdr, buf.data() + 4, sizeof hdr);
    const int32_t version = hdr[0], F = hdr[1], H = hdr[2], C = hdr[3];
    if (version != 1) return bad("unknown version");
    if (F != kFeatures || H < 1 || H > kMaxHidden || C < 1 || C > 4) return bad("unsupported shape");
    const size_t nh = (size_t)F * H + H + (size_t)H * C + C;
    if (buf.size() != 20 + 4 * (size_t)C + 2 * nh) return bad("wrong size");
    std::vector<int32_t> rows(C);
    std::memcpy(rows.data(), buf.data() + 20, 4 * (size_t)C);
    std::vector<uint16_t> w(nh);
    std::memcpy(w.data(), buf.data() + 20 + 4 * (size_t)C, 2 * nh);
    const uint16_t* w1 = w.data();
    const uint16_t* b1 = w1 + (size_t)F * H;
    const uint16_t* w2 = b1 + H;
    const uint16_t* b2 = w2 + (size_t)H * C;
    return scg_set_model(c, F, H, C, w1, b1, w2, b2, rows.data());
}

// helpers for the allocation-free entry point (noalloc.hip)
int capi_check_params(const scg_params* p) { return check_params(p); }
int capi_from_hip(hipError_t e, const char* what) { return from_hip(e, what); }
int capi_ctx_device(const scg_ctx* c) { return c->device; }

extern "C" {

const char* scg_strerror(int code) {
    switch (code) {
    case SCG_OK: return "ok";
    case SCG_EINVAL: return "invalid argument";
    case SCG_EALPHABET: return "character outside A/C/G/T";
    case SCG_ERANGE: return "buffer too small";
    case SCG_ENOMEM: return "out of memory";
    case SCG_EDEVICE: return "HIP runtime error";
    case SCG_ENOMODEL: return "no predictor loaded";
    case SCG_EINTERNAL: return "internal inconsistency";
    case SCG_ELIMIT: return "batch exceeds the allocation-free workspace";
    default: return "unknown status";
    }
}

const char* scg_last_hip_error(void) { return g_last_error; }

void scg_params_default(scg_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->W = 64;
    p->O = 24;
    p->k = 64;
    p->mode = SCG_MODE_PLAIN;
    p->order = SCG_ORDER_AUTO;
    p->fixed_rows = 15;
    p->tau = 0.8f;
    p->yield_chars = -1;
}

int scg_create(scg_ctx** out, int device, const char* weights_path) {
    if (!out) return SCG_EINVAL;
    *out = nullptr;
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return SCG_EINVAL;
    HIP_TRY(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    scg_ctx* c = new (std::nothrow) scg_ctx();
    if (!c) return SCG_ENOMEM;
    c->device = device;
    c->num_cu = prop.multiProcessorCount;
    c->lds_per_cu = prop.maxSharedMemoryPerMultiProcessor ? prop.maxSharedMemoryPerMultiProcessor
                                                          : prop.sharedMemPerMultiprocessor;
    c->lds_per_block = prop.sharedMemPerBlock;
    // device address of the allocation-free workspace (looked up once per
    // device; a failure here is reported by scg_align_batch_noalloc itself)
    (void)noalloc_init(device);
    if (weights_path) {
        const int rc = load_weights_file(c, weights_path);
        if (rc) {
            scg_destroy(c);
            return rc;
        }
    }
    *out = c;
    return SCG_OK;
}

void scg_destroy(scg_ctx* c) {
    if (!c) return;
    if (c->help_stream) {
        (void)hipSetDevice(c->device);
        (void)hipStreamDestroy(c->help_stream);
    }
    if (c->model_d) (void)hipFree(c->model_d);
    if (c->budget_d) (void)hipFree(c->budget_d);
    if (c->operands_d) (void)hipFree(c->operands_d);
    delete c;
}

int scg_device_cus(const scg_ctx* c) { return c ? c->num_cu : 0; }

int scg_set_model(scg_ctx* c, int32_t F, int32_t H, int32_t C, const uint16_t* w1, const uint16_t* b1,
                  const uint16_t* w2, const uint16_t* b2, const int32_t* budget_rows) {
    if (!c || !w1 || !b1 || !w2 || !b2 || !budget_rows) return SCG_EINVAL;
    if (F != kFeatures || H < 1 || H > kMaxHidden || C < 1 || C > 4) return SCG_EINVAL;
    for (int i = 0; i < C; ++i) {
        if (budget_rows[i] < 1 || budget_rows[i] > 64) return SCG_EINVAL;
        if (i > 0 && budget_rows[i] <= budget_rows[i - 1]) return SCG_EINVAL;
    }
    if (budget_rows[C - 1] < 64) return SCG_EINVAL;
    HIP_TRY(hipSetDevice(c->device));
    const size_t n = (size_t)F * H + H + (size_t)H * C + C;
    std::vector<uint16_t> blob(n);
    std::memcpy(blob.data(), w1, sizeof(uint16_t) * F * H);
    std::memcpy(blob.data() + F * H, b1, sizeof(uint16_t) * H);
    std::memcpy(blob.data() + F * H + H, w2, sizeof(uint16_t) * H * C);
    std::memcpy(blob.data() + F * H + H + H * C, b2, sizeof(uint16_t) * C);
    if (c->model_d) (void)hipFree(c->model_d);
    if (c->budget_d) (void)hipFree(c->budget_d);
    if (c->operands_d) (void)hipFree(c->operands_d);
    c->model_d = nullptr;
    c->budget_d = nullptr;
    c->operands_d = nullptr;
    c->has_model = false;
    // MFMA operand registers per lane (layout of mlp_load_packed): lane l
    // holds column l%16 and k-group l/16 of each 16x16x16 operand
    std::vector<uint32_t> op(64 * 36, 0);
    auto h2f = [](uint16_t x) {
        const uint32_t s = (x >> 15) & 1, e = (x >> 10) & 31, m = x & 1023;
        float v;
        if (e == 0) v = std::ldexp((float)m, -24);
        else if (e == 31) v = m ? NAN : INFINITY;
        else v = std::ldexp((float)(m | 1024), (int)e - 25);
        return s ? -v : v;
    };
    auto put_f = [&](int word, float v) { std::memcpy(&op[word], &v, 4); };
    auto put_h = [&](int lane, int idx, uint16_t v) {   // idx-th half of the lane's first 16 words
        uint32_t& w = op[lane * 36 + idx / 2];
        w = (idx & 1) ? ((w & 0xffffu) | ((uint32_t)v << 16)) : ((w & 0xffff0000u) | v);
    };
    for (int l = 0; l < 64; ++l) {
        const int col = l & 15, grp = l >> 4;
        const int fw = l * 36 + 16;
        for (int b = 0; b < 4; ++b)
            for (int e = 0; e < 4; ++e) {
                const int f = 4 * grp + e, h = 16 * b + col, hk = 16 * b + 4 * grp + e;
                put_h(l, b * 4 + e, h < H ? w1[f * H + h] : 0);                          // w1a
                put_h(l, 16 + b * 4 + e, (hk < H && col < C) ? w2[hk * C + col] : 0);    // w2a
                put_f(fw + b * 4 + e, hk < H ? h2f(b1[hk]) : 0.f);                      // b1c
            }
        for (int e = 0; e < 4; ++e) put_f(fw + 16 + e, (4 * grp + e) < C ? h2f(b2[4 * grp + e]) : 0.f);  // b2c
    }
    int rc = dev_alloc(&c->model_d, n);
    if (rc) return rc;
    rc = dev_alloc(&c->budget_d, (size_t)C);
    if (rc) return rc;
    HIP_TRY(hipMemcpy(c->model_d, blob.data(), n * sizeof(uint16_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->budget_d, budget_rows, C * sizeof(int32_t), hipMemcpyHostToDevice));
    rc = dev_alloc(&c->operands_d, op.size());
    if (rc) return rc;
    HIP_TRY(hipMemcpy(c->operands_d, op.data(), op.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    c->F = F;
    c->H = H;
    c->C = C;
    c->has_model = true;
    return SCG_OK;
}

int scg_batch_create(scg_ctx* c, const scg_params* params, int32_t npairs, const void* pat, const int64_t* pat_off,
                     const void* txt, const int64_t* txt_off, int32_t input_kind, int32_t where, void* stream,
                     scg_batch** out) {
    if (!out) return SCG_EINVAL;
    *out = nullptr;
    if (!c || npairs < 0 || !pat_off || !txt_off) return SCG_EINVAL;
    if (where != SCG_WHERE_HOST && where != SCG_WHERE_DEVICE) return SCG_EINVAL;
    if (input_kind != SCG_INPUT_ASCII && input_kind != SCG_INPUT_PACKED2) return SCG_EINVAL;
    const bool packed = input_kind == SCG_INPUT_PACKED2;
    int rc = check_params(params);
    if (rc) return rc;
    if (params->mode == SCG_MODE_LEARNED && !c->has_model) return SCG_ENOMODEL;
    if (pat_off[0] != 0 || txt_off[0] != 0) return SCG_EINVAL;
    for (int32_t i = 0; i < npairs; ++i) {
        const int64_t m = pat_off[i + 1] - pat_off[i], n = txt_off[i + 1] - txt_off[i];
        if (m < 0 || n < 0 || m > (1 << 30) || n > (1 << 30)) return SCG_EINVAL;
    }
    // ASCII: offsets count bytes.  Packed: offsets count bases, and sequence i
    // starts at uint64 word sum over j < i of ceil(len_j / 32).
    std::vector<int64_t> pin, tin;
    if (packed) {
        pin.assign(npairs + 1, 0);
        tin.assign(npairs + 1, 0);
        for (int32_t i = 0; i < npairs; ++i) {
            pin[i + 1] = pin[i] + (pat_off[i + 1] - pat_off[i] + 31) / 32;
            tin[i + 1] = tin[i] + (txt_off[i + 1] - txt_off[i] + 31) / 32;
        }
    }
    const int64_t pbytes = packed ? pin[npairs] * 8 : pat_off[npairs];
    const int64_t tbytes = packed ? tin[npairs] * 8 : txt_off[npairs];
    if ((pbytes > 0 && !pat) || (tbytes > 0 && !txt)) return SCG_EINVAL;
    if (where == SCG_WHERE_HOST && !packed) {
        const uint8_t* ps = (const uint8_t*)pat;
        const uint8_t* ts = (const uint8_t*)txt;
        for (int64_t i = 0; i < pbytes; ++i)
            if (!valid_base(ps[i])) return SCG_EALPHABET;
        for (int64_t i = 0; i < tbytes; ++i)
            if (!valid_base(ts[i])) return SCG_EALPHABET;
    }
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    scg_batch* b = new (std::nothrow) scg_batch();
    if (!b) return SCG_ENOMEM;
    b->ctx = c;
    b->p = *params;
    b->npairs = npairs;
    b->input_kind = input_kind;
    // automatic: column blocks for plain mode, error-row lanes when windows
    // start with a row budget (there lanes above the budget are saved)
    b->cols = params->kernel == SCG_KERNEL_COLUMNS ||
              (params->kernel == SCG_KERNEL_AUTO && params->mode == SCG_MODE_PLAIN);
    // automatic yields: the row-lane kernel hands pairs back every 1280
    // pattern characters; the column-block kernel keeps them (its passes
    // advance every pair by one window, so pairs finish together anyway)
    b->wide = params->W > 64;
    if (b->wide) b->cols = false;
    b->lanes = params->kernel == SCG_KERNEL_LANES;
    if (b->lanes) b->cols = false;
    // the row-lane kernel is the only one that yields by default; the one-lane
    // kernel never yields (its queue holds exactly the pairs)
    if (b->p.yield_chars < 0) b->p.yield_chars = (b->cols || b->wide || b->lanes) ? 0 : 1280;
    // windows wider than 64 read three planes words from their start: two padding words
    const int pad_words = b->wide ? 2 : 1;
    // host-side tables
    std::vector<int64_t> pw(npairs + 1), tw(npairs + 1);
    std::vector<int32_t> pl(npairs), tl(npairs);
    b->runs_off_h.assign(npairs + 1, 0);
    pw[0] = tw[0] = 0;
    for (int32_t i = 0; i < npairs; ++i) {
        pl[i] = (int32_t)(pat_off[i + 1] - pat_off[i]);
        tl[i] = (int32_t)(txt_off[i + 1] - txt_off[i]);
        pw[i + 1] = pw[i] + (pl[i] + 63) / 64 + pad_words;   // + zero padding Plane2s
        tw[i + 1] = tw[i] + (tl[i] + 63) / 64 + pad_words;
        b->runs_off_h[i + 1] = b->runs_off_h[i] + pl[i] + tl[i] + 1;
    }
    b->pwords = pw[npairs];
    b->twords = tw[npairs];
    b->pbytes = pbytes;
    b->tbytes = tbytes;
    // queue capacity: the initial order plus one entry per yield; a pair
    // yields only after advancing yield_chars pattern characters
    b->qcap = npairs;
    if (b->p.yield_chars > 0)
        for (int32_t i = 0; i < npairs; ++i) b->qcap += pl[i] / b->p.yield_chars + 1;
    std::vector<int32_t> order(npairs);
    std::iota(order.begin(), order.end(), 0);
    // automatic order: longest first when the pairs' lengths differ by more than a
    // tenth (coefficient of variation), so that long pairs do not start last
    bool longest_first = params->order == SCG_ORDER_LONGEST_FIRST;
    if (params->order == SCG_ORDER_AUTO && npairs > 1) {
        double sum = 0.0, sq = 0.0;
        for (int32_t i = 0; i < npairs; ++i) {
            const double l = (double)pl[i] + (double)tl[i];
            sum += l;
            sq += l * l;
        }
        const double mean = sum / npairs, var = std::max(0.0, sq / npairs - mean * mean);
        longest_first = mean > 0.0 && std::sqrt(var) > 0.1 * mean;
    }
    if (longest_first)
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t x, int32_t y) { return (int64_t)pl[x] + tl[x] > (int64_t)pl[y] + tl[y]; });
    // device workspace
    auto fail = [&](int code) {
        free_batch(b);
        return code;
    };
    if ((rc = dev_alloc(&b->pat_off_d, npairs + 1)) || (rc = dev_alloc(&b->txt_off_d, npairs + 1)) ||
        (rc = dev_alloc(&b->pplanes, (size_t)b->pwords)) || (rc = dev_alloc(&b->tplanes, (size_t)b->twords)) ||
        (rc = dev_alloc(&b->pword_d, npairs + 1)) || (rc = dev_alloc(&b->tword_d, npairs + 1)) ||
        (rc = dev_alloc(&b->plen_d, npairs)) || (rc = dev_alloc(&b->tlen_d, npairs)) ||
        (rc = dev_alloc(&b->bad_d, npairs)) || (rc = dev_alloc(&b->order_d, npairs)) ||
        (rc = dev_alloc(&b->runs_off_d, npairs + 1)) || (rc = dev_alloc(&b->qctl_d, kQcWords)) ||
        (rc = dev_alloc(&b->ring_d, (size_t)b->qcap)) || (rc = dev_alloc(&b->pstate_d, (size_t)npairs * 8)) ||
        (rc = dev_alloc(&b->stats_d, ST_COUNT)))
        return fail(rc);
    if (packed && ((rc = dev_alloc(&b->pin_d, npairs + 1)) || (rc = dev_alloc(&b->tin_d, npairs + 1)))) return fail(rc);
    if (where == SCG_WHERE_HOST) {
        b->own_seq = true;
        if ((rc = dev_alloc(&b->pat_d, (size_t)pbytes)) || (rc = dev_alloc(&b->txt_d, (size_t)tbytes))) return fail(rc);
        if (pbytes && (rc = from_hip(hipMemcpyAsync(b->pat_d, pat, pbytes, hipMemcpyHostToDevice, s)))) return fail(rc);
        if (tbytes && (rc = from_hip(hipMemcpyAsync(b->txt_d, txt, tbytes, hipMemcpyHostToDevice, s)))) return fail(rc);
    } else {
        b->pat_d = (uint8_t*)pat;
        b->txt_d = (uint8_t*)txt;
    }
    struct Up {
        void* dst;
        const void* src;
        size_t bytes;
    } ups[] = {{b->pat_off_d, pat_off, sizeof(int64_t) * (npairs + 1)},
               {b->txt_off_d, txt_off, sizeof(int64_t) * (npairs + 1)},
               {b->pword_d, pw.data(), sizeof(int64_t) * (npairs + 1)},
               {b->tword_d, tw.data(), sizeof(int64_t) * (npairs + 1)},
               {b->plen_d, pl.data(), sizeof(int32_t) * npairs},
               {b->tlen_d, tl.data(), sizeof(int32_t) * npairs},
               {b->order_d, order.data(), sizeof(int32_t) * npairs},
               {b->runs_off_d, b->runs_off_h.data(), sizeof(int64_t) * (npairs + 1)},
               {b->pin_d, packed ? pin.data() : nullptr, packed ? sizeof(int64_t) * (npairs + 1) : 0},
               {b->tin_d, packed ? tin.data() : nullptr, packed ? sizeof(int64_t) * (npairs + 1) : 0}};
    for (auto& u : ups)
        if (u.bytes && (rc = from_hip(hipMemcpyAsync(u.dst, u.src, u.bytes, hipMemcpyHostToDevice, s)))) return fail(rc);
    // host vectors die at return: wait for the copies
    if ((rc = from_hip(hipStreamSynchronize(s)))) return fail(rc);
    // launch shape
    const bool learned = params->mode == SCG_MODE_LEARNED;
    int per_cu;
    if (b->lanes) {
        b->ns = 64;   // a pair per lane
        b->lds = 0;
        per_cu = lane_max_blocks_per_cu();
    } else if (b->wide) {
        // 4 or 8 windows per wavefront (16 or 8 lanes of 8 or 16 columns each);
        // automatic: 8 with whole 128-bit entries (W - O > 95) once that still
        // gives every SIMD a wavefront, else 4 (with 8- or 12-byte entries the
        // larger grid of four-window wavefronts is the faster one)
        if (params->slots > 0) b->ns = params->slots > 4 ? 8 : 4;
        else b->ns = (params->W - params->O > 95 && npairs >= 8 * c->num_cu) ? 8 : 4;
        b->lds = 0;
        per_cu = wide_max_blocks_per_cu(b->ns, params->W - params->O);
    } else if (b->cols) {
        // windows per wavefront: 4, 8 or 16; automatic = enough wavefronts to
        // give every SIMD two of them
        // Each pair's windows run one after another, so the kernel lasts as long as
        // its slowest wavefront; one that shares a SIMD runs slower.  Automatic: 4
        // windows per wavefront for small batches, 8 while the wavefronts fit one per
        // SIMD, then 10 (six lanes of 12 columns) while those fit, else 8.
        const int64_t simds = (int64_t)kSimdsPerCu * c->num_cu;
        const bool plain_global = params->mode == SCG_MODE_PLAIN &&
                                  !(params->flags & (SCG_FLAG_ROWS_LDS | SCG_FLAG_STORE_EDGES | SCG_FLAG_ROW_RING));
        auto waves = [&](int ng) { return ((int64_t)npairs + ng - 1) / ng; };
        int64_t total_m = 0;
        for (int32_t i = 0; i < npairs; ++i) total_m += pl[i];
        // short reads (16 windows or fewer on average): their passes are short and
        // the skew of many lanes per window dominates, so fewer lanes per window
        // (16 windows per wavefront once those fill the SIMDs, else 8)
        const bool short_reads = npairs > 0 && total_m <= 16LL * (params->W - params->O) * npairs;
        if (params->slots > 0)
            b->ns = params->slots <= 4 ? 4
                  : params->slots <= 8 ? 8
                  : (params->slots <= 10 && !learned) ? 10
                  : params->slots <= 16 ? 16 : 32;
        else if (short_reads && params->mode == SCG_MODE_PLAIN) b->ns = waves(16) >= simds ? 16 : 8;
        else if (npairs < 8 * c->num_cu) b->ns = 4;
        else if (waves(8) > simds && waves(10) <= simds && plain_global && params->one_per_simd >= 0) b->ns = 10;
        else b->ns = 8;
        // Lengths that vary, longest first: the longest pair's chain of windows sets the
        // kernel's time once enough chains run beside it to cover the rest of the work,
        // so a launch needs about (all windows / longest chain) windows in flight.  When
        // that is fewer than the register-limited grid would hold, it runs 4-window
        // wavefronts, just enough of them per CU, and the SIMDs they share are shared
        // by fewer wavefronts.
        if (params->slots == 0 && params->waves_per_cu == 0 && plain_global && longest_first && !short_reads &&
            npairs >= 8 * c->num_cu && params->one_per_simd >= 0) {
            const int64_t capw = params->W - params->O;
            int64_t total_w = 0, max_w = 1;
            for (int32_t i = 0; i < npairs; ++i) {
                const int64_t w = (pl[i] + capw - 1) / capw;
                total_w += w;
                max_w = std::max(max_w, w);
            }
            const int64_t chains = (total_w + max_w - 1) / max_w;
            const int64_t need_waves = (chains + 3) / 4;
            const int occ = cols_max_blocks_per_cu(false, 4, 0, (int)capw, 0, false, false);
            if (need_waves < (int64_t)occ * c->num_cu) {
                b->ns = 4;
                b->chain_waves_per_cu = (int)std::max<int64_t>(1, (need_waves + c->num_cu - 1) / c->num_cu);
            }
        }
        b->one = plain_global && (b->ns == 4 || b->ns == 8 || b->ns == 10 || b->ns == 16) &&
                 (params->one_per_simd == 1 ||
                  (params->one_per_simd == 0 &&
                   (waves(b->ns) <= simds || (b->chain_waves_per_cu > 0 && b->chain_waves_per_cu <= kSimdsPerCu))));
        // Off-track helpers.  A pair that has lost the diagonal keeps d_w near W-O in
        // every window, and such pairs set the kernel's time; a second launch of
        // 4-window wavefronts (16 lanes of 4 columns) on the SIMDs the main launch
        // leaves free takes them over.  The main launch then runs 16 windows per
        // wavefront (unless slots says otherwise), one wavefront per SIMD.
        {
            const bool rows_lds = (params->flags & SCG_FLAG_ROWS_LDS) != 0;
            const bool ok = params->mode == SCG_MODE_PLAIN && (params->flags & ~(SCG_FLAG_ROWS_LDS | SCG_FLAG_GRAPH)) == 0 &&
                            params->yield_chars <= 0 && params->one_per_simd >= 0 && params->offtrack_helpers >= 0;
            const int mng = params->slots > 0 ? b->ns : 16;
            const int64_t mwaves = waves(mng);
            const bool long_pairs = npairs > 0 && total_m / npairs >= 32LL * (params->W - params->O);
            const bool fits = (mng == 8 || mng == 10 || mng == 16) && (!rows_lds || mng == 16) && mwaves + 1 <= simds;
            const bool want = params->offtrack_helpers == 1 ||
                              (long_pairs && params->W - params->O >= 30 && waves(4) >= simds && mwaves + 128 <= simds);
            if (ok && fits && want) {
                b->ns = mng;
                b->one = true;
                b->chain_waves_per_cu = 0;
                b->help_grid = (int)std::min<int64_t>(simds - mwaves, ((int64_t)npairs + kHelperSlots - 1) / kHelperSlots);
                b->mig_k = 3;
                b->mig_d = std::max(1, 3 * (params->W - params->O) / 5);
                b->mig_cap = b->help_grid * kHelperSlots;
                if (const char* e = std::getenv("SCG_HELPER_IDLE_POLLS")) {
                    char* end = nullptr;
                    const long v = std::strtol(e, &end, 10);
                    if (end != e && *end == '\0' && v >= 0 && v <= (1L << 24)) b->idle_limit = (int)v;
                }
                // the helpers keep the lowest stored rows of their windows in LDS (deep
                // windows: nearly all of them).  When the main launch keeps its rows in
                // global memory it uses no LDS, and when its 16-window wavefronts fill more
                // than half the SIMDs a CU holds at most two helper wavefronts, so each may
                // take half of the CU's LDS; otherwise a quarter (one wavefront per SIMD)
                const int hcap = params->W - params->O;
                const size_t rowb = (size_t)kHelperSlots * cols_lds_row_bytes(false, hcap, cols_dent_stride(hcap, kHelperSlots));
                const bool half = !rows_lds && 2 * mwaves >= simds;
                const size_t budget = std::min(c->lds_per_cu / (size_t)(half ? 2 : kSimdsPerCu), c->lds_per_block);
                const size_t reserve = 2048;   // the kernel's own shared records
                const int rows = budget > reserve ? (int)((budget - reserve) / rowb) : 0;
                b->help_lds_rows = std::min(rows, 64);
                b->help_lds = (size_t)b->help_lds_rows * rowb;
            }
        }
        // Lengths that vary, longest first, in a batch too large for the rule above and for
        // one wavefront per SIMD: the longest pairs' chains of windows set the time, so the
        // helper launch, one wavefront per CU, holds the longest pairs from the start, and
        // the main launch runs 16-window wavefronts one per SIMD on the other SIMDs, its
        // slots taking the other pairs from the queue as they free up; off-track pairs are
        // handed over as above while helper slots are free.
        if (b->help_grid == 0 && b->chain_waves_per_cu > kSimdsPerCu && params->mode == SCG_MODE_PLAIN &&
            (params->flags & ~SCG_FLAG_GRAPH) == 0 &&
            params->yield_chars <= 0 && params->one_per_simd >= 0 && params->offtrack_helpers >= 0 &&
            params->W - params->O >= 30 && c->num_cu >= 8) {
            const int h = c->num_cu;
            b->ns = 16;
            b->one = true;
            b->chain_waves_per_cu = 0;
            b->help_grid = h;
            b->main_grid = (int)simds - h;
            b->long_k = (int)std::min<int64_t>((int64_t)h * kHelperSlots * 3 / 4, npairs / 4);
            b->mig_k = 3;
            b->mig_d = std::max(1, 3 * (params->W - params->O) / 5);
            b->mig_cap = h * kHelperSlots;
            const int hcap = params->W - params->O;
            const size_t rowb = (size_t)kHelperSlots * cols_lds_row_bytes(false, hcap, cols_dent_stride(hcap, kHelperSlots));
            const size_t budget = std::min(c->lds_per_cu / 2, c->lds_per_block);   // at most one helper per CU
            const size_t reserve = 2048;
            const int rows = budget > reserve ? (int)((budget - reserve) / rowb) : 0;
            b->help_lds_rows = std::min(rows, 64);
            b->help_lds = (size_t)b->help_lds_rows * rowb;
        }
        // SCG_FLAG_ROWS_LDS: the lowest stored rows of each window in LDS, as
        // many as fit while every wavefront the batch needs (or the
        // register-limited maximum) stays resident on its CU
        const int cap = params->W - params->O;
        const bool edges = (params->flags & SCG_FLAG_STORE_EDGES) != 0;
        const bool lr = (params->flags & SCG_FLAG_ROWS_LDS) && (b->ns == 4 || b->ns == 8 || b->ns == 16);
        b->lds_rows = 0;
        b->lds = 0;
        // extended DENT: traceback reads at most W-O rows below d_w, and the lanes ahead
        // of column 0 store at most 64/ns rows above it before early termination
        b->ring_rows = 0;
        if (params->flags & SCG_FLAG_ROW_RING) {
            const int ring = cap + 64 / b->ns + 1;
            if (ring < 64) b->ring_rows = ring;
        }
        if (lr) {
            const int scap = (params->flags & SCG_FLAG_STORE_ALL_COLUMNS) ? 63 : cap;
            const size_t rowb = (size_t)b->ns * cols_lds_row_bytes(learned, cap, cols_dent_stride(scap, b->ns));
            int vg = cols_max_blocks_per_cu(learned, b->ns, 0, cap, 1, false);
            if (params->waves_per_cu > 0) vg = std::min(vg, params->waves_per_cu);
            const int64_t waves = (npairs + b->ns - 1) / b->ns;
            // one wavefront per SIMD (with the off-track helpers, which take the same share)
            const int resident = b->one ? kSimdsPerCu
                                        : (int)std::max<int64_t>(1, std::min<int64_t>(vg, (waves + c->num_cu - 1) / c->num_cu));
            const size_t budget = std::min(c->lds_per_cu / (size_t)resident, c->lds_per_block);
            const size_t reserve = 2048;   // the kernel's own shared records
            const int rows = budget > reserve ? (int)((budget - reserve) / rowb) : 0;
            b->lds_rows = std::min(rows, 64);
            b->lds = (size_t)b->lds_rows * rowb;
        }
        per_cu = cols_max_blocks_per_cu(learned, b->ns, b->lds, cap, b->lds_rows > 0 ? 1 : (b->ring_rows > 0 ? 2 : 0),
                                        edges, b->one);
    } else {
        b->ns = params->slots > 0 ? params->slots : (params->mode == SCG_MODE_PLAIN ? 1 : 4);
        b->lds = align_lds_bytes(params->W - params->O + 1, b->ns);
        per_cu = align_max_blocks_per_cu(b->lds, learned);
    }
    if (params->waves_per_cu > 0) per_cu = std::min(per_cu, params->waves_per_cu);
    if (b->chain_waves_per_cu > 0) per_cu = std::min(per_cu, b->chain_waves_per_cu);
    b->grid = std::max(1, per_cu * c->num_cu);
    if (b->main_grid > 0) b->grid = std::min(b->grid, b->main_grid);
    const int64_t need = (npairs + b->ns - 1) / b->ns;   // more wavefronts than slots-worth of pairs idle
    if (b->grid > need) b->grid = (int)std::max<int64_t>(1, need);
    if (b->lanes && npairs > 0) {
        if ((rc = dev_alloc(&b->dent_d, lane_dent_bytes(b->grid, params->W - params->O) / sizeof(uint64_t))))
            return fail(rc);
    }
    if (b->wide && npairs > 0) {
        const int cap = params->W - params->O;
        b->dstride = wide_dent_stride(cap, b->ns);
        if ((rc = dev_alloc(&b->dent_d, wide_dent_bytes(b->grid, cap, b->ns) / sizeof(uint64_t)))) return fail(rc);
    }
    if (b->cols && npairs > 0) {
        const int cap = params->W - params->O;
        // stored columns 0..cap (DENT), or all of them for the ablation
        const int scap = (params->flags & SCG_FLAG_STORE_ALL_COLUMNS) ? 63 : cap;
        b->dstride = cols_dent_stride(scap, b->ns);
        const bool edges = (params->flags & SCG_FLAG_STORE_EDGES) != 0;
        if ((rc = dev_alloc(&b->dent_d, cols_dent_bytes(b->grid, scap, b->ns, edges, b->ring_rows) / sizeof(uint64_t))))
            return fail(rc);
    }
    if (b->cols && npairs > 0 && b->help_grid > 0) {
        const int cap = params->W - params->O;
        if ((rc = dev_alloc(&b->help_dent_d, cols_dent_bytes(b->help_grid, cap, kHelperSlots, false, 0) / sizeof(uint64_t))) ||
            (rc = dev_alloc(&b->hring_d, (size_t)npairs)) ||
            (rc = ctx_helper_stream(b->ctx, &b->s2)) ||
            (rc = from_hip(hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming))) ||
            (rc = from_hip(hipEventCreateWithFlags(&b->join_ev, hipEventDisableTiming))))
            return fail(rc);
    }
    *out = b;
    return SCG_OK;
}

void scg_batch_destroy(scg_batch* b) {
    if (b) (void)hipSetDevice(b->ctx->device);
    free_batch(b);
}

int64_t scg_batch_runs_capacity(const scg_batch* b) { return b ? b->runs_off_h.back() : -1; }

int scg_batch_launch_shape(const scg_batch* b, int32_t* out) {
    if (!b || !out) return SCG_EINVAL;
    const int cap = b->p.W - b->p.O;
    const bool learned = b->p.mode == SCG_MODE_LEARNED;
    out[0] = b->wide ? 4 : (b->lanes ? SCG_KERNEL_LANES : (b->cols ? SCG_KERNEL_COLUMNS : SCG_KERNEL_ROWS));
    out[1] = b->ns;
    out[2] = b->grid;
    out[3] = (int32_t)b->lds;
    out[4] = b->one ? 1 : 0;
    out[6] = b->help_grid;
    out[7] = b->help_grid > 0 ? kHelperSlots : 0;
    out[8] = b->help_grid > 0 ? (int32_t)b->help_lds : 0;
    out[9] = b->long_k;
    if (b->wide) out[5] = cap <= 95 ? 96 : 128;
    else if (b->cols) out[5] = (b->p.flags & SCG_FLAG_STORE_EDGES) || learned ? 64 : (cap <= 31 ? 32 : (cap <= 47 ? 48 : 64));
    else if (b->lanes) out[5] = 64;
    else out[5] = 0;
    return SCG_OK;
}

int scg_batch_runs_offsets(const scg_batch* b, int64_t* out) {
    if (!b || !out) return SCG_EINVAL;
    std::memcpy(out, b->runs_off_h.data(), sizeof(int64_t) * b->runs_off_h.size());
    return SCG_OK;
}

int scg_batch_run(scg_batch* b, void* stream, int32_t* edits, int32_t* text_end, int32_t* status, uint32_t* runs,
                  int32_t* n_runs) {
    if (!b) return SCG_EINVAL;
    if (b->npairs > 0 && (!edits || !text_end || !status || !runs || !n_runs)) return SCG_EINVAL;
    HIP_TRY(hipSetDevice(b->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    // with the off-track helpers the launches are enqueued directly even under the graph
    // flag: a captured graph runs the helper branch on a stream the runtime picks, which
    // can share the main launch's hardware queue (the helpers then start late or only
    // after the main launch), and these batches run for milliseconds, so the launch
    // calls a graph saves do not matter
    if (!(b->p.flags & SCG_FLAG_GRAPH) || b->help_grid > 0) {
        b->timed = true;
        return enqueue_run(b, s, edits, text_end, status, runs, n_runs, true);
    }
    const void* key[6] = {edits, text_end, status, runs, n_runs, nullptr};
    bool same = b->gexec != nullptr;
    for (int i = 0; i < 6 && same; ++i) same = key[i] == b->gkey[i];
    if (!same) {
        if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->gexec = nullptr;
        b->graph = nullptr;
        hipStream_t cs;
        HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        int rc = e == hipSuccess ? enqueue_run(b, cs, edits, text_end, status, runs, n_runs, false) : from_hip(e);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        (void)hipStreamDestroy(cs);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        HIP_TRY(e2);
        b->graph = g;
        HIP_TRY(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
        for (int i = 0; i < 6; ++i) b->gkey[i] = key[i];
    }
    b->timed = true;
    hipEvent_t* ev = b->ev[b->ring_next];
    for (int i = 0; i < 3; ++i)
        if (!ev[i]) HIP_TRY(hipEventCreate(&ev[i]));
    HIP_TRY(hipEventRecord(ev[0], s));
    HIP_TRY(hipEventRecord(ev[1], s));
    HIP_TRY(hipGraphLaunch(b->gexec, s));
    HIP_TRY(hipEventRecord(ev[2], s));
    b->ring_next = (b->ring_next + 1) % scg_batch::kRing;
    b->ring_pending = std::min(b->ring_pending + 1, scg_batch::kRing);
    return SCG_OK;
}

int scg_batch_stats(scg_batch* b, scg_stats* out) {
    if (!b || !out) return SCG_EINVAL;
    std::memset(out, 0, sizeof(*out));
    HIP_TRY(hipSetDevice(b->ctx->device));
    if (!b->timed) return SCG_OK;
    const int last = (b->ring_next + scg_batch::kRing - 1) % scg_batch::kRing;
    HIP_TRY(hipEventSynchronize(b->ev[last][2]));
    unsigned long long st[ST_COUNT];
    HIP_TRY(hipMemcpy(st, b->stats_d, sizeof(st), hipMemcpyDeviceToHost));
    // in graph mode the pack/align split is not observable: everything counts as kernel time
    double ksum = 0.0, psum = 0.0;
    for (int r = 0; r < b->ring_pending; ++r) {
        hipEvent_t* ev = b->ev[(last + scg_batch::kRing - r) % scg_batch::kRing];
        float pack = 0.f, kern = 0.f;
        HIP_TRY(hipEventElapsedTime(&pack, ev[0], ev[1]));
        HIP_TRY(hipEventElapsedTime(&kern, ev[1], ev[2]));
        if (r == 0) {
            out->kernel_ms = kern;
            out->pack_ms = pack;
        }
        ksum += kern;
        psum += pack;
    }
    out->timed_runs = b->ring_pending;
    out->kernel_ms_avg = b->ring_pending ? ksum / b->ring_pending : 0.0;
    out->pack_ms_avg = b->ring_pending ? psum / b->ring_pending : 0.0;
    b->ring_pending = 0;
    out->windows = (int64_t)st[ST_WINDOWS];
    out->ops_alg = (int64_t)st[ST_OPS_ALG];
    out->fallback_windows = (int64_t)st[ST_FALLBACK];
    out->lane_steps = (int64_t)st[ST_LANE_STEPS];
    out->rounds = (int64_t)st[ST_ROUNDS];
    out->rows_budgeted = (int64_t)st[ST_ROWS];
    out->yields = (int64_t)st[ST_YIELDS];
    if (st[ST_ERRORS]) return SCG_EINTERNAL;
    return SCG_OK;
}

int scg_runs_to_cigar(const uint32_t* runs, int32_t n_runs, char* cigar, int32_t cap, int32_t* len) {
    if ((!runs && n_runs > 0) || n_runs < 0 || !len || (!cigar && cap > 0)) return SCG_EINVAL;
    static const char sym[4] = {'=', 'X', 'I', 'D'};
    int64_t need = 0;
    char tmp[16];
    for (int32_t i = 0; i < n_runs; ++i) need += std::snprintf(tmp, sizeof tmp, "%u%c", runs[i] >> 2, sym[runs[i] & 3]);
    *len = (int32_t)need;
    if (need + 1 > cap) return SCG_ERANGE;
    int64_t at = 0;
    for (int32_t i = 0; i < n_runs; ++i)
        at += std::snprintf(cigar + at, (size_t)(cap - at), "%u%c", runs[i] >> 2, sym[runs[i] & 3]);
    cigar[at] = '\0';
    return SCG_OK;
}

int scg_align(scg_ctx* c, const char* pattern, int32_t m, const char* text, int32_t n, int32_t W, int32_t O, int32_t k,
              int32_t* edits, int32_t* text_end, char* cigar, int32_t cigar_cap, int32_t* cigar_len) {
    if (!c || m < 0 || n < 0 || (m > 0 && !pattern) || (n > 0 && !text) || !edits || !text_end || !cigar_len)
        return SCG_EINVAL;
    scg_params p;
    scg_params_default(&p);
    p.W = W;
    p.O = O;
    p.k = k;
    const int64_t po[2] = {0, m}, to[2] = {0, n};
    scg_batch* b = nullptr;
    int rc = scg_batch_create(c, &p, 1, pattern, po, text, to, SCG_INPUT_ASCII, SCG_WHERE_HOST, nullptr, &b);
    if (rc) return rc;
    const int64_t cap = scg_batch_runs_capacity(b);
    int32_t* outs = nullptr;
    uint32_t* runs_d = nullptr;
    if ((rc = dev_alloc(&outs, 4)) || (rc = dev_alloc(&runs_d, (size_t)cap))) {
        if (outs) (void)hipFree(outs);
        scg_batch_destroy(b);
        return rc;
    }
    rc = scg_batch_run(b, nullptr, outs, outs + 1, outs + 2, runs_d, outs + 3);
    int32_t h[4] = {0, 0, 0, 0};
    std::vector<uint32_t> runs;
    if (!rc) rc = from_hip(hipMemcpy(h, outs, sizeof(h), hipMemcpyDeviceToHost));
    if (!rc) {
        runs.resize(std::max(0, h[3]));
        if (h[3] > 0) rc = from_hip(hipMemcpy(runs.data(), runs_d, sizeof(uint32_t) * h[3], hipMemcpyDeviceToHost));
    }
    (void)hipFree(outs);
    (void)hipFree(runs_d);
    scg_batch_destroy(b);
    if (rc) return rc;
    *edits = h[0];
    *text_end = h[1];
    if (h[2] == SCG_PAIR_ERROR) return SCG_EINTERNAL;
    return scg_runs_to_cigar(runs.data(), (int32_t)runs.size(), cigar, cigar_cap, cigar_len);
}

int scg_align_batch(scg_ctx* c, const scg_params* params, int32_t npairs, const void* pat, const int64_t* pat_off,
                    const void* txt, const int64_t* txt_off, int32_t input_kind, int32_t where, void* stream,
                    int32_t* edits, int32_t* text_end, int32_t* status, uint8_t* ops, const int64_t* ops_off,
                    int32_t* n_ops) {
    if (!c || npairs < 0 || !pat_off || !txt_off) return SCG_EINVAL;
    if (npairs > 0 && (!edits || !text_end || !status || !ops || !ops_off || !n_ops)) return SCG_EINVAL;
    // every pair's op stream needs ceil((m + n) / 4) bytes (an operation consumes a
    // pattern or a text character)
    for (int32_t i = 0; i < npairs; ++i) {
        const int64_t need = (pat_off[i + 1] - pat_off[i] + txt_off[i + 1] - txt_off[i] + 3) / 4;
        if (ops_off[i] < 0 || ops_off[i + 1] - ops_off[i] < need) return SCG_ERANGE;
    }
    scg_batch* b = nullptr;
    int rc = scg_batch_create(c, params, npairs, pat, pat_off, txt, txt_off, input_kind, where, stream, &b);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int64_t cap = scg_batch_runs_capacity(b);
    const bool host = where == SCG_WHERE_HOST;
    const int64_t obytes = npairs > 0 ? ops_off[npairs] : 0;
    uint32_t* runs_d = nullptr;
    int32_t* rend_d = nullptr;
    int32_t* nr_d = nullptr;
    int64_t* ooff_d = nullptr;
    int32_t* outs = nullptr;     // host outputs: edits, text_end, status, n_ops on the device
    uint8_t* ops_d = nullptr;
    if (npairs > 0) {
        if (!rc) rc = dev_alloc(&runs_d, (size_t)cap);
        if (!rc) rc = dev_alloc(&rend_d, (size_t)cap);
        if (!rc) rc = dev_alloc(&nr_d, (size_t)npairs);
        if (!rc) rc = dev_alloc(&ooff_d, (size_t)npairs + 1);
        if (!rc && host) rc = dev_alloc(&outs, 4 * (size_t)npairs);
        if (!rc && host) rc = dev_alloc(&ops_d, (size_t)std::max<int64_t>(obytes, 1));
        if (!rc) rc = from_hip(hipMemcpyAsync(ooff_d, ops_off, sizeof(int64_t) * (npairs + 1), hipMemcpyHostToDevice, s));
        int32_t* e = host ? outs : edits;
        int32_t* te = host ? outs + npairs : text_end;
        int32_t* st = host ? outs + 2 * (size_t)npairs : status;
        int32_t* no = host ? outs + 3 * (size_t)npairs : n_ops;
        uint8_t* od = host ? ops_d : ops;
        if (!rc) rc = scg_batch_run(b, stream, e, te, st, runs_d, nr_d);
        if (!rc) rc = from_hip(launch_runs_to_ops(runs_d, b->runs_off_d, nr_d, npairs, rend_d, od, ooff_d, no,
                                                  c->num_cu, s), "runs to ops");
        const size_t n4 = sizeof(int32_t) * (size_t)npairs;
        if (!rc && host) {
            rc = from_hip(hipMemcpyAsync(edits, e, n4, hipMemcpyDeviceToHost, s));
            if (!rc) rc = from_hip(hipMemcpyAsync(text_end, te, n4, hipMemcpyDeviceToHost, s));
            if (!rc) rc = from_hip(hipMemcpyAsync(status, st, n4, hipMemcpyDeviceToHost, s));
            if (!rc) rc = from_hip(hipMemcpyAsync(n_ops, no, n4, hipMemcpyDeviceToHost, s));
            if (!rc && obytes > 0) rc = from_hip(hipMemcpyAsync(ops, ops_d, (size_t)obytes, hipMemcpyDeviceToHost, s));
        }
        // the caller's host offsets and this call's buffers are in use until here
        const int src = from_hip(hipStreamSynchronize(s));
        if (!rc) rc = src;
    }
    scg_stats stt{};
    const int brc = rc ? rc : scg_batch_stats(b, &stt);
    for (void* q : {(void*)runs_d, (void*)rend_d, (void*)nr_d, (void*)ooff_d, (void*)outs, (void*)ops_d})
        if (q) (void)hipFree(q);
    scg_batch_destroy(b);
    if (brc && brc != SCG_EINTERNAL) return brc;
    c->last = stt;
    return brc;
}

int scg_last_stats(const scg_ctx* c, double* kernel_ms, int64_t* ops_alg, int64_t* fallback_windows) {
    if (!c) return SCG_EINVAL;
    if (kernel_ms) *kernel_ms = c->last.kernel_ms;
    if (ops_alg) *ops_alg = c->last.ops_alg;
    if (fallback_windows) *fallback_windows = c->last.fallback_windows;
    return SCG_OK;
}

int scg_last_stats_all(const scg_ctx* c, scg_stats* out) {
    if (!c || !out) return SCG_EINVAL;
    *out = c->last;
    return SCG_OK;
}

int scg_ops_to_cigar(const uint8_t* ops, int32_t n_ops, char* cigar, int32_t cap, int32_t* len) {
    if ((!ops && n_ops > 0) || n_ops < 0 || !len || (!cigar && cap > 0)) return SCG_EINVAL;
    static const char sym[4] = {'=', 'X', 'I', 'D'};
    auto op_at = [&](int32_t t) { return (ops[t >> 2] >> (2 * (t & 3))) & 3; };
    char tmp[16];
    int64_t need = 0;
    for (int32_t t = 0; t < n_ops;) {
        int32_t e = t;
        while (e < n_ops && op_at(e) == op_at(t)) ++e;
        need += std::snprintf(tmp, sizeof tmp, "%d%c", e - t, sym[op_at(t)]);
        t = e;
    }
    *len = (int32_t)need;
    if (need + 1 > cap) return SCG_ERANGE;
    int64_t at = 0;
    for (int32_t t = 0; t < n_ops;) {
        int32_t e = t;
        while (e < n_ops && op_at(e) == op_at(t)) ++e;
        at += std::snprintf(cigar + at, (size_t)(cap - at), "%d%c", e - t, sym[op_at(t)]);
        t = e;
    }
    cigar[at] = '\0';
    return SCG_OK;
}

int scg_features(scg_batch* b, int32_t nwin, const int32_t* windows, uint16_t* features, void* stream) {
    if (!b || nwin < 0 || (nwin > 0 && (!windows || !features))) return SCG_EINVAL;
    HIP_TRY(hipSetDevice(b->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    // planes are produced by the pack step of a run; make sure they exist
    HIP_TRY(launch_reset(b->qctl_d, b->ring_d, b->qcap, b->order_d, b->stats_d, b->bad_d, b->npairs, s, b->hring_d));
    int prc = enqueue_pack(b, s);
    if (prc) return prc;
    HIP_TRY(launch_features(b->pplanes, b->tplanes, b->pword_d, b->tword_d, b->plen_d, b->tlen_d, b->npairs, b->p.W,
                            nwin, windows, features, s));
    return SCG_OK;
}

int scg_mlp_forward(int32_t B, int32_t F, int32_t H, int32_t C, const uint16_t* x, const uint16_t* w1,
                    const uint16_t* b1, const uint16_t* w2, const uint16_t* b2, float* logits, uint16_t* hidden,
                    const int32_t* labels, float* loss, float* dlogits, void* stream) {
    if (B < 0 || F != kFeatures || H < 1 || H > kMaxHidden || C < 1 || C > 4) return SCG_EINVAL;
    if (B > 0 && (!x || !w1 || !b1 || !w2 || !b2 || !logits || !hidden)) return SCG_EINVAL;
    if (labels && (!loss || !dlogits)) return SCG_EINVAL;
    HIP_TRY(launch_mlp_forward(B, F, H, C, (const __half*)x, (const __half*)w1, (const __half*)b1,
                               (const __half*)w2, (const __half*)b2, logits, (__half*)hidden, labels, loss, dlogits,
                               (hipStream_t)stream));
    return SCG_OK;
}

int64_t scg_mlp_backward_workspace(int32_t B, int32_t H, int32_t C) {
    if (B < 0 || H < 1 || H > kMaxHidden || C < 1 || C > 4) return -1;
    return mlp_backward_workspace_floats(B, H, C);
}

int scg_mlp_backward(int32_t B, int32_t F, int32_t H, int32_t C, const uint16_t* x, const uint16_t* hidden,
                     const uint16_t* w2, const float* dlogits, float* gw1, float* gb1, float* gw2, float* gb2,
                     float* workspace, int64_t workspace_floats, void* stream) {
    if (B < 0 || F != kFeatures || H < 1 || H > kMaxHidden || C < 1 || C > 4) return SCG_EINVAL;
    if (!gw1 || !gb1 || !gw2 || !gb2) return SCG_EINVAL;
    if (B > 0 && (!x || !hidden || !w2 || !dlogits || !workspace)) return SCG_EINVAL;
    if (workspace_floats < mlp_backward_workspace_floats(B, H, C)) return SCG_ERANGE;
    HIP_TRY(launch_mlp_backward(B, F, H, C, (const __half*)x, (const __half*)hidden, (const __half*)w2, dlogits,
                                gw1, gb1, gw2, gb2, workspace, (hipStream_t)stream));
    return SCG_OK;
}

int scg_adam_step(int32_t n, float* p, const float* g, float* m, float* v, uint16_t* p16, float lr, float beta1,
                  float beta2, float eps, int32_t step, void* stream) {
    if (n < 0 || step < 1 || (n > 0 && (!p || !g || !m || !v || !p16))) return SCG_EINVAL;
    HIP_TRY(launch_adam(n, p, g, m, v, (__half*)p16, lr, beta1, beta2, eps, step, (hipStream_t)stream));
    return SCG_OK;
}

}  // extern "C"
