// Allocation-free batch alignment: scg_align_batch_noalloc (include/scrooge.h).
//
// Every device buffer the plain column-block path needs besides the caller's
// inputs and outputs (2-bit planes, per-pair tables, the pair queue, counters
// and the stored rows of the traceback region) lives in one file-scope device
// array, `scratch`, of a fixed size.  Each device the library runs on holds
// its own copy for the life of the process; its device address is looked up
// once per device (noalloc_init, called from scg_create, or from the entry
// point's first call on a device) and only that address is handed to
// kernels.  The entry point then enqueues a setup kernel, the two pack
// kernels and the fused alignment kernel on the caller's stream and returns:
// no hipMalloc, hipFree, event or other allocating call.  Calls that overlap
// on one device share the array and therefore race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "../../include/scrooge.h"
#include "internal.h"

int capi_check_params(const scg_params* p);   // capi.cpp
int capi_from_hip(hipError_t e, const char* what);
int capi_ctx_device(const scg_ctx* c);

namespace {

constexpr int64_t kMaxPairs = SCG_NOALLOC_MAX_PAIRS;
constexpr int64_t kMaxBases = SCG_NOALLOC_MAX_BASES;               // per side
constexpr int64_t kPlaneWords = kMaxBases / 64 + 2 * kMaxPairs;    // >= sum over sequences of ceil(len/64) + 1
constexpr size_t kDentBytes = (size_t)SCG_NOALLOC_DENT_MIB << 20;  // stored rows of every wavefront

constexpr size_t up256(size_t x) { return (x + 255) / 256 * 256; }

// byte offsets of the regions inside `scratch`
constexpr size_t kPPlanes = 0;
constexpr size_t kTPlanes = kPPlanes + up256((size_t)kPlaneWords * sizeof(Plane2));
constexpr size_t kPWord = kTPlanes + up256((size_t)kPlaneWords * sizeof(Plane2));
constexpr size_t kTWord = kPWord + up256((size_t)(kMaxPairs + 1) * 8);
constexpr size_t kRunsOff = kTWord + up256((size_t)(kMaxPairs + 1) * 8);
constexpr size_t kPOff = kRunsOff + up256((size_t)(kMaxPairs + 1) * 8);   // sanitised CSR offsets
constexpr size_t kTOff = kPOff + up256((size_t)(kMaxPairs + 1) * 8);
constexpr size_t kPLen = kTOff + up256((size_t)(kMaxPairs + 1) * 8);
constexpr size_t kTLen = kPLen + up256((size_t)kMaxPairs * 4);
constexpr size_t kRing = kTLen + up256((size_t)kMaxPairs * 4);
constexpr size_t kBad = kRing + up256((size_t)kMaxPairs * 4);
constexpr size_t kQctl = kBad + up256((size_t)kMaxPairs);
constexpr size_t kStats = kQctl + 256;
constexpr size_t kDent = kStats + up256(ST_COUNT * 8);
constexpr size_t kScratchBytes = kDent + kDentBytes;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_ptr[kMaxDevices] = {};   // per device: the device address of `scratch`

template <class T>
__device__ __forceinline__ T* at(unsigned char* ws, size_t off) {
    return reinterpret_cast<T*>(ws + off);
}

// Per-pair tables for a batch whose CSR offsets are in device memory: lengths,
// Plane2 offsets (each sequence plus one zero padding word), run-word offsets
// (m + n + 1 per pair), the queue in input order, cleared counters.  One
// workgroup: a validation sweep, then a chunked exclusive scan.  If any offset
// is out of order or beyond the stated totals, every pair is given empty
// sequences and marked as bad input, so no later kernel reads outside the
// caller's buffers.
__global__ __launch_bounds__(1024) void noalloc_setup(const int64_t* __restrict__ pat_off,
                                                      const int64_t* __restrict__ txt_off, int32_t npairs,
                                                      int64_t ptotal, int64_t ttotal, unsigned char* ws) {
    __shared__ int bad_any;
    __shared__ int64_t part[3][1024];
    __shared__ int64_t carry[3];
    const int tid = threadIdx.x;
    if (tid == 0) {
        bad_any = 0;
        carry[0] = carry[1] = carry[2] = 0;
        uint32_t* q = at<uint32_t>(ws, kQctl);
        q[0] = 0;                   // head
        q[1] = (uint32_t)npairs;    // tail: the input order is queued
        q[2] = 0;                   // pairs finished
        q[3] = 0;
    }
    if (tid < ST_COUNT) at<unsigned long long>(ws, kStats)[tid] = 0;
    __syncthreads();
    int mine = 0;
    for (int i = tid; i <= npairs; i += 1024) {
        const int64_t p = pat_off[i], t = txt_off[i];
        if (p < 0 || p > ptotal || t < 0 || t > ttotal) mine = 1;
        if (i < npairs && (pat_off[i + 1] < p || txt_off[i + 1] < t)) mine = 1;
    }
    if (mine) atomicOr(&bad_any, 1);
    __syncthreads();
    const bool invalid = bad_any != 0;
    int64_t* pword = at<int64_t>(ws, kPWord);
    int64_t* tword = at<int64_t>(ws, kTWord);
    int64_t* roff = at<int64_t>(ws, kRunsOff);
    int64_t* poff = at<int64_t>(ws, kPOff);
    int64_t* toff = at<int64_t>(ws, kTOff);
    for (int base = 0; base < npairs; base += 1024) {
        const int i = base + tid;
        int64_t m = 0, n = 0, v[3] = {0, 0, 0};
        if (i < npairs) {
            if (!invalid) {
                m = pat_off[i + 1] - pat_off[i];
                n = txt_off[i + 1] - txt_off[i];
            }
            poff[i] = invalid ? 0 : pat_off[i];
            toff[i] = invalid ? 0 : txt_off[i];
            at<int32_t>(ws, kPLen)[i] = (int32_t)m;
            at<int32_t>(ws, kTLen)[i] = (int32_t)n;
            at<int32_t>(ws, kRing)[i] = i + 1;
            at<uint8_t>(ws, kBad)[i] = invalid ? 1 : 0;
            v[0] = (m + 63) / 64 + 1;
            v[1] = (n + 63) / 64 + 1;
            v[2] = m + n + 1;
        }
        // inclusive scan over the chunk (Hillis-Steele in shared memory)
        for (int c = 0; c < 3; ++c) part[c][tid] = v[c];
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            int64_t add[3] = {0, 0, 0};
            if (tid >= d)
                for (int c = 0; c < 3; ++c) add[c] = part[c][tid - d];
            __syncthreads();
            for (int c = 0; c < 3; ++c) part[c][tid] += add[c];
            __syncthreads();
        }
        if (i < npairs) {
            pword[i] = carry[0] + part[0][tid] - v[0];
            tword[i] = carry[1] + part[1][tid] - v[1];
            roff[i] = carry[2] + part[2][tid] - v[2];
        }
        __syncthreads();
        if (tid == 0)
            for (int c = 0; c < 3; ++c) carry[c] += part[c][1023];
        __syncthreads();
    }
    if (tid == 0) {
        pword[npairs] = carry[0];
        tword[npairs] = carry[1];
        roff[npairs] = carry[2];
        poff[npairs] = invalid ? 0 : pat_off[npairs];
        toff[npairs] = invalid ? 0 : txt_off[npairs];
    }
}

}  // namespace

// Look up this device's copy of `scratch` (with `device` current).  Called
// once per device; later calls return the kept address.
int noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return SCG_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return SCG_OK;
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return capi_from_hip(e, "hipGetDevice");
    if (cur != device) return SCG_EINVAL;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return capi_from_hip(e, "hipGetSymbolAddress(scratch)");
    if (!p) return SCG_EDEVICE;
    g_ptr[device] = static_cast<unsigned char*>(p);
    return SCG_OK;
}

extern "C" int scg_align_batch_noalloc(scg_ctx* c, const scg_params* params, int32_t npairs, const void* pat,
                                       const int64_t* pat_off, int64_t pat_total, const void* txt,
                                       const int64_t* txt_off, int64_t txt_total, void* stream, int32_t* edits,
                                       int32_t* text_end, int32_t* status, uint32_t* runs, int32_t* n_runs) {
    if (!c || npairs < 0 || pat_total < 0 || txt_total < 0) return SCG_EINVAL;
    int rc = capi_check_params(params);
    if (rc) return rc;
    // plain mode in the column-block kernel, input order (automatic order means input
    // order here), no yields or flags
    if (params->mode != SCG_MODE_PLAIN || params->W > 64 || params->kernel == SCG_KERNEL_ROWS ||
        params->order == SCG_ORDER_LONGEST_FIRST || params->yield_chars > 0 || params->flags != 0)
        return SCG_EINVAL;
    if (npairs > kMaxPairs || pat_total > kMaxBases || txt_total > kMaxBases) return SCG_ELIMIT;
    if (npairs == 0) return SCG_OK;
    if (!pat_off || !txt_off || !edits || !text_end || !status || !runs || !n_runs) return SCG_EINVAL;
    if ((pat_total > 0 && !pat) || (txt_total > 0 && !txt)) return SCG_EINVAL;
    const int device = capi_ctx_device(c);
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return capi_from_hip(e, "hipSetDevice");
    if ((rc = noalloc_init(device))) return rc;
    unsigned char* ws = g_ptr[device];
    hipStream_t s = (hipStream_t)stream;

    // launch shape: windows per wavefront as scg_batch_create picks them, the
    // grid capped by the stored-row region of the workspace
    const int num_cu = scg_device_cus(c);
    const int ns = params->slots > 0
                       ? (params->slots <= 4 ? 4 : params->slots <= 8 ? 8 : params->slots <= 10 ? 10
                          : params->slots <= 16 ? 16 : 32)
                       : (npairs >= 8 * num_cu ? 8 : 4);
    const int cap = params->W - params->O;
    int grid = cols_max_blocks_per_cu(false, ns, 0, cap, 0, false) * num_cu;
    if (params->waves_per_cu > 0) grid = std::min(grid, params->waves_per_cu * num_cu);
    grid = std::min<int64_t>(grid, (npairs + ns - 1) / ns);
    const size_t per_wave = cols_dent_bytes(1, cap, ns, false, 0);
    grid = (int)std::min<size_t>((size_t)grid, kDentBytes / per_wave);
    if (grid < 1) return SCG_ELIMIT;

    hipLaunchKernelGGL(noalloc_setup, dim3(1), dim3(1024), 0, s, pat_off, txt_off, npairs, pat_total, txt_total, ws);
    if ((e = hipGetLastError()) != hipSuccess) return capi_from_hip(e, "noalloc_setup");
    const int64_t* poff = reinterpret_cast<const int64_t*>(ws + kPOff);
    const int64_t* toff = reinterpret_cast<const int64_t*>(ws + kTOff);
    Plane2* pplanes = reinterpret_cast<Plane2*>(ws + kPPlanes);
    Plane2* tplanes = reinterpret_cast<Plane2*>(ws + kTPlanes);
    int64_t* pword = reinterpret_cast<int64_t*>(ws + kPWord);
    int64_t* tword = reinterpret_cast<int64_t*>(ws + kTWord);
    uint8_t* bad = reinterpret_cast<uint8_t*>(ws + kBad);
    // the pack kernel's word loop ends at each sequence's own word count, and
    // its reads stay below the stated totals
    if ((e = launch_pack((const uint8_t*)pat, poff, pword, npairs, kPlaneWords, pat_total, pplanes, bad, num_cu, s)) !=
        hipSuccess)
        return capi_from_hip(e, "pack (patterns)");
    if ((e = launch_pack((const uint8_t*)txt, toff, tword, npairs, kPlaneWords, txt_total, tplanes, bad, num_cu, s)) !=
        hipSuccess)
        return capi_from_hip(e, "pack (texts)");

    AlignArgs a{};
    a.pplanes = pplanes;
    a.tplanes = tplanes;
    a.pword = pword;
    a.tword = tword;
    a.plen = reinterpret_cast<const int32_t*>(ws + kPLen);
    a.tlen = reinterpret_cast<const int32_t*>(ws + kTLen);
    a.bad = bad;
    a.order = nullptr;   // the setup kernel queued the input order itself
    a.npairs = npairs;
    a.W = params->W;
    a.O = params->O;
    a.k = params->k;
    a.cap = cap;
    a.mode = SCG_MODE_PLAIN;
    a.fixed_rows = params->fixed_rows;
    a.ns = ns;
    a.ccols = cap + 1;
    a.edits = edits;
    a.text_end = text_end;
    a.status = status;
    a.runs = runs;
    a.runs_off = reinterpret_cast<const int64_t*>(ws + kRunsOff);
    a.n_runs = n_runs;
    a.ring = reinterpret_cast<int32_t*>(ws + kRing);
    a.qcap = npairs;
    a.qctl = reinterpret_cast<uint32_t*>(ws + kQctl);
    a.pstate = nullptr;   // read only by pairs that yield; yields are off
    a.yield_chars = 0;
    a.stats = reinterpret_cast<unsigned long long*>(ws + kStats);
    a.dent = reinterpret_cast<uint64_t*>(ws + kDent);
    a.dstride = cols_dent_stride(cap, ns);
    a.lds_rows = 0;   // every stored row in the workspace's global region
    a.edges = 0;
    a.ring_rows = 0;
    a.no_et = 0;
    if ((e = launch_align_cols(a, grid, ns, 0, s)) != hipSuccess) return capi_from_hip(e, "align (column blocks)");
    return SCG_OK;
}
