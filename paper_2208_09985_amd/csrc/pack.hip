// Encode + pack: ASCII sequences to the planar 2-bit layout (Plane2).
//
// The paper's implementations convert each pair to a two-bit-per-base
// encoding before alignment (Section 2.5).  Here a wavefront produces forty
// Plane2 (64 bases each) per iteration from 2.5 KB of input staged in LDS with
// 16-byte loads; for each word, lane t reads byte t of the word's 64 bases,
// and two ballots over the code bits are exactly the low and high bit
// planes.  Lane u collects word u's planes, and one store writes all forty.
// The workload is a single pass over the input bytes, so it is bound by HBM
// bandwidth.
//
// The code of a base is bits 1 and 2 of its ASCII byte: A 0, C 1, T 2, G 3,
// the same for lower case (bit 5 is the case bit).  The kernels only compare
// codes for equality, so any one-to-one code of the four bases serves.
#include "internal.h"

namespace {

__global__ __launch_bounds__(256) void reset_kernel(uint32_t* qctl, int32_t* ring, int64_t qcap,
                                                    const int32_t* order, unsigned long long* stats, uint8_t* bad,
                                                    int32_t npairs, int32_t* hring, int32_t long_k, int32_t* pstate) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (t == 0) {
        qctl[0] = (uint32_t)long_k;  // head: the first long_k pairs of the order go to the helpers
        qctl[1] = (uint32_t)npairs;  // tail: the initial order is already queued
        qctl[2] = 0;                 // pairs finished
        if (hring) {
            // helper queue (holding the long pairs, in flight from the start) and beat
            qctl[kQcHHead] = 0;
            qctl[kQcHTail] = qctl[kQcHInFlight] = (uint32_t)long_k;
            qctl[kQcBeat] = 0;
        }
    }
    if (t < ST_COUNT) stats[t] = 0;
    for (int64_t x = t; x < npairs; x += stride) bad[x] = 0;
    if (hring)
        for (int64_t x = t; x < npairs; x += stride) {
            hring[x] = x < long_k ? order[x] + 1 : 0;
            if (x < long_k)
                for (int i = 0; i < 8; ++i) pstate[8 * (int64_t)order[x] + i] = 0;   // a pair from its start
        }
    for (int64_t x = t; x < qcap; x += stride) ring[x] = x < npairs ? order[x] + 1 : 0;
}

// 1 for the bytes a, c, g, t in either case, else 0
__device__ __forceinline__ uint32_t is_base(uint32_t c) {
    const uint32_t x = (c | 0x20u) - (uint32_t)'a';   // a 0, c 2, g 6, t 19
    return x < 20u ? (0x80045u >> x) & 1u : 0u;
}

// One workgroup per sequence (grid-stride over sequences): wave v of the
// block packs words 40v..40v+39, 40v+160..40v+199, ... of its sequence, so no
// word has to search for the sequence it belongs to.  A wave stages the 2.5 KB
// of its 40 words in LDS with aligned 16-byte loads (the
// chunk's start is arbitrary, so it loads from the 16-byte boundary below it
// and one block more), then reads one byte per lane per word from LDS.
constexpr int kChunkWords = 40;                 // words (64 bases each) per wave and iteration (a 10 kbp read in one)
constexpr int kStageBlocks = kChunkWords * 4 + 1;   // 16-byte blocks staged: the words and the misaligned tail

__global__ __launch_bounds__(256) void pack_kernel(const uint8_t* __restrict__ seq, const int64_t* __restrict__ off,
                                                   const int64_t* __restrict__ wordoff, int32_t npairs, int64_t total,
                                                   Plane2* __restrict__ out, uint8_t* __restrict__ bad) {
    __shared__ uint4 stage[4][kStageBlocks];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const uint8_t* const sb = reinterpret_cast<const uint8_t*>(stage[wave]);
    const uintptr_t sbase = reinterpret_cast<uintptr_t>(seq), send = sbase + (uintptr_t)total;
    for (int s = blockIdx.x; s < npairs; s += gridDim.x) {
        const int64_t start = off[s];
        const int64_t len = off[s + 1] - start;
        const int64_t w0 = wordoff[s];
        const int64_t nwords = wordoff[s + 1] - w0;   // (len + 63) / 64 + 1 padding word
        uint32_t bad_lane = 0;   // a non-base byte seen by this lane
        for (int64_t k0 = (int64_t)wave * kChunkWords; k0 < nwords; k0 += 4 * kChunkWords) {
            // 16-byte blocks at absolute 16-byte boundaries: a block that holds a byte
            // of the input lies in the input's pages, and blocks past its end are not read
            const uintptr_t p0 = sbase + (uintptr_t)(start + k0 * 64);   // first byte of the chunk
            const uintptr_t a0 = p0 & ~(uintptr_t)15;
            const int sh = (int)(p0 - a0);
            for (int blk = lane; blk < kStageBlocks; blk += 64) {
                const uintptr_t ba = a0 + 16u * (uintptr_t)blk;
                uint4 v{0u, 0u, 0u, 0u};
                if (ba < send) v = *reinterpret_cast<const uint4*>(ba);
                stage[wave][blk] = v;
            }
            // the wave reads bytes other lanes staged
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // word u's planes go to lane u (lo.x, lo.y, hi.x, hi.y)
            uint32_t w_lo0 = 0, w_lo1 = 0, w_hi0 = 0, w_hi1 = 0;
            // bases of the sequence in this chunk
            const int rem = (int)max((int64_t)0, min(len - k0 * 64, (int64_t)(kChunkWords * 64)));
#pragma unroll 8
            for (int u = 0; u < kChunkWords; ++u) {
                const uint32_t c = sb[sh + u * 64 + lane];
                const bool in = u * 64 + lane < rem;
                bad_lane |= in ? (is_base(c) ^ 1u) : 0u;
                const uint64_t plo = __ballot(in && (c & 2u) != 0);
                const uint64_t phi = __ballot(in && (c & 4u) != 0);
                const bool mine = lane == u;
                w_lo0 = mine ? (uint32_t)plo : w_lo0;
                w_lo1 = mine ? (uint32_t)(plo >> 32) : w_lo1;
                w_hi0 = mine ? (uint32_t)phi : w_hi0;
                w_hi1 = mine ? (uint32_t)(phi >> 32) : w_hi1;
            }
            if (lane < kChunkWords && k0 + lane < nwords)
                out[w0 + k0 + lane] = Plane2{(uint64_t)w_lo1 << 32 | w_lo0, (uint64_t)w_hi1 << 32 | w_hi0};
            // the next iteration overwrites the staged bytes
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (__ballot(bad_lane != 0) != 0 && lane == 0) bad[s] = 1;
    }
}

// Short sequences (up to kChunkWords words on average): one wavefront per
// sequence instead of one workgroup, staging only the 16-byte blocks the
// sequence covers and running the ballot loop over its own words only.  The
// planes written are those of pack_kernel.
__global__ __launch_bounds__(256) void pack_short_kernel(const uint8_t* __restrict__ seq,
                                                         const int64_t* __restrict__ off,
                                                         const int64_t* __restrict__ wordoff, int32_t npairs,
                                                         int64_t total, Plane2* __restrict__ out,
                                                         uint8_t* __restrict__ bad) {
    __shared__ uint4 stage[4][kStageBlocks];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const uint8_t* const sb = reinterpret_cast<const uint8_t*>(stage[wave]);
    const uintptr_t sbase = reinterpret_cast<uintptr_t>(seq), send = sbase + (uintptr_t)total;
    const int64_t nw_all = (int64_t)gridDim.x * 4;
    for (int64_t s = (int64_t)blockIdx.x * 4 + wave; s < npairs; s += nw_all) {
        const int64_t start = off[s];
        const int64_t len = off[s + 1] - start;
        const int64_t w0 = wordoff[s];
        const int64_t nwords = wordoff[s + 1] - w0;   // (len + 63) / 64 + 1 padding word
        uint32_t bad_lane = 0;
        for (int64_t k0 = 0; k0 < nwords; k0 += kChunkWords) {
            const uintptr_t p0 = sbase + (uintptr_t)(start + k0 * 64);
            const uintptr_t a0 = p0 & ~(uintptr_t)15;
            const int sh = (int)(p0 - a0);
            const int rem = (int)max((int64_t)0, min(len - k0 * 64, (int64_t)(kChunkWords * 64)));
            const int nblk = min(kStageBlocks, (sh + rem + 15) / 16);   // blocks holding the chunk's bases
            for (int blk = lane; blk < nblk; blk += 64) {
                const uintptr_t ba = a0 + 16u * (uintptr_t)blk;
                uint4 v{0u, 0u, 0u, 0u};
                if (ba < send) v = *reinterpret_cast<const uint4*>(ba);
                stage[wave][blk] = v;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            uint32_t w_lo0 = 0, w_lo1 = 0, w_hi0 = 0, w_hi1 = 0;
            const int nwc = (int)min((int64_t)kChunkWords, nwords - k0);   // words of this chunk (with the padding one)
            for (int u = 0; u < nwc; ++u) {
                const bool in = u * 64 + lane < rem;
                // bytes past the chunk's bases are not staged: read them only when in
                const uint32_t c = in ? sb[sh + u * 64 + lane] : 0u;
                bad_lane |= in ? (is_base(c) ^ 1u) : 0u;
                const uint64_t plo = __ballot(in && (c & 2u) != 0);
                const uint64_t phi = __ballot(in && (c & 4u) != 0);
                const bool mine = lane == u;
                w_lo0 = mine ? (uint32_t)plo : w_lo0;
                w_lo1 = mine ? (uint32_t)(plo >> 32) : w_lo1;
                w_hi0 = mine ? (uint32_t)phi : w_hi0;
                w_hi1 = mine ? (uint32_t)(phi >> 32) : w_hi1;
            }
            if (lane < nwc) out[w0 + k0 + lane] = Plane2{(uint64_t)w_lo1 << 32 | w_lo0, (uint64_t)w_hi1 << 32 | w_hi0};
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (__ballot(bad_lane != 0) != 0 && lane == 0) bad[s] = 1;
    }
}

}  // namespace

hipError_t launch_reset(uint32_t* qctl, int32_t* ring, int64_t qcap, const int32_t* order,
                        unsigned long long* stats, uint8_t* bad, int32_t npairs, hipStream_t s, int32_t* hring,
                        int32_t long_k, int32_t* pstate) {
    if (long_k > 0 && (!hring || !pstate || long_k > npairs)) return hipErrorInvalidValue;
    int64_t blocks = (qcap + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(reset_kernel, dim3((unsigned)blocks), dim3(256), 0, s, qctl, ring, qcap, order, stats, bad,
                       npairs, hring, long_k, pstate);
    return hipGetLastError();
}

hipError_t launch_pack(const uint8_t* seq, const int64_t* off, const int64_t* wordoff, int32_t npairs,
                       int64_t total_words, int64_t total_bytes, Plane2* out, uint8_t* bad, int num_cu, hipStream_t s) {
    if (total_words <= 0 || npairs <= 0) return hipSuccess;
    if (total_words <= (int64_t)npairs * kChunkWords) {
        // short sequences on average: a wavefront per sequence
        int64_t blocks = ((int64_t)npairs + 3) / 4;
        const int64_t cap = (int64_t)num_cu * 64;
        if (blocks > cap) blocks = cap;
        hipLaunchKernelGGL(pack_short_kernel, dim3((unsigned)blocks), dim3(256), 0, s, seq, off, wordoff, npairs,
                           total_bytes, out, bad);
        return hipGetLastError();
    }
    int64_t blocks = npairs;
    const int64_t cap = (int64_t)num_cu * 64;           // grid-stride over sequences beyond this
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(pack_kernel, dim3((unsigned)blocks), dim3(256), 0, s, seq, off, wordoff, npairs, total_bytes, out,
                       bad);
    return hipGetLastError();
}
