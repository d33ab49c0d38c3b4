// Input and output forms of the batch call besides ASCII in / run words out.
//
// repack2_kernel: sequences already encoded with two bits per base (32 bases
//   per uint64, base t of a word in bits 2t and 2t+1, every sequence starting
//   on a word boundary; the packed form of Section 2.5) become the planar
//   layout the alignment kernels read (Plane2: bit t of lo / hi is the low /
//   high code bit of base t, 64 bases per Plane2, one zero Plane2 after each
//   sequence).  The alignment kernels only compare codes, so the code
//   assignment is the caller's.  Bound by HBM bandwidth: one read of the
//   packed words, one write of the planes.
//
// ops_kernel: a pair's run words ((len << 2) | op, runs merged) become its
//   operation stream at two bits per operation (operation t of a pair in
//   byte t / 4, bits 2 (t % 4) and 2 (t % 4) + 1).  One wavefront per pair:
//   an inclusive scan of the run lengths gives every run's end position;
//   then each output byte finds the run holding its first operation by
//   binary search and fills its four operations, so every byte is written
//   once by one lane.
#include "internal.h"

namespace {

// the even bits (0, 2, ..., 62) of x gathered into bits 0..31
__device__ __forceinline__ uint32_t even_bits(uint64_t x) {
    x &= 0x5555555555555555ull;
    x = (x | (x >> 1)) & 0x3333333333333333ull;
    x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
    x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
    x = (x | (x >> 16)) & 0x00000000FFFFFFFFull;
    return (uint32_t)x;
}

// One thread per output Plane2 word; the owning sequence is found by binary
// search over the Plane2 offsets (npairs + 1 entries, first 0).
__global__ __launch_bounds__(256) void repack2_kernel(const uint64_t* __restrict__ in, const int64_t* __restrict__ inword,
                                                     const int32_t* __restrict__ len, const int64_t* __restrict__ wordoff,
                                                     int32_t nseq, int64_t total_words, Plane2* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < total_words; w += stride) {
        int lo = 0, hi = nseq - 1;   // last sequence whose first word is <= w
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (wordoff[mid] <= w) lo = mid;
            else hi = mid - 1;
        }
        const int64_t k = w - wordoff[lo];     // Plane2 index inside the sequence
        const int64_t n = len[lo];             // bases
        const int64_t b0 = 64 * k;             // first base of this word
        Plane2 p{0, 0};
        if (b0 < n) {
            const uint64_t* src = in + inword[lo] + 2 * k;
            const uint64_t x0 = src[0];
            const uint64_t x1 = b0 + 32 < n ? src[1] : 0ull;
            uint64_t plo = (uint64_t)even_bits(x0) | ((uint64_t)even_bits(x1) << 32);
            uint64_t phi = (uint64_t)even_bits(x0 >> 1) | ((uint64_t)even_bits(x1 >> 1) << 32);
            const int64_t keep = n - b0;       // bases of this word inside the sequence
            if (keep < 64) {
                const uint64_t m = (1ull << keep) - 1ull;
                plo &= m;
                phi &= m;
            }
            p = Plane2{plo, phi};
        }
        out[w] = p;
    }
}

__device__ __forceinline__ int64_t wave_incl_scan(int64_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

__global__ __launch_bounds__(64) void ops_kernel(const uint32_t* __restrict__ runs, const int64_t* __restrict__ runs_off,
                                                 const int32_t* __restrict__ n_runs, int32_t npairs,
                                                 int32_t* __restrict__ rend, uint8_t* __restrict__ ops,
                                                 const int64_t* __restrict__ ops_off, int32_t* __restrict__ n_ops) {
    const int lane = threadIdx.x;
    for (int p = blockIdx.x; p < npairs; p += gridDim.x) {
        const int64_t r0 = runs_off[p];
        const int nr = max(n_runs[p], 0);
        // run end positions (inclusive scan of the lengths), in the pair's slots of rend
        int64_t carry = 0;
        for (int base = 0; base < nr; base += 64) {
            const int j = base + lane;
            const int64_t l = j < nr ? (int64_t)(runs[r0 + j] >> 2) : 0;
            const int64_t s = wave_incl_scan(l) + carry;
            if (j < nr) rend[r0 + j] = (int32_t)s;
            carry = __shfl(s, 63, 64);
        }
        const int64_t total = carry;
        if (lane == 0) n_ops[p] = (int32_t)total;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        uint8_t* const out = ops + ops_off[p];
        const int64_t nbytes = (total + 3) >> 2;
        for (int64_t b = lane; b < nbytes; b += 64) {
            const int64_t t0 = 4 * b;
            int lo = 0, hi = nr - 1;   // first run whose end is > t0
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if ((int64_t)rend[r0 + mid] > t0) hi = mid;
                else lo = mid + 1;
            }
            uint32_t byte = 0;
            int r = lo;
            for (int e = 0; e < 4 && t0 + e < total; ++e) {
                while ((int64_t)rend[r0 + r] <= t0 + e) ++r;
                byte |= (runs[r0 + r] & 3u) << (2 * e);
            }
            out[b] = (uint8_t)byte;
        }
        // the next pair's scan reuses nothing of this one, but its lanes must not
        // overtake the reads above in rend of a neighbouring pair
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_repack2(const uint64_t* in, const int64_t* inword, const int32_t* len, const int64_t* wordoff,
                          int32_t nseq, int64_t total_words, Plane2* out, int num_cu, hipStream_t s) {
    if (total_words <= 0 || nseq <= 0) return hipSuccess;
    int64_t blocks = (total_words + 255) / 256;
    const int64_t cap = (int64_t)num_cu * 32;
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(repack2_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in, inword, len, wordoff, nseq,
                       total_words, out);
    return hipGetLastError();
}

hipError_t launch_runs_to_ops(const uint32_t* runs, const int64_t* runs_off, const int32_t* n_runs, int32_t npairs,
                              int32_t* rend, uint8_t* ops, const int64_t* ops_off, int32_t* n_ops, int num_cu,
                              hipStream_t s) {
    if (npairs <= 0) return hipSuccess;
    int64_t blocks = npairs;
    const int64_t cap = (int64_t)num_cu * 16;
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(ops_kernel, dim3((unsigned)blocks), dim3(64), 0, s, runs, runs_off, n_runs, npairs, rend, ops,
                       ops_off, n_ops);
    return hipGetLastError();
}
