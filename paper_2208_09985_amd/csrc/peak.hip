// Microbenchmarks of the gfx950 resources that bound windowed GenASM:
// 32-bit bitwise VALU issue (the roofline's peak), the issue interval and
// dependent latency of a lone wavefront, LDS bandwidth and latency, and the
// latency of an L2-resident global load.  Built into libscrooge_peak.so, a
// measurement library separate from the alignment library; the benchmark
// script records its figures beside the alignment throughput.
//
// Every kernel touches only the buffers it is given, with indices reduced
// modulo their sizes, and runs a fixed number of iterations.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

extern "C" {
typedef struct {
    double valu_lane_ops_per_s;      // 32-bit bitwise lane-ops/s, all CUs, 8 wavefronts per SIMD
    double valu_t64_ops_per_s;       // the same as 64-bit operations (two 32-bit halves each)
    double lone_issue_cycles;        // cycles per independent VALU instruction, one wavefront on the GPU
    double lone_dep_cycles;          // cycles per dependent VALU instruction, one wavefront
    double lone_dpp_cycles;          // cycles per dependent DPP lane shift (with its wait state)
    double lds_bytes_per_s;          // ds_read_b128 bandwidth, all CUs
    double lds_lat_cycles;           // dependent LDS load
    double l2_lat_cycles;            // dependent global load, 1 MiB buffer (past the vector L1, inside L2)
    double sclk_mhz;                 // shader clock: s_memtime ticks per 100 MHz s_memrealtime tick
    double valu_kernel_ms;           // duration of the VALU throughput kernel (HIP events)
    int32_t num_cu;
    int32_t valu_waves;              // wavefronts of the VALU throughput kernel
} scg_peak_result;

int scg_peak_measure(int device, scg_peak_result* out);
}

namespace {

constexpr int kValuIters = 16384;   // 32 instructions per iteration and lane

__global__ __launch_bounds__(256) void valu_kernel(uint32_t* sink, uint32_t seed) {
    uint32_t a0 = seed ^ threadIdx.x, a1 = a0 * 3u, a2 = a0 * 5u, a3 = a0 * 7u;
    uint32_t a4 = a0 * 11u, a5 = a0 * 13u, a6 = a0 * 17u, a7 = a0 * 19u;
    const uint32_t c0 = seed * 0x9e3779b9u, c1 = c0 ^ 0x5bd1e995u;
    for (int it = 0; it < kValuIters; ++it) {
        // eight independent chains; each instruction is one 32-bit lane operation
        asm volatile(
            "v_alignbit_b32 %0, %0, %8, 1\n\t"
            "v_alignbit_b32 %1, %1, %8, 1\n\t"
            "v_alignbit_b32 %2, %2, %8, 1\n\t"
            "v_alignbit_b32 %3, %3, %8, 1\n\t"
            "v_alignbit_b32 %4, %4, %8, 1\n\t"
            "v_alignbit_b32 %5, %5, %8, 1\n\t"
            "v_alignbit_b32 %6, %6, %8, 1\n\t"
            "v_alignbit_b32 %7, %7, %8, 1\n\t"
            "v_or3_b32 %0, %0, %8, %9\n\t"
            "v_or3_b32 %1, %1, %8, %9\n\t"
            "v_or3_b32 %2, %2, %8, %9\n\t"
            "v_or3_b32 %3, %3, %8, %9\n\t"
            "v_or3_b32 %4, %4, %8, %9\n\t"
            "v_or3_b32 %5, %5, %8, %9\n\t"
            "v_or3_b32 %6, %6, %8, %9\n\t"
            "v_or3_b32 %7, %7, %8, %9\n\t"
            "v_and_or_b32 %0, %0, %9, %8\n\t"
            "v_and_or_b32 %1, %1, %9, %8\n\t"
            "v_and_or_b32 %2, %2, %9, %8\n\t"
            "v_and_or_b32 %3, %3, %9, %8\n\t"
            "v_and_or_b32 %4, %4, %9, %8\n\t"
            "v_and_or_b32 %5, %5, %9, %8\n\t"
            "v_and_or_b32 %6, %6, %9, %8\n\t"
            "v_and_or_b32 %7, %7, %9, %8\n\t"
            "v_xor_b32 %0, %0, %9\n\t"
            "v_xor_b32 %1, %1, %9\n\t"
            "v_xor_b32 %2, %2, %9\n\t"
            "v_xor_b32 %3, %3, %9\n\t"
            "v_xor_b32 %4, %4, %9\n\t"
            "v_xor_b32 %5, %5, %9\n\t"
            "v_xor_b32 %6, %6, %9\n\t"
            "v_xor_b32 %7, %7, %9"
            : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
            : "v"(c0), "v"(c1));
    }
    sink[blockIdx.x * blockDim.x + threadIdx.x] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
}

constexpr int kLoneIters = 4096;

// One wavefront: cycles of kLoneIters x 16 independent (mode 0) or
// dependent (mode 1) VALU instructions, or kLoneIters x 16 dependent DPP
// lane shifts (mode 2).  out[0] = s_memtime ticks, out[1] = s_memrealtime ticks.
__global__ __launch_bounds__(64) void lone_kernel(uint64_t* out, uint32_t* sink, int mode) {
    uint32_t a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3;
    const uint32_t c = 0x9e3779b9u;
    __builtin_amdgcn_s_waitcnt(0);
    const uint64_t t0 = __builtin_amdgcn_s_memtime();
    const uint64_t r0 = __builtin_amdgcn_s_memrealtime();
    if (mode == 0) {
        for (int it = 0; it < kLoneIters; ++it) {
            asm volatile(
                "v_or3_b32 %0, %0, %4, 1\n\t"
                "v_or3_b32 %1, %1, %4, 1\n\t"
                "v_or3_b32 %2, %2, %4, 1\n\t"
                "v_or3_b32 %3, %3, %4, 1\n\t"
                "v_alignbit_b32 %0, %0, %4, 1\n\t"
                "v_alignbit_b32 %1, %1, %4, 1\n\t"
                "v_alignbit_b32 %2, %2, %4, 1\n\t"
                "v_alignbit_b32 %3, %3, %4, 1\n\t"
                "v_and_or_b32 %0, %0, %4, %1\n\t"
                "v_and_or_b32 %1, %1, %4, %2\n\t"
                "v_and_or_b32 %2, %2, %4, %3\n\t"
                "v_and_or_b32 %3, %3, %4, %0\n\t"
                "v_xor_b32 %0, %0, %4\n\t"
                "v_xor_b32 %1, %1, %4\n\t"
                "v_xor_b32 %2, %2, %4\n\t"
                "v_xor_b32 %3, %3, %4"
                : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3)
                : "v"(c));
        }
    } else if (mode == 1) {
        for (int it = 0; it < kLoneIters; ++it) {
            asm volatile(
                "v_or3_b32 %0, %0, %1, 1\n\t"
                "v_alignbit_b32 %0, %0, %1, 1\n\t"
                "v_and_or_b32 %0, %0, %1, %0\n\t"
                "v_xor_b32 %0, %0, %1\n\t"
                "v_or3_b32 %0, %0, %1, 1\n\t"
                "v_alignbit_b32 %0, %0, %1, 1\n\t"
                "v_and_or_b32 %0, %0, %1, %0\n\t"
                "v_xor_b32 %0, %0, %1\n\t"
                "v_or3_b32 %0, %0, %1, 1\n\t"
                "v_alignbit_b32 %0, %0, %1, 1\n\t"
                "v_and_or_b32 %0, %0, %1, %0\n\t"
                "v_xor_b32 %0, %0, %1\n\t"
                "v_or3_b32 %0, %0, %1, 1\n\t"
                "v_alignbit_b32 %0, %0, %1, 1\n\t"
                "v_and_or_b32 %0, %0, %1, %0\n\t"
                "v_xor_b32 %0, %0, %1"
                : "+v"(a0)
                : "v"(c));
        }
    } else {
        for (int it = 0; it < kLoneIters; ++it) {
#pragma unroll
            for (int u = 0; u < 16; ++u) a0 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)a0, 0x130, 0xF, 0xF, true) + 1u;
        }
    }
    __builtin_amdgcn_s_waitcnt(0);
    const uint64_t t1 = __builtin_amdgcn_s_memtime();
    const uint64_t r1 = __builtin_amdgcn_s_memrealtime();
    if (threadIdx.x == 0) {
        out[0] = t1 - t0;
        out[1] = r1 - r0;
    }
    sink[threadIdx.x] = a0 ^ a1 ^ a2 ^ a3;
}

constexpr int kLdsWords = 4096;   // 64 KiB of uint4 per workgroup
constexpr int kLdsIters = 8192;

__global__ __launch_bounds__(256) void lds_bw_kernel(uint4* sink, uint32_t seed) {
    __shared__ uint4 buf[kLdsWords];
    for (int i = threadIdx.x; i < kLdsWords; i += blockDim.x) buf[i] = uint4{seed ^ i, seed + i, seed * i, ~seed ^ i};
    __syncthreads();
    uint4 acc{0, 0, 0, 0};
    // each lane reads consecutive 16-byte words: one ds_read_b128 per lane and iteration, no bank conflicts
    for (int it = 0; it < kLdsIters; ++it) {
        const uint4 v = buf[(threadIdx.x + it * 256) & (kLdsWords - 1)];
        acc.x ^= v.x;
        acc.y ^= v.y;
        acc.z ^= v.z;
        acc.w ^= v.w;
    }
    sink[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

constexpr int kChaseSteps = 4096;

// dependent loads: idx = table[idx], lane-uniform, from LDS (where = 0) or
// from a global table of `words` entries, a power of two (where = 1)
__global__ __launch_bounds__(64) void chase_kernel(const uint32_t* table, int words, int where, uint64_t* out,
                                                   uint32_t* sink) {
    __shared__ uint32_t lt[1024];
    for (int i = threadIdx.x; i < 1024; i += 64) lt[i] = (uint32_t)((i * 389 + 17) & 1023);
    __syncthreads();
    uint32_t idx = 0;
    __builtin_amdgcn_s_waitcnt(0);
    const uint64_t t0 = __builtin_amdgcn_s_memtime();
    if (where == 0) {
        for (int s = 0; s < kChaseSteps; ++s) idx = lt[idx & 1023];
    } else {
        for (int s = 0; s < kChaseSteps; ++s) idx = table[idx & (uint32_t)(words - 1)];
    }
    __builtin_amdgcn_s_waitcnt(0);
    const uint64_t t1 = __builtin_amdgcn_s_memtime();
    if (threadIdx.x == 0) out[0] = t1 - t0;
    sink[threadIdx.x] = idx;
}

struct Dev {
    void* p = nullptr;
    ~Dev() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

#define PK_CHECK(x)                          \
    do {                                     \
        if ((x) != hipSuccess) return -5;    \
    } while (0)

int scg_peak_measure(int device, scg_peak_result* out) {
    if (!out) return -1;
    *out = scg_peak_result{};
    PK_CHECK(hipSetDevice(device));
    hipDeviceProp_t prop;
    PK_CHECK(hipGetDeviceProperties(&prop, device));
    const int ncu = prop.multiProcessorCount;
    out->num_cu = ncu;

    // ---- VALU throughput: 8 wavefronts per SIMD (4 SIMDs per CU) ----
    const int vblocks = ncu * 8;   // 256 threads = 4 wavefronts per block
    Dev sink, times, table;
    const size_t sink_bytes = (size_t)ncu * 16 * 256 * sizeof(uint4);
    PK_CHECK(hipMalloc(&sink.p, sink_bytes));
    PK_CHECK(hipMalloc(&times.p, 64));
    hipEvent_t e0, e1;
    PK_CHECK(hipEventCreate(&e0));
    PK_CHECK(hipEventCreate(&e1));
    float best = 1e30f;
    for (int rep = 0; rep < 4; ++rep) {
        PK_CHECK(hipEventRecord(e0, 0));
        hipLaunchKernelGGL(valu_kernel, dim3(vblocks), dim3(256), 0, 0, (uint32_t*)sink.p, 0x1234u + rep);
        PK_CHECK(hipGetLastError());
        PK_CHECK(hipEventRecord(e1, 0));
        PK_CHECK(hipEventSynchronize(e1));
        float ms = 0;
        PK_CHECK(hipEventElapsedTime(&ms, e0, e1));
        if (rep > 0) best = std::min(best, ms);   // the first launch warms up
    }
    const double lane_ops = (double)vblocks * 256.0 * kValuIters * 32.0;
    out->valu_kernel_ms = best;
    out->valu_lane_ops_per_s = lane_ops / (best * 1e-3);
    out->valu_t64_ops_per_s = out->valu_lane_ops_per_s / 2.0;
    out->valu_waves = vblocks * 4;

    // ---- one wavefront alone on the GPU ----
    uint64_t h[2];
    double lone[3];
    double sclk = 0;
    for (int mode = 0; mode < 3; ++mode) {
        double bestc = 1e30;
        for (int rep = 0; rep < 3; ++rep) {
            hipLaunchKernelGGL(lone_kernel, dim3(1), dim3(64), 0, 0, (uint64_t*)times.p, (uint32_t*)sink.p, mode);
            PK_CHECK(hipGetLastError());
            PK_CHECK(hipMemcpy(h, times.p, sizeof h, hipMemcpyDeviceToHost));
            bestc = std::min(bestc, (double)h[0]);
            if (mode == 0 && h[1] > 0) sclk = std::max(sclk, (double)h[0] / (double)h[1] * 100.0);
        }
        lone[mode] = bestc / (kLoneIters * 16.0);
    }
    out->lone_issue_cycles = lone[0];
    out->lone_dep_cycles = lone[1];
    out->lone_dpp_cycles = lone[2];
    out->sclk_mhz = sclk;

    // ---- LDS bandwidth ----
    {
        const int lblocks = ncu * 2;   // two 64 KiB workgroups per CU
        best = 1e30f;
        for (int rep = 0; rep < 4; ++rep) {
            PK_CHECK(hipEventRecord(e0, 0));
            hipLaunchKernelGGL(lds_bw_kernel, dim3(lblocks), dim3(256), 0, 0, (uint4*)sink.p, 77u + rep);
            PK_CHECK(hipGetLastError());
            PK_CHECK(hipEventRecord(e1, 0));
            PK_CHECK(hipEventSynchronize(e1));
            float ms = 0;
            PK_CHECK(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) best = std::min(best, ms);
        }
        out->lds_bytes_per_s = (double)lblocks * 256.0 * kLdsIters * 16.0 / (best * 1e-3);
    }

    // ---- dependent load latency: LDS, then a 1 MiB global table ----
    {
        const int words = 1 << 18;
        std::vector<uint32_t> t(words);
        // a single cycle through all words with a 4 KiB stride between consecutive loads
        for (int i = 0; i < words; ++i) t[i] = (uint32_t)((i + 1031) % words);
        PK_CHECK(hipMalloc(&table.p, words * sizeof(uint32_t)));
        PK_CHECK(hipMemcpy(table.p, t.data(), words * sizeof(uint32_t), hipMemcpyHostToDevice));
        for (int where = 0; where < 2; ++where) {
            double bestc = 1e30;
            for (int rep = 0; rep < 3; ++rep) {
                hipLaunchKernelGGL(chase_kernel, dim3(1), dim3(64), 0, 0, (const uint32_t*)table.p, words, where,
                                   (uint64_t*)times.p, (uint32_t*)sink.p);
                PK_CHECK(hipGetLastError());
                PK_CHECK(hipMemcpy(h, times.p, sizeof(uint64_t), hipMemcpyDeviceToHost));
                bestc = std::min(bestc, (double)h[0]);
            }
            (where == 0 ? out->lds_lat_cycles : out->l2_lat_cycles) = bestc / kChaseSteps;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return 0;
}
