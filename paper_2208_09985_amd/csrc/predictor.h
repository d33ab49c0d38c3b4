// Device functions of the learned row budget: per-window features and the
// FP16 MLP forward pass on MFMA.  Shared by the fused alignment kernel
// (inference inside the window loop) and the training kernels, so training
// and inference compute the same function.
#pragma once
#include "internal.h"

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// A 64-character window in planar form: bit t of lo/hi = code bits of char t.
struct WinPlanes {
    uint64_t plo, phi, tlo, thi;
    int32_t m_w, n_w;
};

// 64 characters starting at `pos` of a sequence in Plane2 form (bit t =
// character pos+t).  The sequence's padding Plane2 keeps base[q+1] in bounds
// for every pos inside the sequence.
__device__ __forceinline__ void load_window(const Plane2* __restrict__ base, int pos, uint64_t& lo, uint64_t& hi) {
    const int q = pos >> 6, r = pos & 63;
    const Plane2 a = base[q];
    const Plane2 b = base[q + 1];
    if (r == 0) {
        lo = a.lo;
        hi = a.hi;
    } else {
        lo = (a.lo >> r) | (b.lo << (64 - r));
        hi = (a.hi >> r) | (b.hi << (64 - r));
    }
}

__device__ __forceinline__ uint64_t low_bits(int n) {
    return n >= 64 ? ~0ull : (n <= 0 ? 0ull : ((1ull << n) - 1ull));
}

// Feature f (0..15) of a window:
//   f = 0..6   number of 4-mers starting at t with pattern[t..t+3] ==
//              text[t+delta .. t+delta+3], delta = f - 3, all inside the window
//   f = 7..13  number of t with pattern[t] == text[t+delta], delta = f - 10
//   f = 14     m_w,   f = 15  n_w
__device__ __forceinline__ int window_feature(const WinPlanes& w, int f) {
    if (f == 14) return w.m_w;
    if (f == 15) return w.n_w;
    const int delta = (f < 7 ? f : f - 7) - 3;
    // text shifted so that bit t holds text[t + delta]
    uint64_t tl, th;
    uint64_t valid = low_bits(w.m_w);
    if (delta >= 0) {
        tl = w.tlo >> delta;
        th = w.thi >> delta;
        valid &= low_bits(w.n_w - delta);               // t + delta < n_w
    } else {
        const int s = -delta;
        tl = w.tlo << s;
        th = w.thi << s;
        valid &= low_bits(w.n_w + s) & ~low_bits(s);    // s <= t < n_w + s
    }
    const uint64_t eq = ~(tl ^ w.plo) & ~(th ^ w.phi) & valid;
    if (f >= 7) return __popcll(eq);
    const uint64_t eq4 = eq & (eq >> 1) & (eq >> 2) & (eq >> 3);
    return __popcll(eq4);
}

// MLP weights laid out as MFMA operands for one 16-sample tile.
// GEMM1 (transposed): Ht[h][s] = sum_f W1[f][h] * X[s][f] + b1[h]
//   A = W1^T block b (hidden 16b..16b+15), B = X^T, C = bias.
// GEMM2 (transposed): Lt[c][s] = sum_h W2[h][c] * relu(Ht[h][s]) + b2[c]
//   A = W2^T, B = relu(Ht) -- GEMM1's D layout is exactly GEMM2's B layout.
// v_mfma_f32_16x16x16f16 operand layout: A[i][k] in lane i + 16*(k/4),
// element k%4; B[k][j] in lane j + 16*(k/4), element k%4; D[i][j] in lane
// j + 16*(i/4), element i%4.
struct MlpRegs {
    half4_t w1a[4];
    float4_t b1c[4];
    half4_t w2a[4];
    float4_t b2c;
};

__device__ inline void mlp_load_regs(MlpRegs& r, const __half* w1, const __half* b1, const __half* w2,
                                     const __half* b2, int H, int C, int lane) {
    const int col = lane & 15, grp = lane >> 4;
    for (int b = 0; b < 4; ++b) {
        for (int e = 0; e < 4; ++e) {
            const int f = 4 * grp + e;          // k of GEMM1 = feature
            const int h = 16 * b + col;         // i of GEMM1 = hidden
            r.w1a[b][e] = (h < H) ? (_Float16)__half2float(w1[f * H + h]) : (_Float16)0.0f;
            const int hb = 16 * b + 4 * grp + e;  // i of GEMM1's D = hidden (bias)
            r.b1c[b][e] = (hb < H) ? __half2float(b1[hb]) : 0.0f;
            const int hk = 16 * b + 4 * grp + e;  // k of GEMM2 = hidden
            r.w2a[b][e] = (hk < H && col < C) ? (_Float16)__half2float(w2[hk * C + col]) : (_Float16)0.0f;
        }
    }
    for (int e = 0; e < 4; ++e) {
        const int c = 4 * grp + e;
        r.b2c[e] = (c < C) ? __half2float(b2[c]) : 0.0f;
    }
}

// The same registers from a host-prepared blob: per lane 9 x 16 bytes in the
// order w1a[0..3] (32 B), w2a[0..3] (32 B), b1c[0..3] (64 B), b2c (16 B).
constexpr int kMlpOperandWords = 9;   // uint4 per lane

__device__ __forceinline__ void mlp_load_packed(MlpRegs& r, const uint4* __restrict__ blob, int lane) {
    const uint4* q = blob + kMlpOperandWords * lane;
    uint4 v[kMlpOperandWords];
    for (int i = 0; i < kMlpOperandWords; ++i) v[i] = q[i];
    __builtin_memcpy(&r.w1a[0], &v[0], 32);
    __builtin_memcpy(&r.w2a[0], &v[2], 32);
    __builtin_memcpy(&r.b1c[0], &v[4], 64);
    __builtin_memcpy(&r.b2c, &v[8], 16);
}

// x4: features 4*(lane/16)..+3 of sample lane%16, already scaled, as fp16.
// Returns logits: lane l holds classes 4*(l/16)+e of sample l%16.
// hid[b] receives relu(hidden) 16b + 4*(l/16) + e of sample l%16 (fp16).
__device__ __forceinline__ float4_t mlp_tile_forward(const MlpRegs& r, half4_t x4, half4_t hid[4]) {
    float4_t acc = r.b2c;
    for (int b = 0; b < 4; ++b) {
        float4_t h = __builtin_amdgcn_mfma_f32_16x16x16f16(r.w1a[b], x4, r.b1c[b], 0, 0, 0);
        half4_t hh;
        for (int e = 0; e < 4; ++e) hh[e] = (_Float16)(h[e] > 0.0f ? h[e] : 0.0f);
        hid[b] = hh;
        acc = __builtin_amdgcn_mfma_f32_16x16x16f16(r.w2a[b], hh, acc, 0, 0, 0);
    }
    return acc;
}

// feature scaling shared by training and inference
__device__ __forceinline__ _Float16 feature_to_input(int v) { return (_Float16)((float)v * (1.0f / 64.0f)); }
