// Learned row budget: feature extraction and the predictor's training kernels
// (FP16 storage, FP32 accumulation).  Inference inside the alignment kernel
// uses the same window_feature / mlp_tile_forward device functions.
#include "predictor.h"

namespace {

// One thread per window (pair, p0, t0): 16 integer features.
__global__ __launch_bounds__(256) void features_kernel(const Plane2* __restrict__ pplanes,
                                                       const Plane2* __restrict__ tplanes,
                                                       const int64_t* __restrict__ pword,
                                                       const int64_t* __restrict__ tword,
                                                       const int32_t* __restrict__ plen,
                                                       const int32_t* __restrict__ tlen, int32_t npairs, int32_t W,
                                                       int32_t nwin, const int32_t* __restrict__ windows,
                                                       uint16_t* __restrict__ features) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nwin) return;
    const int pair = windows[3 * x], p0 = windows[3 * x + 1], t0 = windows[3 * x + 2];
    WinPlanes w{0, 0, 0, 0, 0, 0};
    if (pair < 0 || pair >= npairs || p0 < 0 || t0 < 0) {   // out-of-range window: all-zero features
        for (int f = 0; f < kFeatures; ++f) features[x * kFeatures + f] = 0;
        return;
    }
    const int m = plen[pair], n = tlen[pair];
    w.m_w = (p0 < m) ? min(W, m - p0) : 0;
    w.n_w = (t0 < n) ? min(W, n - t0) : 0;
    if (w.m_w > 0) load_window(pplanes + pword[pair], p0, w.plo, w.phi);
    if (w.n_w > 0) load_window(tplanes + tword[pair], t0, w.tlo, w.thi);
    for (int f = 0; f < kFeatures; ++f) features[x * kFeatures + f] = (uint16_t)window_feature(w, f);
}

// One wavefront per 16-sample tile.  F must be 16, H <= 64, C <= 4.
__global__ __launch_bounds__(64) void mlp_forward_kernel(int32_t B, int32_t H, int32_t C,
                                                         const __half* __restrict__ x,
                                                         const __half* __restrict__ w1,
                                                         const __half* __restrict__ b1,
                                                         const __half* __restrict__ w2,
                                                         const __half* __restrict__ b2, float* __restrict__ logits,
                                                         __half* __restrict__ hidden,
                                                         const int32_t* __restrict__ labels,
                                                         float* __restrict__ loss, float* __restrict__ dlogits) {
    const int lane = threadIdx.x;
    const int col = lane & 15, grp = lane >> 4;
    const int64_t sample = (int64_t)blockIdx.x * 16 + col;
    const bool in = sample < B;
    MlpRegs r;
    mlp_load_regs(r, w1, b1, w2, b2, H, C, lane);
    half4_t x4 = {0, 0, 0, 0};
    if (in)
        for (int e = 0; e < 4; ++e) x4[e] = (_Float16)__half2float(x[sample * kFeatures + 4 * grp + e]);
    half4_t hid[4];
    const float4_t lg = mlp_tile_forward(r, x4, hid);
    if (!in) return;
    for (int b = 0; b < 4; ++b)
        for (int e = 0; e < 4; ++e) {
            const int h = 16 * b + 4 * grp + e;
            if (h < H) hidden[sample * H + h] = __float2half((float)hid[b][e]);
        }
    if (grp != 0) return;  // lanes 0..15 hold classes 0..3 of their sample
    for (int c = 0; c < C; ++c) logits[sample * C + c] = lg[c];
    if (labels) {
        float mx = lg[0];
        for (int c = 1; c < C; ++c) mx = fmaxf(mx, lg[c]);
        float p[4], tot = 0.f;
        for (int c = 0; c < C; ++c) { p[c] = expf(lg[c] - mx); tot += p[c]; }
        const int y = labels[sample];
        loss[sample] = -(lg[y] - mx - logf(tot));
        const float inv = 1.0f / (float)B;
        for (int c = 0; c < C; ++c) dlogits[sample * C + c] = (p[c] / tot - (c == y ? 1.0f : 0.0f)) * inv;
    }
}

// Backward, stage 1: block b sums its chunk of samples into partial[b][*]
// laid out as [gw1 F*H | gb1 H | gw2 H*C | gb2 C].  One thread per hidden unit.
__global__ __launch_bounds__(64) void mlp_backward_partial(int32_t B, int32_t H, int32_t C, int32_t chunk,
                                                           const __half* __restrict__ x,
                                                           const __half* __restrict__ hidden,
                                                           const __half* __restrict__ w2,
                                                           const float* __restrict__ dlogits,
                                                           float* __restrict__ partial) {
    const int h = threadIdx.x;
    const int64_t s0 = (int64_t)blockIdx.x * chunk;
    const int64_t s1 = min((int64_t)B, s0 + chunk);
    const int P = kFeatures * H + H + H * C + C;
    float* out = partial + (int64_t)blockIdx.x * P;
    float gw1[kFeatures], gw2[4] = {0, 0, 0, 0}, gb1 = 0.f, gb2[4] = {0, 0, 0, 0};
    for (int f = 0; f < kFeatures; ++f) gw1[f] = 0.f;
    float w2h[4] = {0, 0, 0, 0};
    if (h < H)
        for (int c = 0; c < C; ++c) w2h[c] = __half2float(w2[h * C + c]);
    for (int64_t s = s0; s < s1; ++s) {
        float dl[4] = {0, 0, 0, 0};
        for (int c = 0; c < C; ++c) dl[c] = dlogits[s * C + c];
        if (h == 0)
            for (int c = 0; c < C; ++c) gb2[c] += dl[c];
        if (h >= H) continue;
        const float hv = __half2float(hidden[s * H + h]);
        float back = 0.f;
        for (int c = 0; c < C; ++c) {
            gw2[c] += hv * dl[c];
            back += w2h[c] * dl[c];
        }
        const float dh = hv > 0.f ? back : 0.f;
        gb1 += dh;
        for (int f = 0; f < kFeatures; ++f) gw1[f] += __half2float(x[s * kFeatures + f]) * dh;
    }
    if (h < H) {
        for (int f = 0; f < kFeatures; ++f) out[f * H + h] = gw1[f];
        out[kFeatures * H + h] = gb1;
        for (int c = 0; c < C; ++c) out[kFeatures * H + H + h * C + c] = gw2[c];
    }
    if (h == 0)
        for (int c = 0; c < C; ++c) out[kFeatures * H + H + H * C + c] = gb2[c];
}

// Backward, stage 2: sum the partials in block order (deterministic).
__global__ __launch_bounds__(256) void mlp_backward_reduce(int32_t nblocks, int32_t P, const float* __restrict__ partial,
                                                           float* __restrict__ g0, int32_t n0, float* __restrict__ g1,
                                                           int32_t n1, float* __restrict__ g2, int32_t n2,
                                                           float* __restrict__ g3, int32_t n3) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P) return;
    float acc = 0.f;
    for (int b = 0; b < nblocks; ++b) acc += partial[(int64_t)b * P + t];
    if (t < n0) g0[t] = acc;
    else if (t < n0 + n1) g1[t - n0] = acc;
    else if (t < n0 + n1 + n2) g2[t - n0 - n1] = acc;
    else if (t < n0 + n1 + n2 + n3) g3[t - n0 - n1 - n2] = acc;
}

__global__ __launch_bounds__(256) void adam_kernel(int32_t n, float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   __half* __restrict__ p16, float lr, float b1, float b2, float eps,
                                                   float c1, float c2) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.f - b1) * gt;
    const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    const float pt = p[t] - lr * (mt / c1) / (sqrtf(vt / c2) + eps);
    p[t] = pt;
    p16[t] = __float2half(pt);
}

}  // namespace

hipError_t launch_features(const Plane2* pplanes, const Plane2* tplanes, const int64_t* pword, const int64_t* tword,
                           const int32_t* plen, const int32_t* tlen, int32_t npairs, int32_t W, int32_t nwin,
                           const int32_t* windows, uint16_t* features, hipStream_t s) {
    if (nwin <= 0) return hipSuccess;
    hipLaunchKernelGGL(features_kernel, dim3((nwin + 255) / 256), dim3(256), 0, s, pplanes, tplanes, pword, tword,
                       plen, tlen, npairs, W, nwin, windows, features);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(int32_t B, int32_t F, int32_t H, int32_t C, const __half* x, const __half* w1,
                              const __half* b1, const __half* w2, const __half* b2, float* logits, __half* hidden,
                              const int32_t* labels, float* loss, float* dlogits, hipStream_t s) {
    (void)F;
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((B + 15) / 16), dim3(64), 0, s, B, H, C, x, w1, b1, w2, b2, logits,
                       hidden, labels, loss, dlogits);
    return hipGetLastError();
}

// per-block partial gradients: one row of P floats per chunk of samples
int64_t mlp_backward_workspace_floats(int32_t B, int32_t H, int32_t C) {
    if (B <= 0) return 0;
    const int chunk = 256;
    const int64_t nblocks = (B + chunk - 1) / chunk;
    return nblocks * (int64_t)(kFeatures * H + H + H * C + C);
}

hipError_t launch_mlp_backward(int32_t B, int32_t F, int32_t H, int32_t C, const __half* x, const __half* hidden,
                               const __half* w2, const float* dlogits, float* gw1, float* gb1, float* gw2, float* gb2,
                               float* g_partial, hipStream_t s) {
    (void)F;
    if (B <= 0) return hipSuccess;
    const int chunk = 256;
    const int nblocks = (B + chunk - 1) / chunk;
    const int P = kFeatures * H + H + H * C + C;
    hipLaunchKernelGGL(mlp_backward_partial, dim3(nblocks), dim3(64), 0, s, B, H, C, chunk, x, hidden, w2, dlogits,
                       g_partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mlp_backward_reduce, dim3((P + 255) / 256), dim3(256), 0, s, nblocks, P, g_partial, gw1,
                       kFeatures * H, gb1, H, gw2, H * C, gb2, C);
    return hipGetLastError();
}

hipError_t launch_adam(int32_t n, float* p, const float* g, float* m, float* v, __half* p16, float lr, float b1,
                       float b2, float eps, int32_t step, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const float c1 = 1.f - powf(b1, (float)step);
    const float c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, p, g, m, v, p16, lr, b1, b2, eps, c1,
                       c2);
    return hipGetLastError();
}
