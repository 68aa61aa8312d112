// Learned closure: layout of the network state kept in the workspace.
// Internal to libtc (the ABI is include/tc.h).
#pragma once

#include <stdint.h>

namespace tc {

// erf by Abramowitz and Stegun, Handbook of Mathematical Functions, formula
// 7.1.26 (absolute error at most 1.5e-7 in exact arithmetic, about 5e-7 in
// FP32), extended to x < 0 by oddness;
// also returns exp(-x^2).  The network's GELU uses it in training and in
// inference alike.
__device__ __forceinline__ float erf_as(float x, float& ex2) {
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
    float p = fmaf(t, 1.061405429f, -1.453152027f);
    p = fmaf(t, p, 1.421413741f);
    p = fmaf(t, p, -0.284496736f);
    p = fmaf(t, p, 0.254829592f);
    p *= t;
    ex2 = __builtin_amdgcn_exp2f(-(ax * ax) * 1.44269504088896341f);
    return copysignf(fmaf(-p, ex2, 1.0f), x);
}

// GELU in its erf form, z (1 + erf(z / sqrt 2)) / 2, and its derivative
// (1 + erf(z / sqrt 2)) / 2 + z exp(-z^2 / 2) / sqrt(2 pi).
__device__ __forceinline__ float gelu_f(float z) {
    float e;
    return 0.5f * z * (1.0f + erf_as(z * 0.70710678118654752f, e));
}
__device__ __forceinline__ float gelu_grad_f(float z) {
    float e;
    const float er = erf_as(z * 0.70710678118654752f, e);
    return fmaf(z * e, 0.39894228040143268f, 0.5f * (1.0f + er));
}

// Canonical flat parameter order (FP32): W1 [10][64], b1 [64], W2 [64][64],
// b2 [64], W3 [64][3], b3 [3].
constexpr int kNIn = 10, kNHid = 64, kNOut = 3;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kNIn * kNHid;        // 640
constexpr int kOffW2 = kOffB1 + kNHid;               // 704
constexpr int kOffB2 = kOffW2 + kNHid * kNHid;       // 4800
constexpr int kOffW3 = kOffB2 + kNHid;               // 4864
constexpr int kOffB3 = kOffW3 + kNHid * kNOut;       // 5056
constexpr int kNParam = kOffB3 + kNOut;              // 5059

constexpr int kMlpBatchMax = 65536;                  // samples per training step
constexpr int kMlpBlock = 64;                        // samples per block (one wave)
constexpr int kMlpMaxBlocks = kMlpBatchMax / kMlpBlock;
constexpr int kResidMaxTargets = 65536;

// Network state in device memory.  The BF16 copies are padded for 16x16x16
// matrix-core tiles: W1 to [16][64] (input rows 10..15 zero), W3 to [64][16]
// (output columns 3..15 zero), b3 to 16.
struct MlpState {
    float master[kNParam];
    float m[kNParam];
    float v[kNParam];
    float b1[kNHid];
    float b2[kNHid];
    float b3[16];
    uint16_t w1[16 * kNHid];
    uint16_t w2[kNHid * kNHid];
    uint16_t w3[kNHid * 16];
    float loss;
    float pad[63];
    float partials[kMlpMaxBlocks][kNParam + 1];     // per block gradient sums and squared error
};

}  // namespace tc
