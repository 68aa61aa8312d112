// Learned closure: layout of the network state kept in the workspace.
// Internal to libtc (the ABI is include/tc.h).
#pragma once

#include <stdint.h>

namespace tc {

// GELU in its tanh form (Hendrycks and Gimpel, 2016),
//     gelu(z) = z (1 + tanh(c (z + a z^3))) / 2,  c = sqrt(2/pi), a = 0.044715,
// evaluated as z / (1 + 2^(-z (k0 + k1 z^2))) with k0 = 2 c log2(e) and
// k1 = a k0 (one exponential, one reciprocal), and its derivative
//     (1 + t)/2 + z (1 - t^2) c (1 + 3 a z^2) / 2,  t = tanh(c (z + a z^3)),
// with sigma = (1 + t)/2 = 1 / (1 + 2^(-z (k0 + k1 z^2))) and 1 - t^2 =
// 4 sigma (1 - sigma).  Training and inference both use these.
constexpr float kGeluK0 = 2.3022082f;        // 2 sqrt(2/pi) log2(e)
constexpr float kGeluK1 = 0.10294324f;       // 0.044715 * kGeluK0
constexpr float kGeluC = 0.7978845608f;      // sqrt(2/pi)
constexpr float kGeluA = 0.044715f;

__device__ __forceinline__ float gelu_sigma(float z) {
    const float v = z * fmaf(z * z, kGeluK1, kGeluK0);
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-v));
}
__device__ __forceinline__ float gelu_f(float z) { return z * gelu_sigma(z); }
__device__ __forceinline__ float gelu_grad_f(float z) {
    const float sg = gelu_sigma(z);
    const float dv = kGeluC * fmaf(3.0f * kGeluA, z * z, 1.0f);   // d/dz of c (z + a z^3)
    return fmaf(2.0f * z * sg * (1.0f - sg), dv, sg);
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

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef short short8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef float float2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned int uint2_t __attribute__((ext_vector_type(2)));

// The network's BF16 weights as matrix-core operand fragments, for
// inference on 16 samples at a time by one wave (net_tile).  Every layer is
// computed transposed, Z^T = W^T H^T: a 16x16 FP32 output tile gives lane l
// rows 4(l/16)..4(l/16)+3 of sample column l%16, which is what the next
// layer's B operand needs once the K order of that layer's weights follows
// the lanes: input unit sigma(kc, 8g + j) = 16 (2 kc + j/4) + 4 g + j%4 of K
// chunk kc sits in lane group g, slot j (its own outputs of hidden tiles
// 2kc and 2kc + 1).  Layer 1 uses 16x16x16 tiles (10 of 16 inputs used),
// layers 2 and 3 16x16x32 tiles (3 of layer 3's 16 output rows used).
struct NetF {
    short4_t f1[4][kNHid];       // [hidden tile][lane]: W1[4g + j][16 ht + r]
    short8_t f2[4][2][kNHid];    // [output tile][K chunk][lane]: W2[sigma(kc, 8g + j)][16 ht + r]
    short8_t f3[2][kNHid];       // [K chunk][lane]: W3[sigma(kc, 8g + j)][r] (r >= 3: 0)
    float b1[kNHid], b2[kNHid], b3[16];
};

__device__ __forceinline__ int net_sigma(int kc, int g, int j) { return 16 * (2 * kc + (j >> 2)) + 4 * g + (j & 3); }

// Fill the fragments from the state's padded BF16 copies; tid/nthreads split
// the work among the block's threads (a __syncthreads must follow).
__device__ inline void load_net_frags(const MlpState* __restrict__ st, NetF& N, int tid, int nthreads) {
    for (int i = tid; i < 4 * kNHid; i += nthreads) {
        const int ht = i / kNHid, l = i % kNHid, g = l >> 4, r = l & 15;
        short4_t v;
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = (short)st->w1[(4 * g + j) * kNHid + 16 * ht + r];
        N.f1[ht][l] = v;
    }
    for (int i = tid; i < 8 * kNHid; i += nthreads) {
        const int ht = i / (2 * kNHid), kc = (i / kNHid) & 1, l = i % kNHid, g = l >> 4, r = l & 15;
        short8_t v;
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = (short)st->w2[net_sigma(kc, g, j) * kNHid + 16 * ht + r];
        N.f2[ht][kc][l] = v;
    }
    for (int i = tid; i < 2 * kNHid; i += nthreads) {
        const int kc = i / kNHid, l = i % kNHid, g = l >> 4, r = l & 15;
        short8_t v;
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = (short)st->w3[net_sigma(kc, g, j) * 16 + r];
        N.f3[kc][l] = v;
    }
    for (int i = tid; i < kNHid; i += nthreads) {
        N.b1[i] = st->b1[i];
        N.b2[i] = st->b2[i];
    }
    for (int i = tid; i < 16; i += nthreads) N.b3[i] = st->b3[i];
}

// GELU of the four values, rounded to BF16 (nearest, ties to even) in pairs.
__device__ __forceinline__ short4_t gelu_pack(float4_t z) {
    const float2_t lo = {gelu_f(z[0]), gelu_f(z[1])}, hi = {gelu_f(z[2]), gelu_f(z[3])};
    const uint2_t u = {__builtin_bit_cast(unsigned, __builtin_convertvector(lo, bf16x2_t)),
                       __builtin_bit_cast(unsigned, __builtin_convertvector(hi, bf16x2_t))};
    return __builtin_bit_cast(short4_t, u);
}

__device__ __forceinline__ bf16x8_t cat8(short4_t a, short4_t b) {
    return __builtin_bit_cast(bf16x8_t, __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7));
}

// The network on 16 samples: lane l = 16 g + r supplies x = the BF16
// features 4g..4g+3 of sample r (zero beyond the tenth) and receives the
// outputs 4g..4g+3 of sample r: lanes 0..15 hold yhat (outputs 0..2, b3
// included) of samples 0..15.  Biases start the FP32 accumulators.
__device__ __forceinline__ float4_t net_tile(const NetF& N, short4_t x) {
    const int l = threadIdx.x & 63, g = l >> 4;
    short4_t h1[4], h2[4];
#pragma unroll
    for (int ht = 0; ht < 4; ++ht) {
        float4_t z = *reinterpret_cast<const float4_t*>(&N.b1[16 * ht + 4 * g]);
        z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(N.f1[ht][l], x, z, 0, 0, 0);
        h1[ht] = gelu_pack(z);
    }
    const bf16x8_t k0 = cat8(h1[0], h1[1]), k1 = cat8(h1[2], h1[3]);
#pragma unroll
    for (int ht = 0; ht < 4; ++ht) {
        float4_t z = *reinterpret_cast<const float4_t*>(&N.b2[16 * ht + 4 * g]);
        z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, N.f2[ht][0][l]), k0, z, 0, 0, 0);
        z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, N.f2[ht][1][l]), k1, z, 0, 0, 0);
        h2[ht] = gelu_pack(z);
    }
    float4_t y = *reinterpret_cast<const float4_t*>(&N.b3[4 * g]);
    y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, N.f3[0][l]), cat8(h2[0], h2[1]), y, 0, 0,
                                                0);
    y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, N.f3[1][l]), cat8(h2[2], h2[3]), y, 0, 0,
                                                0);
    return y;
}

// Round a float to BF16 (nearest, ties to even).
__device__ __forceinline__ short bf16_bits(float f) { return __builtin_bit_cast(short, (__bf16)f); }

}  // namespace tc
