// Learned closure: layout of the network state kept in the workspace.
// Internal to libtc (the ABI is include/tc.h).
#pragma once

#include <stdint.h>

namespace tc {

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
