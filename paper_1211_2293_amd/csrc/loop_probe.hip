// Throughput of the force loop alone (a benchmark program, not part of
// libtc): every wave sums a 256-entry list held in LDS for its 64 bodies,
// over and over, with the same flush the walk kernels use (entry by entry
// in rounds of 8 or 4, and staged), at 5 and 8 resident waves per SIMD; and plain FP32 FMA
// chains, for the unpacked VALU peak.  It shows what the loop can reach on
// this chip when no walk shares the SIMD with it, which the 14 VALU
// instructions per entry and a 4-cycle issue per wave64 instruction do not
// tell: results are printed as interactions/s and TFLOP/s at 20 flops per
// interaction (3D).
//
// Usage: loop_probe [reps]   (one line per measurement on stdout)
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#include "walk_common.h"

namespace {

using namespace tc;
using namespace tc::walk;

#define PROBE_CHECK(x)                                                                       \
    do {                                                                                     \
        hipError_t e_ = (x);                                                                 \
        if (e_ != hipSuccess) {                                                              \
            std::fprintf(stderr, "loop_probe: %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            std::exit(1);                                                                    \
        }                                                                                    \
    } while (0)

constexpr int kWavesPerBlock = 4;

// Each rep moves the bodies by a tiny amount, so no rep's sums can be
// reused for the next; flush's LDS fences keep the list reads in the rep.
template <bool STAGED, int STEP>
__global__ void __launch_bounds__(kWavesPerBlock * kWave) k_probe_loop(const float4* __restrict__ list, int reps,
                                                                       float eps2, float* __restrict__ out) {
    __shared__ float4 s_list[kWavesPerBlock][kListCap];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    float4* L = s_list[wv];
    for (int j = lane; j < kListCap; j += kWave) L[j] = list[j];
    __syncthreads();
    const float xi = 0.01f * lane, yi = -0.02f * lane, zi = 0.005f * lane;
    Acc a = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int r = 0; r < reps; ++r)
        flush<3, false, STAGED, STEP>(L, kListCap, xi + 1e-7f * (float)r, yi, zi, eps2, a);
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = (a.sx + a.cx) + (a.sy + a.cy) + (a.sz + a.cz) + (a.sp + a.cp);
}

// Eight independent FMA chains per lane.
__global__ void __launch_bounds__(256) k_probe_fma(int iters, float b, float c, float* __restrict__ out) {
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = threadIdx.x * 1e-3f + (float)k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = fmaf(v[k], b, c);
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += v[k];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

float time_ms(hipEvent_t e0, hipEvent_t e1) {
    PROBE_CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    PROBE_CHECK(hipEventElapsedTime(&ms, e0, e1));
    return ms;
}

template <bool STAGED, int STEP = 8>
void probe_loop(int cus, int waves_per_simd, int reps, const float4* list, float* out, hipEvent_t e0, hipEvent_t e1) {
    const int blocks = cus * waves_per_simd;          // 4 waves per block: waves_per_simd per SIMD
    for (int pass = 0; pass < 3; ++pass) {            // the first pass warms up
        PROBE_CHECK(hipEventRecord(e0, 0));
        hipLaunchKernelGGL((k_probe_loop<STAGED, STEP>), dim3(blocks), dim3(kWavesPerBlock * kWave), 0, 0, list,
                           reps, 1e-4f, out);
        PROBE_CHECK(hipGetLastError());
        PROBE_CHECK(hipEventRecord(e1, 0));
        const float ms = time_ms(e0, e1);
        if (pass == 0) continue;
        const double inter = (double)reps * kListCap * blocks * kWavesPerBlock * kWave;
        std::printf("force loop %s, %d waves per SIMD: %.3f ms, %.3e interactions/s, %.1f TFLOP/s\n",
                    STAGED ? "staged" : STEP == 4 ? "entry by entry (rounds of 4)" : "entry by entry",
                    waves_per_simd, ms, inter / (ms * 1e-3), 20.0 * inter / (ms * 1e-3) / 1e12);
    }
}

}  // namespace

int main(int argc, char** argv) {
    const int reps = argc > 1 ? std::atoi(argv[1]) : 400;
    if (reps < 1) {
        std::fprintf(stderr, "loop_probe: reps must be positive\n");
        return 2;
    }
    hipDeviceProp_t prop;
    PROBE_CHECK(hipGetDeviceProperties(&prop, 0));
    const int cus = prop.multiProcessorCount;
    std::printf("device %s, %d compute units\n", prop.gcnArchName, cus);

    // the list: 256 entries at distinct offsets, equal small masses
    std::vector<float4> h(kListCap);
    for (int j = 0; j < kListCap; ++j)
        h[j] = make_float4(0.5f + 0.01f * j, -0.3f + 0.002f * j, 0.2f - 0.001f * j, 1e-3f);
    float4* list = nullptr;
    PROBE_CHECK(hipMalloc(&list, sizeof(float4) * kListCap));
    PROBE_CHECK(hipMemcpy(list, h.data(), sizeof(float4) * kListCap, hipMemcpyHostToDevice));
    // outputs: one float per thread of the largest grid (FMA: 16 blocks of 256 per CU)
    const size_t nout = (size_t)cus * 16 * 256;
    float* out = nullptr;
    PROBE_CHECK(hipMalloc(&out, sizeof(float) * nout));
    hipEvent_t e0, e1;
    PROBE_CHECK(hipEventCreate(&e0));
    PROBE_CHECK(hipEventCreate(&e1));

    for (int pass = 0; pass < 3; ++pass) {
        const int iters = 20000, blocks = cus * 16;
        PROBE_CHECK(hipEventRecord(e0, 0));
        hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(256), 0, 0, iters, 0.999f, 1e-3f, out);
        PROBE_CHECK(hipGetLastError());
        PROBE_CHECK(hipEventRecord(e1, 0));
        const float ms = time_ms(e0, e1);
        if (pass == 0) continue;
        const double flops = 2.0 * 8 * iters * (double)blocks * 256;
        std::printf("FP32 FMA chains: %.3f ms, %.1f TFLOP/s\n", ms, flops / (ms * 1e-3) / 1e12);
    }
    for (int w : {5, 8}) {
        probe_loop<false>(cus, w, reps, list, out, e0, e1);
        probe_loop<false, 4>(cus, w, reps, list, out, e0, e1);
        probe_loop<true>(cus, w, reps, list, out, e0, e1);
    }
    std::vector<float> back(nout);
    PROBE_CHECK(hipMemcpy(back.data(), out, sizeof(float) * nout, hipMemcpyDeviceToHost));
    double cs = 0.0;
    for (float v : back) cs += v;
    std::printf("checksum %.6e\n", cs);
    PROBE_CHECK(hipFree(list));
    PROBE_CHECK(hipFree(out));
    return 0;
}
