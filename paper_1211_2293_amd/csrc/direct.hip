// FP64 direct sum for a sample of target bodies: the exact softened
// Newtonian sum over every other body (the force law of §3.1 without the
// tree), the yardstick against which treecode force errors are stated.
//
// A block takes kDirTargets targets; its threads stride over the sorted
// bodies, each body read once per block and applied to every target held
// in registers.  Per-thread partial sums are folded by a fixed xor pattern
// within each wave and then wave by wave in order, so the result does not
// depend on scheduling.
#include "tc_internal.h"

#include <math.h>

namespace tc {
namespace {

constexpr int kDirTargets = 8;
constexpr int kDirThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__global__ void __launch_bounds__(kDirThreads) k_direct64(const Body* __restrict__ bodies,
                                                          const uint32_t* __restrict__ inv_perm, int64_t n,
                                                          const int32_t* __restrict__ targets, int nt, double eps2,
                                                          double G, DevParams* __restrict__ prm,
                                                          double* __restrict__ acc, double* __restrict__ pot) {
    __shared__ double s_part[kDirThreads / kWave][kDirTargets][4];
    __shared__ int s_ok[kDirTargets];
    const int t0 = blockIdx.x * kDirTargets;
    double tx[kDirTargets], ty[kDirTargets], tz[kDirTargets];
    int64_t tp[kDirTargets];
#pragma unroll
    for (int k = 0; k < kDirTargets; ++k) {
        const int t = t0 + k;
        const int64_t o = t < nt ? (int64_t)targets[t] : -1;
        const bool ok = o >= 0 && o < n;
        if (t < nt && !ok && threadIdx.x == 0) atomicOr(&prm->status, kFlagBadIndex);
        tp[k] = ok ? (int64_t)inv_perm[o] : -1;
        if (threadIdx.x == 0) s_ok[k] = ok;
        const Body b = bodies[ok ? tp[k] : 0];
        tx[k] = b.x;
        ty[k] = b.y;
        tz[k] = b.z;
    }
    double ax[kDirTargets], ay[kDirTargets], az[kDirTargets], ph[kDirTargets];
#pragma unroll
    for (int k = 0; k < kDirTargets; ++k) ax[k] = ay[k] = az[k] = ph[k] = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += kDirThreads) {
        const Body q = bodies[j];
#pragma unroll
        for (int k = 0; k < kDirTargets; ++k) {
            const double dx = q.x - tx[k], dy = q.y - ty[k], dz = q.z - tz[k];
            const double r2 = ((dx * dx + dy * dy) + dz * dz) + eps2;
            const double inv = j == tp[k] ? 0.0 : 1.0 / sqrt(r2);
            const double mi = q.m * inv;
            const double w3 = mi * inv * inv;
            ax[k] += w3 * dx;
            ay[k] += w3 * dy;
            az[k] += w3 * dz;
            ph[k] += mi;
        }
    }
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
#pragma unroll
    for (int k = 0; k < kDirTargets; ++k) {
        const double sx = wave_sum(ax[k]), sy = wave_sum(ay[k]), sz = wave_sum(az[k]), sp = wave_sum(ph[k]);
        if (lane == 0) {
            s_part[wv][k][0] = sx;
            s_part[wv][k][1] = sy;
            s_part[wv][k][2] = sz;
            s_part[wv][k][3] = sp;
        }
    }
    __syncthreads();
    if (threadIdx.x < kDirTargets * 4) {
        const int k = threadIdx.x / 4, c = threadIdx.x % 4;
        const int t = t0 + k;
        double s = 0.0;
        for (int w = 0; w < kDirThreads / kWave; ++w) s += s_part[w][k][c];
        if (t < nt) {
            if (!s_ok[k]) s = NAN;
            if (c < 3) {
                if (acc) acc[(int64_t)t * 3 + c] = G * s;
            } else if (pot) {
                pot[t] = -G * s;
            }
        }
    }
}

}  // namespace

hipError_t launch_direct64(const Body* bodies, const uint32_t* inv_perm, int64_t n, const int32_t* targets, int nt,
                           double eps2, double G, DevParams* prm, double* acc, double* pot, hipStream_t s) {
    const unsigned nb = (unsigned)((nt + kDirTargets - 1) / kDirTargets);
    hipLaunchKernelGGL(k_direct64, dim3(nb), dim3(kDirThreads), 0, s, bodies, inv_perm, n, targets, nt, eps2, G,
                       prm, acc, pot);
    return hipGetLastError();
}

}  // namespace tc
