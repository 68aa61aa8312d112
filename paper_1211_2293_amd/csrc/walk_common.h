// Device helpers shared by the walk kernels (plain and learned).
// Internal to libtc.
#pragma once

#include "tc_internal.h"

#include <math.h>

namespace tc {
namespace walk {

constexpr int kListCap = 256;     // LDS list entries per wave (16 B each)
constexpr int kStackCap = 320;    // LDS range-stack entries per wave (4 B each)
constexpr int kQuadCap = 64;      // LDS quadrupole-list entries per wave (48 B each)

// Order LDS accesses of the lanes of one wave (a wave's LDS operations are
// performed in program order; this keeps the compiler from reordering them).
static __device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

static __device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
    return v;
}

static __device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// A value equal in every lane, made visibly uniform (scalar registers).
static __device__ __forceinline__ double uniform(double v) {
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

// Neumaier compensated accumulation of x into (s, c).
static __device__ __forceinline__ void comp_add(float& s, float& c, float x) {
    const float t = s + x;
    if (fabsf(s) >= fabsf(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
}

struct Acc {
    float sx, sy, sz, sp, cx, cy, cz, cp;
};

// Sum the first `cnt` list entries for this lane's body.  cnt is padded up
// to a multiple of 8 with massless entries, which add exactly zero.  By
// default each chunk of 64 entries is summed plainly and folded into the
// Neumaier-compensated totals; with PLAIN the whole list is one running
// FP32 sum (the uncompensated reference of the precision study).
//
// STAGED takes each half of a batch of 8 entries in three stages
// (distances, reciprocal square roots, sums): the same operations in the
// same order, so the same bits, but the four v_rsq issue back to back and
// their latencies overlap instead of each stalling the wave in turn.
// Measured with loop_probe (this loop alone over a list in LDS): 2.9e12
// interactions/s entry by entry and 3.0e12 staged at 5 waves per SIMD,
// 3.15e12 either way at 8.  In the walk kernels it pays in the shared walks
// (8% at 50,000 bodies); with one wave per group the compiler then issues
// four list reads at a time instead of eight, and that kernel ran as fast at
// 1M bodies and 1.8% slower at 4M.
template <int D, bool PLAIN = false, bool STAGED = false, int STEP = 8>
static __device__ __forceinline__ void flush(float4* L, int cnt, float xi, float yi, float zi, float eps2, Acc& a) {
    // entries per unrolled round: the staged form takes batches of 8; the
    // order of the sums is the same for any STEP
    constexpr int kStep = STAGED ? 8 : STEP;
    static_assert(8 % kStep == 0, "rounds of 1, 2, 4 or 8 entries");
    const int lane = threadIdx.x & (kWave - 1);
    // zero entries pad the list to whole rounds (they add exact zeros)
    const int padded = (cnt + kStep - 1) & ~(kStep - 1);
    for (int j = cnt + lane; j < padded; j += kWave) L[j] = make_float4(0.f, 0.f, 0.f, 0.f);
    wave_lds_sync();
    for (int e = 0; e < padded; e += kWave) {
        const int lim = min(kWave, padded - e);
        float ax = 0.f, ay = 0.f, az = 0.f, ap = 0.f;
        if (PLAIN) {
            ax = a.sx;
            ay = a.sy;
            az = a.sz;
            ap = a.sp;
        }
        for (int k = 0; k < lim; k += kStep) {
            if (STAGED) {
#pragma unroll
                for (int h4 = 0; h4 < 8; h4 += 4) {
                    float dx[4], dy[4], dz[4], m[4], s[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const float4 p = L[e + k + h4 + u];
                        dx[u] = p.x - xi;
                        dy[u] = p.y - yi;
                        m[u] = p.w;
                        if (D == 3) {
                            dz[u] = p.z - zi;
                            s[u] = fmaf(dx[u], dx[u], fmaf(dy[u], dy[u], fmaf(dz[u], dz[u], eps2)));
                        } else {
                            dz[u] = 0.f;
                            s[u] = fmaf(dx[u], dx[u], fmaf(dy[u], dy[u], eps2));
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) s[u] = __builtin_amdgcn_rsqf(s[u]);
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const float ms = m[u] * s[u];
                        const float s2 = s[u] * s[u];
                        const float ms3 = ms * s2;
                        ap -= ms;
                        ax = fmaf(ms3, dx[u], ax);
                        ay = fmaf(ms3, dy[u], ay);
                        if (D == 3) az = fmaf(ms3, dz[u], az);
                    }
                }
                continue;
            }
#pragma unroll
            for (int u = 0; u < kStep; ++u) {
                const float4 p = L[e + k + u];
                const float dx = p.x - xi, dy = p.y - yi;
                float r2, dz = 0.f;
                if (D == 3) {
                    dz = p.z - zi;
                    r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
                } else {
                    r2 = fmaf(dx, dx, fmaf(dy, dy, eps2));
                }
                const float s = __builtin_amdgcn_rsqf(r2);
                const float ms = p.w * s;
                const float s2 = s * s;
                const float ms3 = ms * s2;
                ap -= ms;
                ax = fmaf(ms3, dx, ax);
                ay = fmaf(ms3, dy, ay);
                if (D == 3) az = fmaf(ms3, dz, az);
            }
        }
        if (PLAIN) {
            a.sx = ax;
            a.sy = ay;
            a.sz = az;
            a.sp = ap;
        } else {
            comp_add(a.sx, a.cx, ax);
            comp_add(a.sy, a.cy, ay);
            if (D == 3) comp_add(a.sz, a.cz, az);
            comp_add(a.sp, a.cp, ap);
        }
    }
    wave_lds_sync();
}

// Sum the first `cnt` entries of a quadrupole list (3 float4 per entry:
// offset and mass, (Qxx, Qyy, Qzz, Qxy), (Qxz, Qyz, 0, 0)) for this lane's
// body: the monopole term plus, with d the entry's offset from the body and
// s = (|d|^2 + eps^2)^{-1/2}, a += -Q d s^5 + (5/2) (d.Q d) d s^7 and
// phi -= (1/2) (d.Q d) s^5.  Padded to a multiple of 8 with zero entries.
template <bool PLAIN = false>
static __device__ __forceinline__ void flush_quad(float4* LQ, int cnt, float xi, float yi, float zi, float eps2,
                                                  Acc& a) {
    const int lane = threadIdx.x & (kWave - 1);
    const int padded = (cnt + 7) & ~7;
    for (int j = cnt + lane; j < padded; j += kWave) {
        LQ[3 * j] = make_float4(0.f, 0.f, 0.f, 0.f);
        LQ[3 * j + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
        LQ[3 * j + 2] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    wave_lds_sync();
    for (int e = 0; e < padded; e += kWave) {
        const int lim = min(kWave, padded - e);
        float ax = 0.f, ay = 0.f, az = 0.f, ap = 0.f;
        if (PLAIN) {
            ax = a.sx;
            ay = a.sy;
            az = a.sz;
            ap = a.sp;
        }
        for (int k = 0; k < lim; k += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float4 p = LQ[3 * (e + k + u)];
                const float4 qa = LQ[3 * (e + k + u) + 1];
                const float4 qb = LQ[3 * (e + k + u) + 2];
                const float dx = p.x - xi, dy = p.y - yi, dz = p.z - zi;
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
                const float s = __builtin_amdgcn_rsqf(r2);
                const float s2 = s * s;
                const float ms = p.w * s;
                const float ms3 = ms * s2;
                const float qx = fmaf(qa.x, dx, fmaf(qa.w, dy, qb.x * dz));
                const float qy = fmaf(qa.w, dx, fmaf(qa.y, dy, qb.y * dz));
                const float qz = fmaf(qb.x, dx, fmaf(qb.y, dy, qa.z * dz));
                const float dqd = fmaf(dx, qx, fmaf(dy, qy, dz * qz));
                const float s5 = (s2 * s2) * s;
                const float c = fmaf(2.5f * dqd, s5 * s2, ms3);
                ap -= fmaf(0.5f * dqd, s5, ms);
                ax = fmaf(-qx, s5, fmaf(c, dx, ax));
                ay = fmaf(-qy, s5, fmaf(c, dy, ay));
                az = fmaf(-qz, s5, fmaf(c, dz, az));
            }
        }
        if (PLAIN) {
            a.sx = ax;
            a.sy = ay;
            a.sz = az;
            a.sp = ap;
        } else {
            comp_add(a.sx, a.cx, ax);
            comp_add(a.sy, a.cy, ay);
            comp_add(a.sz, a.cz, az);
            comp_add(a.sp, a.cp, ap);
        }
    }
    wave_lds_sync();
}

// List entry of a body relative to the group origin.  FP32 inputs keep a
// 16-byte FP32 copy of the sorted bodies (exact: it is the input itself);
// the FP64 difference is the same either way.
static __device__ __forceinline__ float4 body_entry(const Body* __restrict__ bodies, const float4* __restrict__ bodies32,
                                             int64_t j, double rx, double ry, double rz) {
    if (bodies32) {
        const float4 b = bodies32[j];
        return make_float4((float)((double)b.x - rx), (float)((double)b.y - ry), (float)((double)b.z - rz), b.w);
    }
    const Body b = bodies[j];
    return make_float4((float)(b.x - rx), (float)(b.y - ry), (float)(b.z - rz), (float)b.m);
}

static __device__ __forceinline__ WalkCell load_cell(const WalkCell* __restrict__ walk, uint32_t c, bool v) {
    WalkCell wc;
    if (v) {
        wc = walk[c];
    } else {
        wc.cx = wc.cy = wc.cz = 0.0;
        wc.rcrit2 = INFINITY;
        wc.m = 0.f;
        wc.a = 0;
        wc.b = 0;
        wc.pad = 0;
    }
    return wc;
}

// Scheduling of the persistent walk kernels over NG groups.  The groups are
// cut into one contiguous share per XCD (blocks are dealt round-robin over
// the XCDs, so block b runs on XCD b mod 8): neighbouring groups walk nearly
// the same cells and then share one L2.  The waves resident on XCD x take
// the first groups of share x without any atomic, one each by their rank
// among those waves; counter x hands out the rest of share x.  A wave works
// through its own share, then helps the others.  Each pop reads the counter
// first and skips a share found drained (counters only grow, so a stale
// read costs at most one extra pop), and a share no larger than its static
// part never touches its counter: returning atomics on one address from
// thousands of waves serialise, and the memory accesses queued behind them
// stall the walks.
struct GroupSched {
    uint32_t* queue;
    uint32_t ng;       // groups
    uint32_t rank;     // this wave's rank among the waves of its XCD
    int home;          // this wave's XCD
    int wpb;           // waves per block

    __device__ uint32_t share_lo(int x) const { return (uint32_t)(((uint64_t)ng * x) / kXcd); }
    // first group of share x handed out by its counter
    __device__ uint32_t dyn_lo(int x) const {
        const uint32_t blocks = (gridDim.x - (uint32_t)x + kXcd - 1) / kXcd;
        return share_lo(x) + blocks * (uint32_t)wpb;
    }
    // the next group of share x from its counter, or share_lo(x + 1) once it is drained
    __device__ uint32_t pop(int x) const {
        const uint32_t lo = dyn_lo(x), hi = share_lo(x + 1);
        if (lo >= hi) return hi;
        uint32_t* q = queue + x * kQueueStride;
        const uint32_t seen = (uint32_t)__builtin_amdgcn_readfirstlane(
            (int)__hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (seen >= hi - lo) return hi;
        // every lane takes part (lane 0 adds 1, the others 0), so the loop
        // stays uniform; lane 0's result is the counter before its own
        // increment whatever order the lanes are served in
        const int lane = threadIdx.x & (kWave - 1);
        const uint32_t k = (uint32_t)__builtin_amdgcn_readfirstlane((int)atomicAdd(q, lane == 0 ? 1u : 0u));
        return k >= hi - lo ? hi : lo + k;
    }
    // the first group a wave takes in share x (hop 0 is its own share)
    __device__ uint32_t first(int x, int hop) const {
        if (hop == 0 && share_lo(x) + rank < share_lo(x + 1)) return share_lo(x) + rank;
        return pop(x);
    }
};

// Requires gridDim.x >= kXcd, so every share has waves of its own XCD.
static __device__ __forceinline__ GroupSched make_sched(uint32_t* queue, uint32_t ng, int wpb) {
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    return GroupSched{queue, ng, (blockIdx.x / kXcd) * (uint32_t)wpb + (uint32_t)wv, (int)(blockIdx.x % kXcd), wpb};
}

// Zero the kXcd counters (one block of 64 threads).
static __device__ __forceinline__ void reset_sched(uint32_t* queue) {
    if (threadIdx.x < kXcd) queue[threadIdx.x * kQueueStride] = 0u;
}

}  // namespace walk
}  // namespace tc
