// The treecode with per-body interaction lists (§3.1 as the paper states it:
// every body builds its own list of distant-enough cells and nearby bodies,
// and the list is then summed; §3.2 ships such lists to the servers).
//
// Three passes over the bodies in key order, one wavefront per body:
//   count: the body walks alone (its box is the point itself) at the opening
//          radii of tc_walk and counts its list entries;
//   (an exclusive 64-bit scan of the counts gives each list's offset)
//   write: the same walk writes the entries to the caller's list buffer:
//          a cell as its level-order index, a body as 0x80000000 | index;
//   sum:   the wave's lanes take the list 64 entries at a time, form each
//          entry's offset from the body in FP64, round it to FP32 and apply
//          the softened force law in FP32; lane sums are folded chunk by
//          chunk (Neumaier) and reduced across the wave in FP64 in a fixed
//          order.
// The walk is the batched level-order walk of the group kernel: an LDS stack
// of sibling ranges, up to 64 cells tested per round in FP64.
#include "tc_internal.h"

#include <math.h>

namespace tc {
namespace {

constexpr int kPbStack = 320;
constexpr int kPbWaves = 4;
constexpr uint32_t kBodyTag = 0x80000000u;

__device__ __forceinline__ void pb_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o, kWave);
    return v;
}

// Exclusive prefix sum of v over the wave's lanes.
__device__ __forceinline__ uint32_t wave_exscan_u32(uint32_t v) {
    const int lane = threadIdx.x & (kWave - 1);
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, o, kWave);
        if (lane >= o) x += y;
    }
    return x - v;
}

// One body's walk.  on_round(accept, direct, b, wc) runs with the whole
// wave once per round: lane j tested cell b (level-order index) with record
// wc; accept / direct say whether it is a list entry as a cell or gives its
// bodies.
template <int D, typename F>
__device__ void walk_body(const WalkCell* __restrict__ walk, uint32_t* S, double px, double py, double pz,
                          F&& on_round) {
    constexpr int R = D == 3 ? 8 : 4, RP = kWave / R;
    constexpr int kReserve = (R - 1) * (D == 3 ? 21 : 31) + R;
    static_assert(kPbStack >= kWave + kReserve + kWave, "stack bound");
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    if (lane == 0) S[0] = 0u;
    pb_sync();
    int top = 1;
    while (top > 0) {
        const int nr = (top + kWave + kReserve <= kPbStack) ? min(top, RP) : 1;
        const int rr = lane / R, j = lane % R;
        uint32_t packed = 0;
        if (rr < nr) packed = S[top - 1 - rr];
        top -= nr;
        const int rlen = (int)(packed & 7u) + 1;
        const bool vc = rr < nr && j < rlen;
        const uint32_t b = (packed >> 3) + (uint32_t)j;
        pb_sync();
        WalkCell wc;
        if (vc) {
            wc = walk[b];
        } else {
            wc.cx = wc.cy = wc.cz = 0.0;
            wc.rcrit2 = INFINITY;
            wc.m = 0.f;
            wc.a = 0;
            wc.b = 0;
            wc.pad = 0;
        }
        const double dx = wc.cx - px, dy = wc.cy - py;
        double d2 = dx * dx + dy * dy;
        if (D == 3) {
            const double dz = wc.cz - pz;
            d2 = d2 + dz * dz;
        }
        const bool leaf = vc && wc.b < 0;
        const bool accept = vc && d2 > wc.rcrit2;
        const bool opened = vc && !accept && !leaf;
        const bool direct = leaf && !accept;
        const uint64_t O = __ballot(opened);
        if (opened) S[top + __popcll(O & below)] = ((uint32_t)wc.a << 3) | (uint32_t)(wc.b - 1);
        top += __popcll(O);
        pb_sync();
        on_round(accept, direct, b, wc);
    }
}

template <int D, bool WRITE>
__global__ void __launch_bounds__(kWave * kPbWaves) k_pb_walk(const WalkCell* __restrict__ walk,
                                                               const Body* __restrict__ bodies, int64_t n,
                                                               uint32_t* __restrict__ counts,
                                                               const uint64_t* __restrict__ offs,
                                                               uint32_t* __restrict__ lists, int64_t cap) {
    __shared__ uint32_t s_stack[kPbWaves][kPbStack];
    const int wv = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    const int64_t i = (int64_t)blockIdx.x * kPbWaves + wv;
    if (i >= n) return;
    const Body me = bodies[i];
    uint64_t k = WRITE ? offs[i] : 0;
    const uint64_t end = WRITE ? offs[i + 1] : 0;
    walk_body<D>(walk, s_stack[wv], me.x, me.y, D == 3 ? me.z : 0.0,
                 [&](bool accept, bool direct, uint32_t b, const WalkCell& wc) {
                     const uint32_t cnt = accept ? 1u : direct ? (uint32_t)(wc.b & 0x7fffffff) : 0u;
                     if (WRITE) {
                         const uint64_t at = k + wave_exscan_u32(cnt);
                         if (accept) {
                             if (at < end && at < (uint64_t)cap) lists[at] = b;
                         } else if (direct) {
                             for (uint32_t q = 0; q < cnt; ++q)
                                 if (at + q < end && at + q < (uint64_t)cap)
                                     lists[at + q] = kBodyTag | (uint32_t)(wc.a + (int)q);
                         }
                     }
                     k += wave_sum_u32(cnt);
                 });
    if (!WRITE && lane == 0) counts[i] = (uint32_t)k;
}

// Exclusive scan of u32 counts into u64 offsets (offs[n] = total): per-tile
// sums, one block scanning the tile sums, then each tile applied.
constexpr int kPbScanTile = 4096;

__global__ void __launch_bounds__(256) k_pb_tile_sum(const uint32_t* __restrict__ c, int64_t n,
                                                     uint64_t* __restrict__ part) {
    __shared__ uint64_t s[256];
    const int64_t base = (int64_t)blockIdx.x * kPbScanTile;
    uint64_t v = 0;
    for (int j = threadIdx.x; j < kPbScanTile; j += 256) {
        const int64_t i = base + j;
        if (i < n) v += c[i];
    }
    s[threadIdx.x] = v;
    __syncthreads();
    for (unsigned o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void __launch_bounds__(256) k_pb_part_scan(uint64_t* __restrict__ part, int64_t tiles) {
    __shared__ uint64_t carry;
    __shared__ uint64_t s[256];
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t t0 = 0; t0 < tiles; t0 += 256) {
        const int64_t t = t0 + threadIdx.x;
        const uint64_t v = t < tiles ? part[t] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (unsigned o = 1; o < 256; o <<= 1) {     // inclusive Hillis-Steele scan
            const uint64_t y = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
            __syncthreads();
            s[threadIdx.x] += y;
            __syncthreads();
        }
        if (t < tiles) part[t] = carry + s[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 255) carry += s[255];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_pb_apply(const uint32_t* __restrict__ c, int64_t n,
                                                  const uint64_t* __restrict__ part, uint64_t* __restrict__ offs) {
    __shared__ uint64_t s[256];
    const int64_t base = (int64_t)blockIdx.x * kPbScanTile;
    constexpr int per = kPbScanTile / 256;             // consecutive items per thread
    uint64_t v[per];
    uint64_t mine = 0;
#pragma unroll
    for (int q = 0; q < per; ++q) {
        const int64_t i = base + threadIdx.x * per + q;
        v[q] = i < n ? c[i] : 0;
        mine += v[q];
    }
    s[threadIdx.x] = mine;
    __syncthreads();
    for (unsigned o = 1; o < 256; o <<= 1) {
        const uint64_t y = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += y;
        __syncthreads();
    }
    uint64_t run = part[blockIdx.x] + s[threadIdx.x] - mine;
#pragma unroll
    for (int q = 0; q < per; ++q) {
        const int64_t i = base + threadIdx.x * per + q;
        if (i < n) offs[i] = run;
        run += v[q];
        if (i == n - 1) offs[n] = run;
    }
}

__device__ __forceinline__ void pb_comp(float& s, float& c, float x) {
    const float t = s + x;
    if (fabsf(s) >= fabsf(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

template <int D>
__global__ void __launch_bounds__(kWave * kPbWaves) k_pb_sum(const WalkCell* __restrict__ walk,
                                                              const Body* __restrict__ bodies,
                                                              const uint32_t* __restrict__ perm, int64_t n,
                                                              const uint64_t* __restrict__ offs,
                                                              const uint32_t* __restrict__ lists, int64_t cap,
                                                              int64_t cbound, float G, float eps2,
                                                              float* __restrict__ acc, float* __restrict__ pot) {
    const int wv = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    const int64_t i = (int64_t)blockIdx.x * kPbWaves + wv;
    if (i >= n) return;
    const Body me = bodies[i];
    const uint64_t b0 = offs[i];
    uint64_t e0 = offs[i + 1];
    if (e0 > (uint64_t)cap) e0 = (uint64_t)cap;
    float sx = 0.f, sy = 0.f, sz = 0.f, sp = 0.f, cx = 0.f, cy = 0.f, cz = 0.f, cp = 0.f;
    for (uint64_t k0 = b0; k0 < e0; k0 += 64 * kWave) {
        float ax = 0.f, ay = 0.f, az = 0.f, ap = 0.f;
        for (uint64_t k = k0 + lane; k < e0 && k < k0 + 64 * kWave; k += kWave) {
            const uint32_t v = lists[k];
            double qx, qy, qz;
            float m;
            // entries come from the write pass; an index outside its array
            // (never written) is skipped rather than read
            if ((v & kBodyTag) ? (int64_t)(v & ~kBodyTag) >= n : (int64_t)v >= cbound) continue;
            if (v & kBodyTag) {
                const Body q = bodies[v & ~kBodyTag];
                qx = q.x;
                qy = q.y;
                qz = q.z;
                m = (float)q.m;
            } else {
                const WalkCell& c = walk[v];
                qx = c.cx;
                qy = c.cy;
                qz = c.cz;
                m = c.m;
            }
            const float dx = (float)(qx - me.x), dy = (float)(qy - me.y);
            const float dz = D == 3 ? (float)(qz - me.z) : 0.f;
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
            const float s = __builtin_amdgcn_rsqf(r2);
            const float ms = m * s;
            const float ms3 = ms * (s * s);
            ap -= ms;
            ax = fmaf(ms3, dx, ax);
            ay = fmaf(ms3, dy, ay);
            az = fmaf(ms3, dz, az);
        }
        pb_comp(sx, cx, ax);
        pb_comp(sy, cy, ay);
        pb_comp(sz, cz, az);
        pb_comp(sp, cp, ap);
    }
    const double tx = wave_sum_f64((double)sx + (double)cx);
    const double ty = wave_sum_f64((double)sy + (double)cy);
    const double tz = wave_sum_f64((double)sz + (double)cz);
    const double tp = wave_sum_f64((double)sp + (double)cp);
    if (lane == 0) {
        // the body's own entry gave no force and a -m/eps potential term
        const float mself = (float)me.m;
        const double ph = tp + (double)(mself * __builtin_amdgcn_rsqf(eps2));
        const int64_t o = perm[i];
        acc[o * D + 0] = (float)((double)G * tx);
        acc[o * D + 1] = (float)((double)G * ty);
        if (D == 3) acc[o * D + 2] = (float)((double)G * tz);
        pot[o] = (float)((double)G * ph);
    }
}

}  // namespace

hipError_t launch_pb_count(const WalkCell* walk, const Body* bodies, int64_t n, int dim, uint32_t* counts,
                           uint64_t* offs, uint64_t* part, hipStream_t s) {
    const unsigned nb = (unsigned)((n + kPbWaves - 1) / kPbWaves);
    if (dim == 3)
        hipLaunchKernelGGL((k_pb_walk<3, false>), dim3(nb), dim3(kWave * kPbWaves), 0, s, walk, bodies, n, counts,
                           (const uint64_t*)nullptr, (uint32_t*)nullptr, (int64_t)0);
    else
        hipLaunchKernelGGL((k_pb_walk<2, false>), dim3(nb), dim3(kWave * kPbWaves), 0, s, walk, bodies, n, counts,
                           (const uint64_t*)nullptr, (uint32_t*)nullptr, (int64_t)0);
    const int64_t tiles = (n + kPbScanTile - 1) / kPbScanTile;
    hipLaunchKernelGGL(k_pb_tile_sum, dim3((unsigned)tiles), dim3(256), 0, s, counts, n, part);
    hipLaunchKernelGGL(k_pb_part_scan, dim3(1), dim3(256), 0, s, part, tiles);
    hipLaunchKernelGGL(k_pb_apply, dim3((unsigned)tiles), dim3(256), 0, s, counts, n, part, offs);
    return hipGetLastError();
}

hipError_t launch_pb_write_sum(const WalkCell* walk, const Body* bodies, const uint32_t* perm, int64_t n, int dim,
                               const uint64_t* offs, uint32_t* lists, int64_t cap, int64_t cbound, float G,
                               float eps2, float* acc, float* pot, hipStream_t s) {
    const unsigned nb = (unsigned)((n + kPbWaves - 1) / kPbWaves);
    if (dim == 3) {
        hipLaunchKernelGGL((k_pb_walk<3, true>), dim3(nb), dim3(kWave * kPbWaves), 0, s, walk, bodies, n,
                           (uint32_t*)nullptr, offs, lists, cap);
        hipLaunchKernelGGL(k_pb_sum<3>, dim3(nb), dim3(kWave * kPbWaves), 0, s, walk, bodies, perm, n, offs, lists,
                           cap, cbound, G, eps2, acc, pot);
    } else {
        hipLaunchKernelGGL((k_pb_walk<2, true>), dim3(nb), dim3(kWave * kPbWaves), 0, s, walk, bodies, n,
                           (uint32_t*)nullptr, offs, lists, cap);
        hipLaunchKernelGGL(k_pb_sum<2>, dim3(nb), dim3(kWave * kPbWaves), 0, s, walk, bodies, perm, n, offs, lists,
                           cap, cbound, G, eps2, acc, pot);
    }
    return hipGetLastError();
}

}  // namespace tc
