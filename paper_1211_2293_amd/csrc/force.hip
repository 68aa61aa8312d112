// Fused tree walk and force summation (§3.1: a cell goes on a body's
// interaction list when it is distant enough, otherwise the walk descends
// into its children; the list is then summed to give the force; §3.2: the
// per-body sums are independent of each other).
//
// One wavefront per group of 64 consecutive bodies in key order, one lane
// per body.  The walk is stackless: cells are in depth-first pre-order, so
// the traversal state is a single cursor that only moves forward (to c+1
// when a cell is opened, to skip[c] when it is accepted or is a leaf).  Each
// step the wave evaluates the opening test for the 64 cells
// [cursor, cursor+64) at once, one per lane, in FP64; the visited chain
// inside that window is then followed with scalar bit operations (only the
// terminal cells, accepted or leaf, need a jump), and their entries are
// appended to a per-wave list in LDS.  When the list is full it is flushed:
// every lane sums the whole list for its own body in FP32, reading each entry
// as an LDS broadcast.  Coordinates are relative to the group's box centre
// (computed in FP64, then rounded) so FP32 keeps the digits that matter.
// Chunks of 64 entries are summed plainly and folded into Neumaier-
// compensated totals.
#include "tc_internal.h"

#include <math.h>

namespace tc {
namespace {

constexpr int kCap = 512;        // LDS list entries per wave (8 KiB)
constexpr int kWavesPerBlock = 4;

__device__ __forceinline__ void lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

__device__ __forceinline__ int wave_incl_scan(int x) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    return x;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// Neumaier compensated accumulation of x into (s, c).
__device__ __forceinline__ void comp_add(float& s, float& c, float x) {
    const float t = s + x;
    if (fabsf(s) >= fabsf(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
}

struct Acc {
    float sx, sy, sz, sp, cx, cy, cz, cp;
};

// Sum `cnt` list entries (padded to a multiple of 8 with massless entries)
// for this lane's body.
template <int D>
__device__ __forceinline__ void flush(const float4* L, int cnt, float xi, float yi, float zi,
                                      float eps2, Acc& a) {
    for (int e = 0; e < cnt; e += kWave) {
        const int lim = min(kWave, cnt - e);
        float ax = 0.f, ay = 0.f, az = 0.f, ap = 0.f;
        for (int k = 0; k < lim; k += 8) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const float4 p = L[e + k + u];
                const float dx = p.x - xi, dy = p.y - yi;
                float r2;
                float dz = 0.f;
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
        comp_add(a.sx, a.cx, ax);
        comp_add(a.sy, a.cy, ay);
        if (D == 3) comp_add(a.sz, a.cz, az);
        comp_add(a.sp, a.cp, ap);
    }
}

template <int D>
__device__ __forceinline__ void pad_and_flush(float4* L, int cnt, float xi, float yi, float zi,
                                              float eps2, Acc& a) {
    const int lane = threadIdx.x & (kWave - 1);
    const int padded = (cnt + 7) & ~7;
    for (int j = cnt + lane; j < padded; j += kWave) L[j] = make_float4(0.f, 0.f, 0.f, 0.f);
    lds_fence();
    flush<D>(L, padded, xi, yi, zi, eps2, a);
    lds_fence();
}

__device__ __forceinline__ float4 rel_entry(const Body& b, double rx, double ry, double rz) {
    return make_float4((float)(b.x - rx), (float)(b.y - ry), (float)(b.z - rz), (float)b.m);
}

template <int D>
__global__ void __launch_bounds__(256) k_walk_force(const WalkCell* __restrict__ walk,
                                                    const Body* __restrict__ bodies,
                                                    const uint32_t* __restrict__ perm, int64_t n,
                                                    int64_t ngroups, float G, float eps2,
                                                    const DevParams* __restrict__ prm,
                                                    float* __restrict__ acc, float* __restrict__ pot,
                                                    int64_t* __restrict__ m2p_out,
                                                    int64_t* __restrict__ p2p_out) {
    __shared__ float4 s_list[kWavesPerBlock][kCap];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);

    // XCD-aware order: hardware deals blocks round-robin over the 8 XCDs; give
    // each XCD a contiguous range of groups so neighbouring groups, which walk
    // nearly the same cells, share one L2.
    const unsigned B = gridDim.x, b = blockIdx.x;
    const unsigned q = B / 8, r = B % 8, x = b % 8;
    const unsigned lb = x * q + (x < r ? x : r) + b / 8;
    const int64_t g = (int64_t)lb * kWavesPerBlock + wv;
    if (g >= ngroups) return;

    const int64_t i0 = g * kGroup;
    const int64_t i = i0 + lane;
    const bool valid = i < n;
    const Body me = bodies[valid ? i : i0];

    // group bounding box (exact) and its centre, the group's FP32 origin
    const double lox = wave_min(me.x), hix = wave_max(me.x);
    const double loy = wave_min(me.y), hiy = wave_max(me.y);
    const double loz = D == 3 ? wave_min(me.z) : 0.0, hiz = D == 3 ? wave_max(me.z) : 0.0;
    const double rx = (lox + hix) * 0.5, ry = (loy + hiy) * 0.5, rz = (loz + hiz) * 0.5;
    const float xi = (float)(me.x - rx), yi = (float)(me.y - ry), zi = (float)(me.z - rz);

    float4* L = s_list[wv];
    Acc a = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int len = 0;
    int64_t nm2p = 0, np2p = 0;
    const uint32_t C = prm->ncells;
    uint32_t cursor = 0;

    while (cursor < C) {
        const uint32_t c = cursor + lane;
        const bool vc = c < C;
        WalkCell wc;
        if (vc) {
            wc = walk[c];
        } else {
            wc.cx = wc.cy = wc.cz = 0.0;
            wc.rcrit2 = INFINITY;
            wc.m = 0.f;
            wc.skip = (int32_t)C;
            wc.begin = 0;
            wc.cnt_leaf = 0;
        }
        // opening test: squared distance from the centre of mass to the box
        const double dxm = fmax(fmax(lox - wc.cx, 0.0), wc.cx - hix);
        const double dym = fmax(fmax(loy - wc.cy, 0.0), wc.cy - hiy);
        double d2 = dxm * dxm + dym * dym;
        if (D == 3) {
            const double dzm = fmax(fmax(loz - wc.cz, 0.0), wc.cz - hiz);
            d2 = d2 + dzm * dzm;
        }
        const bool accept = vc && d2 > wc.rcrit2;
        const bool leaf = vc && wc.cnt_leaf < 0;
        const bool opened = vc && !accept && !leaf;
        const uint64_t O = __ballot(opened);
        const uint64_t V = __ballot(vc);

        // follow the visited chain inside the window
        uint64_t T = 0;
        int v = 0;
        uint32_t next;
        while (true) {
            if (v >= kWave || !((V >> v) & 1ull)) {
                next = cursor + (uint32_t)v;
                break;
            }
            const uint64_t rest = ~O & V & (~0ull << v);
            if (rest == 0) {
                next = cursor + (uint32_t)__popcll(V);
                break;
            }
            const int t = __builtin_ctzll(rest);
            T |= 1ull << t;
            v = __builtin_amdgcn_readlane(wc.skip, t) - (int)cursor;
        }

        bool term = (T >> lane) & 1ull;
        const int cnt = wc.cnt_leaf & 0x7fffffff;
        int ne = term ? (accept ? 1 : cnt) : 0;
        int incl = wave_incl_scan(ne);
        int total = __builtin_amdgcn_readlane(incl, kWave - 1);
        if (len + total > kCap) {
            pad_and_flush<D>(L, len, xi, yi, zi, eps2, a);
            len = 0;
            if (total > kCap) {
                const uint64_t keep = __ballot(term && incl <= kCap);
                const int t0 = __builtin_ctzll(T & ~keep);
                if (keep == 0) {
                    // the first terminal is a leaf too large for the list
                    // (only bodies with identical keys): stream it through
                    const int bcount = __builtin_amdgcn_readlane(cnt, t0);
                    const int bbeg = __builtin_amdgcn_readlane(wc.begin, t0);
                    for (int off = 0; off < bcount; off += kCap) {
                        const int m = min(kCap, bcount - off);
                        for (int j = lane; j < m; j += kWave) L[j] = rel_entry(bodies[bbeg + off + j], rx, ry, rz);
                        pad_and_flush<D>(L, m, xi, yi, zi, eps2, a);
                    }
                    np2p += bcount;
                    cursor = (uint32_t)__builtin_amdgcn_readlane(wc.skip, t0);
                    continue;
                }
                T = keep;
                term = (T >> lane) & 1ull;
                total = __builtin_amdgcn_readlane(incl, 63 - __builtin_clzll(keep));
                next = cursor + (uint32_t)t0;
            }
        }
        if (term) {
            const int off = len + incl - ne;
            if (accept) {
                L[off] = make_float4((float)(wc.cx - rx), (float)(wc.cy - ry), (float)(wc.cz - rz), wc.m);
            } else {
                for (int j = 0; j < ne; ++j) L[off + j] = rel_entry(bodies[wc.begin + j], rx, ry, rz);
            }
        }
        const int nacc = __popcll(__ballot(term && accept));
        nm2p += nacc;
        np2p += total - nacc;
        len += total;
        cursor = next;
    }
    pad_and_flush<D>(L, len, xi, yi, zi, eps2, a);

    if (valid) {
        // the body met itself once as a direct entry: no force (zero
        // displacement) but a -m/eps potential term, removed here exactly as
        // it was formed
        const float mself = (float)me.m;
        const float sself = __builtin_amdgcn_rsqf(eps2);
        const float ph = (a.sp + a.cp) + mself * sself;
        const int64_t o = perm[i];
        acc[o * D + 0] = G * (a.sx + a.cx);
        acc[o * D + 1] = G * (a.sy + a.cy);
        if (D == 3) acc[o * D + 2] = G * (a.sz + a.cz);
        pot[o] = G * ph;
    }
    if (lane == 0) {
        m2p_out[g] = nm2p;
        p2p_out[g] = np2p;
    }
}

}  // namespace

hipError_t launch_walk_force(const WalkCell* walk, const Body* bodies, const uint32_t* perm,
                             int64_t n, int dim, float G, float eps2, const DevParams* prm,
                             float* acc, float* pot, int64_t* m2p, int64_t* p2p, hipStream_t s) {
    const int64_t ngroups = (n + kGroup - 1) / kGroup;
    const unsigned nb = (unsigned)((ngroups + kWavesPerBlock - 1) / kWavesPerBlock);
    if (dim == 3)
        hipLaunchKernelGGL(k_walk_force<3>, dim3(nb), dim3(256), 0, s, walk, bodies, perm, n, ngroups, G, eps2,
                           prm, acc, pot, m2p, p2p);
    else
        hipLaunchKernelGGL(k_walk_force<2>, dim3(nb), dim3(256), 0, s, walk, bodies, perm, n, ngroups, G, eps2,
                           prm, acc, pot, m2p, p2p);
    return hipGetLastError();
}

}  // namespace tc
