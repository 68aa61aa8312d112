// Walk and force summation with the learned closure (3D).
//
// The walk of the plain kernel with two opening radii, theta_L (large, the
// learned walk) and theta_P (the plain walk it stands in for), and a mode
// per stacked range:
//   mode L: a cell accepted at both radii is a plain monopole entry; a cell
//           accepted at theta_L but opened at theta_P is a learned cell; a
//           cell opened at theta_L is opened (children stay in mode L);
//   mode P: the plain walk at theta_P (children stay in mode P).
// For a learned cell the network predicts the normalised residual for each
// of the group's bodies; if the largest predicted residual relative to the
// monopole, |yhat| s^2 / |x - C|^2, over the group exceeds tau the cell falls
// back to the plain walk of its subtree at theta_P (its
// children in mode P, or its bodies directly if it is a leaf), otherwise it
// enters as a monopole entry plus, per body, G M s^2 yhat / |x - C|^4 (the
// network predicts the residual in units of the quadrupole scale).  With
// tau = 0 every learned cell falls back and the walk is exactly the plain
// walk at theta_P; with tau = inf it is the plain walk at theta_L plus the
// corrections.  The potential keeps the monopoles.
//
// The network runs on 16x16x16 BF16 matrix-core tiles.  Each layer is
// computed transposed, Z^T = W^T H^T, so the FP32 output tile a lane holds
// (rows 4(l/16)+q, column l%16) is exactly the B operand of the next layer:
// activations never leave registers, and only the transposed BF16 weights
// (about 12 KiB per block) sit in LDS.
#include "tc_internal.h"
#include "closure.h"
#include "walk_common.h"

#include <math.h>

namespace tc {
namespace {

using namespace walk;
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int kWPB = 4;                               // waves per block

struct NetT {                                         // transposed BF16 weights
    short4_t w1t[kNHid * 16 / 4];                     // W1^T [64 hidden][16 inputs]
    short4_t w2t[kNHid * kNHid / 4];                  // W2^T [64 out][64 in]
    short4_t w3t[16 * kNHid / 4];                     // W3^T [16 outputs][64 hidden]
    float b1[kNHid], b2[kNHid], b3[16];
};

__device__ __forceinline__ uint16_t f2bf(float f) {   // round to nearest, ties to even
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}

__device__ __forceinline__ float gelu(float z) { return gelu_f(z); }

__device__ __forceinline__ short4_t pack_gelu(float4_t z, const float* b, int h0) {
    short4_t r;
#pragma unroll
    for (int q = 0; q < 4; ++q) r[q] = (short)f2bf(gelu(z[q] + b[h0 + q]));
    return r;
}

__device__ void load_net_t(const MlpState* __restrict__ st, NetT& N) {
    uint16_t* w1t = reinterpret_cast<uint16_t*>(N.w1t);
    uint16_t* w2t = reinterpret_cast<uint16_t*>(N.w2t);
    uint16_t* w3t = reinterpret_cast<uint16_t*>(N.w3t);
    for (int i = threadIdx.x; i < kNHid * 16; i += blockDim.x) {
        const int h = i / 16, in = i % 16;
        w1t[i] = st->w1[in * kNHid + h];
    }
    for (int i = threadIdx.x; i < kNHid * kNHid; i += blockDim.x) {
        const int o = i / kNHid, in = i % kNHid;
        w2t[i] = st->w2[in * kNHid + o];
    }
    for (int i = threadIdx.x; i < 16 * kNHid; i += blockDim.x) {
        const int o = i / kNHid, h = i % kNHid;
        w3t[i] = st->w3[h * 16 + o];
    }
    for (int i = threadIdx.x; i < kNHid; i += blockDim.x) {
        N.b1[i] = st->b1[i];
        N.b2[i] = st->b2[i];
    }
    if (threadIdx.x < 16) N.b3[threadIdx.x] = st->b3[threadIdx.x];
}

// Network outputs for the wave's 64 samples; xs holds one BF16 feature row
// (16 entries, 10 used) per sample.  Returns lane l's outputs in y[0..2].
__device__ void net_infer(const NetT& N, const short4_t* xs, float4_t* ys, float y[3]) {
    const int l = threadIdx.x & (kWave - 1);
    const int r = l & 15, g = l >> 4;
    short4_t h1[4][4], h2[4][4];                      // [hidden tile][sample tile]
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        const short4_t b = xs[(16 * st + r) * 4 + g];  // X^T rows 4g..4g+3, column 16st+r
#pragma unroll
        for (int ht = 0; ht < 4; ++ht) {
            const short4_t a = N.w1t[(16 * ht + r) * 4 + g];
            float4_t z = {0.f, 0.f, 0.f, 0.f};
            z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, z, 0, 0, 0);
            h1[ht][st] = pack_gelu(z, N.b1, 16 * ht + 4 * g);
        }
    }
#pragma unroll
    for (int ht = 0; ht < 4; ++ht)
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            float4_t z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kc = 0; kc < 4; ++kc)
                z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(N.w2t[(16 * ht + r) * 16 + 4 * kc + g], h1[kc][st],
                                                            z, 0, 0, 0);
            h2[ht][st] = pack_gelu(z, N.b2, 16 * ht + 4 * g);
        }
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        float4_t z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < 4; ++kc)
            z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(N.w3t[r * 16 + 4 * kc + g], h2[kc][st], z, 0, 0, 0);
        if (g == 0) ys[16 * st + r] = z;               // outputs 0..3 of sample 16st+r
    }
    wave_lds_sync();
    const float4_t o = ys[l];
    y[0] = o[0] + N.b3[0];
    y[1] = o[1] + N.b3[1];
    y[2] = o[2] + N.b3[2];
    wave_lds_sync();
}

__global__ void __launch_bounds__(256) k_walk_force_learned(
    const WalkCell* __restrict__ walk, const double* __restrict__ rcp2, const Body* __restrict__ bodies,
    const float4* __restrict__ bodies32, const Cell* __restrict__ cells, const Moments* __restrict__ mom,
    const uint32_t* __restrict__ bfs2pre, const uint32_t* __restrict__ perm, const int32_t* __restrict__ gbeg,
    const int32_t* __restrict__ gcnt, uint32_t* queue, const MlpState* __restrict__ st, int lpl_log2, float G,
    float eps2, float tau, int64_t n, const DevParams* __restrict__ prm, float* __restrict__ acc,
    float* __restrict__ pot, int64_t* __restrict__ m2p_out, int64_t* __restrict__ p2p_out,
    int64_t* __restrict__ learned_out, int64_t* __restrict__ fallback_out) {
    constexpr int R = 8, RP = kWave / R;
    constexpr int kReserve = (R - 1) * 21 + R;
    static_assert(kStackCap >= kWave + kReserve + kWave, "stack too small for its bound");

    __shared__ NetT N;
    __shared__ float4 s_list[kWPB][kListCap];
    __shared__ uint32_t s_stack[kWPB][kStackCap];
    __shared__ short4_t s_x[kWPB][kWave * 4];
    __shared__ float4_t s_y[kWPB][kWave];
    load_net_t(st, N);
    __syncthreads();

    const int wv = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    float4* L = s_list[wv];
    uint32_t* S = s_stack[wv];
    short4_t* xs = s_x[wv];
    float4_t* ys = s_y[wv];
    const int lpl = 1 << lpl_log2;
    const int slot = lane >> lpl_log2, jj = lane & (lpl - 1);
    const double size = prm->size;
    const double mbar = mom[0].M / (double)n;          // mean body mass (root cell)

    const GroupSched sched = make_sched(queue, prm->ngroups, kWPB);
    for (int hop = 0; hop < kXcd; ++hop) {
        const int xq = (sched.home + hop) % kXcd;
        const uint32_t g_hi = sched.share_lo(xq + 1);
        uint32_t g = sched.first(xq, hop);
        while (g < g_hi) {
            const int64_t i0 = gbeg[g];
            const int gn = gcnt[g];
            const int64_t i = i0 + lane;
            const bool valid = lane < gn;
            const Body me = bodies[valid ? i : i0];
            const double lox = uniform(wave_min(me.x)), hix = uniform(wave_max(me.x));
            const double loy = uniform(wave_min(me.y)), hiy = uniform(wave_max(me.y));
            const double loz = uniform(wave_min(me.z)), hiz = uniform(wave_max(me.z));
            const double rx = (lox + hix) * 0.5, ry = (loy + hiy) * 0.5, rz = (loz + hiz) * 0.5;
            const float xi = (float)(me.x - rx), yi = (float)(me.y - ry), zi = (float)(me.z - rz);

            Acc a = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            float kx = 0.f, ky = 0.f, kz = 0.f, ckx = 0.f, cky = 0.f, ckz = 0.f;  // closure corrections
            int len = 0;
            int64_t nm2p = 0, np2p = 0, nlearn = 0, nfall = 0;
            if (lane == 0) S[0] = 0u;                    // root, mode L
            wave_lds_sync();
            int top = 1;

            // copy bodies [bl, bl + cl) into the list in pieces of 64
            auto copy_bodies = [&](int bl, int cl) {
                for (int o = 0; o < cl; o += kWave) {
                    const int m = min(kWave, cl - o);
                    if (len + m > kListCap) {
                        flush<3>(L, len, xi, yi, zi, eps2, a);
                        len = 0;
                    }
                    if (lane < m) L[len + lane] = body_entry(bodies, bodies32, bl + o + lane, rx, ry, rz);
                    len += m;
                }
                np2p += cl;
            };

            while (top > 0) {
                const int nr = (top + kWave + kReserve <= kStackCap) ? min(top, RP) : 1;
                const int rr = lane / R, j = lane % R;
                uint32_t packed = 0;
                if (rr < nr) packed = S[top - 1 - rr];
                top -= nr;
                const bool modeP = (packed >> 3) & 1u;
                const int rlen = (int)(packed & 7u) + 1;
                const bool vc = rr < nr && j < rlen;
                const uint32_t bidx = (packed >> 4) + (uint32_t)j;
                wave_lds_sync();
                const WalkCell wc = load_cell(walk, bidx, vc);
                const double rp = vc ? rcp2[bidx] : INFINITY;

                const double dxm = fmax(fmax(lox - wc.cx, 0.0), wc.cx - hix);
                const double dym = fmax(fmax(loy - wc.cy, 0.0), wc.cy - hiy);
                const double dzm = fmax(fmax(loz - wc.cz, 0.0), wc.cz - hiz);
                const double d2 = (dxm * dxm + dym * dym) + dzm * dzm;
                const bool leaf = vc && wc.b < 0;
                const bool accL = vc && d2 > wc.rcrit2;
                const bool accP = vc && d2 > rp;
                const bool acc_plain = modeP ? accP : accL && accP;
                const bool learned = !modeP && accL && !accP;
                const bool closed = modeP ? accP : accL;   // accepted in its own mode
                const bool opened = vc && !closed && !leaf;
                const bool direct = leaf && !closed;

                const uint64_t O = __ballot(opened);
                if (opened)
                    S[top + __popcll(O & below)] =
                        ((uint32_t)wc.a << 4) | (modeP ? 8u : 0u) | (uint32_t)(wc.b - 1);
                top += __popcll(O);
                wave_lds_sync();

                // plain monopole entries
                const uint64_t A = __ballot(acc_plain);
                const int na = __popcll(A);
                if (na) {
                    if (len + na > kListCap) {
                        flush<3>(L, len, xi, yi, zi, eps2, a);
                        len = 0;
                    }
                    if (acc_plain)
                        L[len + __popcll(A & below)] =
                            make_float4((float)(wc.cx - rx), (float)(wc.cy - ry), (float)(wc.cz - rz), wc.m);
                    len += na;
                    nm2p += na;
                }

                // leaves taken directly
                const int cnt = direct ? (wc.b & 0x7fffffff) : 0;
                const uint64_t P = __ballot(direct);
                if (P) {
                    const uint64_t big = __ballot(direct && cnt > lpl);
                    uint64_t small = P & ~big;
                    while (small) {
                        int my_begin = 0, my_cnt = 0, my_off = 0, tot = 0;
                        for (int s = 0; s < (kWave >> lpl_log2) && small; ++s) {
                            const int l = __builtin_ctzll(small);
                            small &= small - 1;
                            const int cl = __builtin_amdgcn_readlane(cnt, l);
                            const int bl = __builtin_amdgcn_readlane(wc.a, l);
                            if (slot == s) {
                                my_begin = bl;
                                my_cnt = cl;
                                my_off = tot;
                            }
                            tot += cl;
                        }
                        if (len + tot > kListCap) {
                            flush<3>(L, len, xi, yi, zi, eps2, a);
                            len = 0;
                        }
                        if (jj < my_cnt)
                            L[len + my_off + jj] = body_entry(bodies, bodies32, my_begin + jj, rx, ry, rz);
                        len += tot;
                        np2p += tot;
                    }
                    uint64_t bg = big;
                    while (bg) {
                        const int l = __builtin_ctzll(bg);
                        bg &= bg - 1;
                        copy_bodies(__builtin_amdgcn_readlane(wc.a, l), __builtin_amdgcn_readlane(cnt, l));
                    }
                }

                // learned cells, one at a time with the whole wave
                uint64_t Lm = __ballot(learned);
                while (Lm) {
                    const int l = __builtin_ctzll(Lm);
                    Lm &= Lm - 1;
                    const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)bidx, l);
                    const int64_t kc = bfs2pre[b];
                    const Moments& mo = mom[kc];
                    const double cx = mo.com[0], cy = mo.com[1], cz = mo.com[2], M = mo.M;
                    const int lev = cells[kc].level;
                    const double s = ldexp(size, -lev);
                    const double inv_s = ldexp(1.0 / size, lev);   // exact: size is a power of two
                    const double iq = 1.0 / (M * s * s);
                    short4_t f4[4];
                    {
                        float f[16];
                        f[0] = (float)((me.x - cx) * inv_s);
                        f[1] = (float)((me.y - cy) * inv_s);
                        f[2] = (float)((me.z - cz) * inv_s);
#pragma unroll
                        for (int q = 0; q < 6; ++q) f[3 + q] = (float)(mo.Q[q] * iq);
                        f[9] = (float)log(M / mbar);
#pragma unroll
                        for (int q = 10; q < 16; ++q) f[q] = 0.f;
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            f4[q] = short4_t{(short)f2bf(f[4 * q]), (short)f2bf(f[4 * q + 1]),
                                             (short)f2bf(f[4 * q + 2]), (short)f2bf(f[4 * q + 3])};
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) xs[lane * 4 + q] = f4[q];
                    wave_lds_sync();
                    float yh[3];
                    net_infer(N, xs, ys, yh);
                    // predicted residual relative to the monopole: |yhat| s^2 / |x - C|^2
                    const double ex = me.x - cx, ey = me.y - cy, ez = me.z - cz;
                    const double dd = (ex * ex + ey * ey) + ez * ez;
                    const float ratio =
                        valid ? sqrtf(yh[0] * yh[0] + yh[1] * yh[1] + yh[2] * yh[2]) * (float)(s * s / dd) : 0.f;
                    float gmax = ratio;
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) gmax = fmaxf(gmax, __shfl_xor(gmax, o, kWave));
                    gmax = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(gmax)));
                    if (gmax > tau) {
                        // fall back to the plain walk of this cell at theta_P
                        nfall += 1;
                        const int wa = __builtin_amdgcn_readlane(wc.a, l);
                        const int wb = __builtin_amdgcn_readlane(wc.b, l);
                        if (wb < 0) {
                            copy_bodies(wa, wb & 0x7fffffff);
                        } else {
                            if (lane == 0) S[top] = ((uint32_t)wa << 4) | 8u | (uint32_t)(wb - 1);
                            top += 1;
                            wave_lds_sync();
                        }
                    } else {
                        nlearn += 1;
                        nm2p += 1;
                        if (len + 1 > kListCap) {
                            flush<3>(L, len, xi, yi, zi, eps2, a);
                            len = 0;
                        }
                        if (lane == 0)
                            L[len] = make_float4((float)(cx - rx), (float)(cy - ry), (float)(cz - rz), (float)M);
                        len += 1;
                        const float w = (float)(M * s * s / (dd * dd));   // quadrupole scale
                        comp_add(kx, ckx, w * yh[0]);
                        comp_add(ky, cky, w * yh[1]);
                        comp_add(kz, ckz, w * yh[2]);
                    }
                }
                wave_lds_sync();
            }
            flush<3>(L, len, xi, yi, zi, eps2, a);

            if (valid) {
                const float mself = (float)me.m;
                const float sself = __builtin_amdgcn_rsqf(eps2);
                const float ph = (a.sp + a.cp) + mself * sself;
                const int64_t o = perm[i];
                acc[o * 3 + 0] = G * ((a.sx + a.cx) + (kx + ckx));
                acc[o * 3 + 1] = G * ((a.sy + a.cy) + (ky + cky));
                acc[o * 3 + 2] = G * ((a.sz + a.cz) + (kz + ckz));
                pot[o] = G * ph;
            }
            if (lane == 0) {
                m2p_out[g] = nm2p;
                p2p_out[g] = np2p;
                learned_out[g] = nlearn;
                fallback_out[g] = nfall;
            }
            g = sched.pop(xq);
        }
    }
}

__global__ void k_reset_queue_l(uint32_t* queue) { reset_sched(queue); }

}  // namespace

hipError_t launch_walk_force_learned(const WalkCell* walk, const double* rcp2, const Body* bodies,
                                     const float4* bodies32, const Cell* cells, const Moments* mom,
                                     const uint32_t* bfs2pre, const uint32_t* perm, const int32_t* gbeg,
                                     const int32_t* gcnt, int64_t gmax, uint32_t* queue, const MlpState* st,
                                     int leaf_cap, float G, float eps2, float tau, int64_t n,
                                     const DevParams* prm, float* acc, float* pot, int64_t* m2p, int64_t* p2p,
                                     int64_t* learned, int64_t* fallback, hipStream_t s) {
    static int resident = 0;
    if (resident == 0) {
        int dev = 0, cus = 0, per_cu = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_walk_force_learned, 256, 0);
        if (e != hipSuccess) return e;
        resident = cus * (per_cu > 0 ? per_cu : 1);
    }
    int64_t want = (gmax + kWPB - 1) / kWPB;
    if (want > resident) want = resident;
    if (want < kXcd) want = kXcd;
    int lpl_log2 = 0;
    while ((1 << lpl_log2) < leaf_cap && lpl_log2 < 6) ++lpl_log2;
    hipLaunchKernelGGL(k_reset_queue_l, dim3(1), dim3(64), 0, s, queue);
    hipLaunchKernelGGL(k_walk_force_learned, dim3((unsigned)want), dim3(256), 0, s, walk, rcp2, bodies, bodies32, cells,
                       mom, bfs2pre, perm, gbeg, gcnt, queue, st, lpl_log2, G, eps2, tau, n, prm, acc, pot, m2p,
                       p2p, learned, fallback);
    return hipGetLastError();
}

}  // namespace tc
