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
// A learned cell costs the wave one network pass over its 64 bodies, in
// four tiles of 16 samples (net_tile in closure.h: activations stay in
// registers, weights are matrix-core fragments in LDS shared by the block's
// eight waves, biases start the accumulators).  Sample tiles past the
// group's last body are skipped.  Each lane computes the features of the
// samples its lane group feeds to the matrix cores from the group's FP64
// positions, staged in LDS once per group.
#include "tc_internal.h"
#include "closure.h"
#include "walk_common.h"

#include <math.h>

namespace tc {
namespace {

using namespace walk;

constexpr int kWPB = 8;                               // waves per block (one copy of the weights each)

__global__ void __launch_bounds__(kWPB * 64, 4) k_walk_force_learned(
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

    __shared__ NetF N;
    __shared__ float4 s_list[kWPB][kListCap];
    __shared__ uint32_t s_stack[kWPB][kStackCap];
    __shared__ double s_pos[kWPB][3][kWave];          // the group's FP64 positions
    __shared__ float4_t s_y[kWPB][kWave];              // network outputs per body
    load_net_frags(st, N, threadIdx.x, blockDim.x);
    __syncthreads();

    const int wv = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    const int lg = lane >> 4, lr = lane & 15;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    float4* L = s_list[wv];
    uint32_t* S = s_stack[wv];
    double* PX = s_pos[wv][0];
    double* PY = s_pos[wv][1];
    double* PZ = s_pos[wv][2];
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
            const int ntiles = (gn + 15) >> 4;              // sample tiles holding bodies

            Acc a = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            float kx = 0.f, ky = 0.f, kz = 0.f, ckx = 0.f, cky = 0.f, ckz = 0.f;  // closure corrections
            int len = 0;
            int64_t nm2p = 0, np2p = 0, nlearn = 0, nfall = 0;
            PX[lane] = me.x;
            PY[lane] = me.y;
            PZ[lane] = me.z;
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
                    // features the lane group feeds: g = 0: u (3) and Q_xx; g = 1: Q_yy, Q_zz,
                    // Q_xy, Q_xz; g = 2: Q_yz and ln(M / mbar); g = 3: zero padding
                    short4_t xc = {0, 0, 0, 0};
                    if (lg == 1)
                        xc = short4_t{bf16_bits((float)(mo.Q[1] * iq)), bf16_bits((float)(mo.Q[2] * iq)),
                                      bf16_bits((float)(mo.Q[3] * iq)), bf16_bits((float)(mo.Q[4] * iq))};
                    else if (lg == 2)
                        xc = short4_t{bf16_bits((float)(mo.Q[5] * iq)), bf16_bits((float)log(M / mbar)), 0, 0};
                    const short qxx = bf16_bits((float)(mo.Q[0] * iq));
                    for (int t = 0; t < ntiles; ++t) {
                        // the weight fragments are read from LDS per tile, not held in registers
                        __asm__ volatile("" ::: "memory");
                        short4_t x = xc;
                        if (lg == 0) {
                            const int sb = 16 * t + lr;
                            x = short4_t{bf16_bits((float)((PX[sb] - cx) * inv_s)),
                                         bf16_bits((float)((PY[sb] - cy) * inv_s)),
                                         bf16_bits((float)((PZ[sb] - cz) * inv_s)), qxx};
                        }
                        const float4_t yt = net_tile(N, x);
                        if (lg == 0) ys[16 * t + lr] = yt;
                    }
                    wave_lds_sync();
                    const float4_t yo = ys[lane];
                    wave_lds_sync();
                    // predicted residual relative to the monopole: |yhat| s^2 / |x - C|^2
                    const double ex = me.x - cx, ey = me.y - cy, ez = me.z - cz;
                    const double dd = (ex * ex + ey * ey) + ez * ez;
                    const float ratio =
                        valid ? sqrtf(yo[0] * yo[0] + yo[1] * yo[1] + yo[2] * yo[2]) * (float)(s * s / dd) : 0.f;
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
                        comp_add(kx, ckx, w * yo[0]);
                        comp_add(ky, cky, w * yo[1]);
                        comp_add(kz, ckz, w * yo[2]);
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
            wave_lds_sync();                          // positions are rewritten by the next group
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
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_walk_force_learned, kWPB * 64, 0);
        if (e != hipSuccess) return e;
        resident = cus * (per_cu > 0 ? per_cu : 1);
    }
    int64_t want = (gmax + kWPB - 1) / kWPB;
    if (want > resident) want = resident;
    if (want < kXcd) want = kXcd;
    int lpl_log2 = 0;
    while ((1 << lpl_log2) < leaf_cap && lpl_log2 < 6) ++lpl_log2;
    hipLaunchKernelGGL(k_reset_queue_l, dim3(1), dim3(64), 0, s, queue);
    hipLaunchKernelGGL(k_walk_force_learned, dim3((unsigned)want), dim3(kWPB * 64), 0, s, walk, rcp2, bodies,
                       bodies32, cells, mom, bfs2pre, perm, gbeg, gcnt, queue, st, lpl_log2, G, eps2, tau, n, prm, acc,
                       pot, m2p, p2p, learned, fallback);
    return hipGetLastError();
}

}  // namespace tc
