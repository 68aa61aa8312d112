// Fast multipole method (§5 of the paper points to it as the step beyond the
// treecode): cell-cell interactions through Cartesian expansions, 3D.
//
//   * every cell has its multipole about its centre of mass (mass M and the
//     traceless quadrupole Q; the dipole vanishes there) and a local
//     expansion about its geometric centre z: 20 FP64 coefficients of
//       phi(z + dl) = -G sum_{n<=3} (1/n!) Lam_n[dl^n];
//   * a dual tree traversal, one level of pairs per launch, sorts every
//     (target A, source B) pair reached from (root, root): a cell with
//     itself becomes all pairs of its children (a leaf: a direct sum); A and
//     B are far enough for an expansion when |z_A - com_B| > (rho_A + rho_B)
//     / theta, rho_A and rho_B bounding their bodies about z_A and com_B
//     (from the bodies for a leaf, from the children for a cell, capped by
//     the geometric bounds); two leaves that are not sum
//     directly; otherwise the larger cell (smaller level, A on a tie, never
//     a leaf) is split;
//   * M2L: with g(R) = (|R|^2 + eps^2)^(-1/2), D_n its derivative tensors and
//     R = z_A - com_B, Lam_n += M D_n(R) + (1/6) Q:D_(n+2)(R), truncated at
//     total order 3 (the quadrupole acts on Lam_0 and Lam_1);
//   * L2L from every parent to its children, level by level;
//   * per leaf: the expansion at each body (L2P) plus the direct sums over
//     its partner leaves in FP32 (P2P), coordinates relative to the leaf
//     centre, compensated as in the treecode force loop.
//
// The traversal writes its pairs in a fixed order and a stable sort groups
// them by target, so every sum runs in a fixed order and results are
// reproducible bit for bit.
#include "tc_internal.h"
#include "walk_common.h"

#include <math.h>

namespace tc {
namespace {

using namespace walk;

constexpr double kHalfSqrt3 = 0.8660254037844386;   // sqrt(3)/2, rounded to FP64

// Symmetric tensor slots of a local expansion:
//   0: Lam_0;  1..3: x, y, z;  4..9: xx, yy, zz, xy, xz, yz;
//   10..19: xxx, yyy, zzz, xxy, xxz, xyy, yyz, xzz, yzz, xyz.
constexpr int kNL = 20;

__device__ __forceinline__ bool is_leaf(const Cell& c) { return c.leaf_nch < 0; }
__device__ __forceinline__ int nchildren(const Cell& c) { return c.leaf_nch & 0x7fffffff; }

__global__ void __launch_bounds__(256) k_fmm_geo(const Cell* __restrict__ cells, const Moments* __restrict__ mom,
                                                 const WalkCell* __restrict__ walk,
                                                 const uint32_t* __restrict__ pre2bfs,
                                                 const DevParams* __restrict__ prm, int64_t cmax,
                                                 FmmGeo* __restrict__ geo, DttCell* __restrict__ dc) {
    int64_t C = prm->ncells;
    if (C > cmax) C = cmax;
    const double size = prm->size;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < C; k += (int64_t)gridDim.x * blockDim.x) {
        const Cell c = cells[k];
        const int l = c.level;
        const double s = ldexp(size, -l);
        uint64_t org[3] = {0, 0, 0};
        for (int j = 1; j <= l; ++j) {
            const unsigned d = (unsigned)((c.prefix >> (3 * (l - j))) & 7u);
#pragma unroll
            for (int a = 0; a < 3; ++a) org[a] = (org[a] << 1) | ((d >> (2 - a)) & 1u);
        }
        FmmGeo g;
        double d[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            g.z[a] = prm->lo[a] + ((double)org[a] + 0.5) * s;
            d[a] = mom[k].com[a] - g.z[a];
        }
        // geometric bounds; k_fmm_radii tightens them from the bodies
        g.rhoA = kHalfSqrt3 * s;
        g.rhoB = kHalfSqrt3 * s + sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
        g.pad[0] = g.pad[1] = g.pad[2] = 0.0;
        geo[k] = g;
        const uint32_t kb = pre2bfs[k];
        DttCell t;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            t.z[a] = g.z[a];
            t.com[a] = mom[k].com[a];
        }
        t.rhoA = g.rhoA;
        t.rhoB = g.rhoB;
        t.child = is_leaf(c) ? -1 : walk[kb].a;
        t.nch_leaf = c.leaf_nch;
        t.level = l;
        t.pre = (int32_t)k;
        dc[kb] = t;
    }
}

__device__ __forceinline__ uint64_t pair_key(uint32_t a, uint32_t b) { return ((uint64_t)a << 32) | b; }

__device__ __forceinline__ double dist3(double ax, double ay, double az, double bx, double by, double bz) {
    const double dx = ax - bx, dy = ay - by, dz = az - bz;
    return sqrt((dx * dx + dy * dy) + dz * dz);
}

// The radii of the cells of one level (level-order range), deepest level
// first: rho_A bounds the cell's bodies about its centre z, rho_B about its
// centre of mass; for a leaf the largest distance of one of its bodies, for
// an internal cell the largest (distance between the centres + the child's
// radius) over its children; each capped by the geometric bound.
__global__ void __launch_bounds__(256) k_fmm_radii(const Cell* __restrict__ cells, const Moments* __restrict__ mom,
                                                   const Body* __restrict__ bodies, const WalkCell* __restrict__ walk,
                                                   const uint32_t* __restrict__ bfs2pre,
                                                   const uint32_t* __restrict__ lvl_off, int level,
                                                   FmmGeo* __restrict__ geo, DttCell* __restrict__ dc) {
    const int64_t lo = lvl_off[level], hi = lvl_off[level + 1];
    for (int64_t k = lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < hi;
         k += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t c = bfs2pre[k];
        const Cell cc = cells[c];
        FmmGeo g = geo[c];
        const double cx = mom[c].com[0], cy = mom[c].com[1], cz = mom[c].com[2];
        double ra = 0.0, rb = 0.0;
        if (is_leaf(cc)) {
            for (int64_t j = cc.begin; j < (int64_t)cc.begin + cc.count; ++j) {
                const Body b = bodies[j];
                ra = fmax(ra, dist3(b.x, b.y, b.z, g.z[0], g.z[1], g.z[2]));
                rb = fmax(rb, dist3(b.x, b.y, b.z, cx, cy, cz));
            }
        } else {
            const int32_t first = walk[k].a;
            const int nch = nchildren(cc);
            for (int i = 0; i < nch; ++i) {
                const uint32_t ch = bfs2pre[first + i];
                const FmmGeo gc = geo[ch];
                ra = fmax(ra, dist3(gc.z[0], gc.z[1], gc.z[2], g.z[0], g.z[1], g.z[2]) + gc.rhoA);
                rb = fmax(rb, dist3(mom[ch].com[0], mom[ch].com[1], mom[ch].com[2], cx, cy, cz) + gc.rhoB);
            }
        }
        g.rhoA = fmin(ra, g.rhoA);
        g.rhoB = fmin(rb, g.rhoB);
        geo[c] = g;
        dc[k].rhoA = g.rhoA;
        dc[k].rhoB = g.rhoB;
    }
}

// One level of the traversal, on level-order cell indices: every input
// pair becomes an M2L pair, a P2P pair, or pairs of the next level.  Three
// launches per level keep the output order fixed: each block counts the
// outputs of its contiguous chunk of the input, one block turns the counts
// into every block's first slots (and advances the running totals), and
// each block writes its outputs in thread order.  A slot at or beyond a
// capacity is counted but not written.  M2L and P2P pairs are stored as
// (source << 32) | target with pre-order indices, ready for the sort by
// target; pairs of the next level as (A << 32) | B in level order.
struct DttOut {
    int kind;          // 0: nothing, 1: M2L, 2: P2P, 3: children x children, 4: children x B, 5: A x children
    uint32_t A, B;
    int32_t child, nch;
};

__device__ __forceinline__ DttOut dtt_classify(const DttCell* __restrict__ dc, double theta, uint64_t pr) {
    DttOut o;
    o.A = (uint32_t)(pr >> 32);
    o.B = (uint32_t)pr;
    o.child = 0;
    o.nch = 0;
    const DttCell ca = dc[o.A];
    const bool la = ca.nch_leaf < 0;
    if (o.A == o.B) {
        o.kind = la ? 2 : 3;
        o.child = ca.child;
        o.nch = ca.nch_leaf & 0x7fffffff;
        return o;
    }
    const DttCell cb = dc[o.B];
    bool acc = false;
    if (theta != 0.0) {
        double d[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) d[a] = ca.z[a] - cb.com[a];
        const double d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
        const double r = (ca.rhoA + cb.rhoB) / theta;
        acc = d2 > r * r;
    }
    const bool lb = cb.nch_leaf < 0;
    if (acc) {
        o.kind = 1;
    } else if (la && lb) {
        o.kind = 2;
    } else if (!la && (lb || ca.level <= cb.level)) {
        o.kind = 4;
        o.child = ca.child;
        o.nch = ca.nch_leaf & 0x7fffffff;
    } else {
        o.kind = 5;
        o.child = cb.child;
        o.nch = cb.nch_leaf & 0x7fffffff;
    }
    return o;
}

__device__ __forceinline__ uint32_t dtt_next(const DttOut& o) {
    return o.kind == 3 ? (uint32_t)(o.nch * o.nch) : (o.kind >= 4 ? (uint32_t)o.nch : 0u);
}

constexpr int kDttBlock = 256;
constexpr int kDttWaves = kDttBlock / kWave;

// The same contiguous chunk of the input for a block in both sweeps.
__device__ __forceinline__ void dtt_chunk(int64_t nin, int64_t& begin, int64_t& end) {
    const int64_t chunk = ((nin + gridDim.x - 1) / gridDim.x + kDttBlock - 1) / kDttBlock * kDttBlock;
    begin = (int64_t)blockIdx.x * chunk;
    end = min(nin, begin + chunk);
    if (end < begin) end = begin;
}

// Exclusive prefix of (a, b, c) over the block's threads in thread order;
// returns the block totals in tot.  All threads must call it.
__device__ __forceinline__ void block_scan3(uint32_t a, uint32_t b, uint32_t c, uint32_t* ex, uint32_t* tot,
                                            uint32_t (*sw)[3]) {
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    uint32_t v[3] = {a, b, c};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t y = __shfl_up(v[k], o, kWave);
            if (lane >= o) v[k] += y;
        }
    }
    if (lane == kWave - 1) {
        sw[wv][0] = v[0];
        sw[wv][1] = v[1];
        sw[wv][2] = v[2];
    }
    __syncthreads();
    uint32_t before[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        tot[k] = 0;
        for (int w = 0; w < kDttWaves; ++w) {
            if (w < wv) before[k] += sw[w][k];
            tot[k] += sw[w][k];
        }
    }
    ex[0] = before[0] + v[0] - a;
    ex[1] = before[1] + v[1] - b;
    ex[2] = before[2] + v[2] - c;
    __syncthreads();
}

// Sweep 1: bt[k * gridDim.x + block] = the block's M2L (k = 0), P2P (1)
// and next-level (2) output counts.
__global__ void __launch_bounds__(kDttBlock) k_fmm_dtt_count(const DttCell* __restrict__ dc, double theta,
                                                             const uint64_t* __restrict__ fin, int64_t nin,
                                                             uint32_t* __restrict__ bt) {
    __shared__ uint32_t sw[kDttWaves][3];
    int64_t begin, end;
    dtt_chunk(nin, begin, end);
    uint32_t cm = 0, cp = 0, cn = 0;
    for (int64_t i = begin + threadIdx.x; i < end; i += kDttBlock) {
        const DttOut o = dtt_classify(dc, theta, fin[i]);
        cm += o.kind == 1;
        cp += o.kind == 2;
        cn += dtt_next(o);
    }
    uint32_t ex[3], tot[3];
    block_scan3(cm, cp, cn, ex, tot, sw);
    if (threadIdx.x == 0) {
        bt[blockIdx.x] = tot[0];
        bt[gridDim.x + blockIdx.x] = tot[1];
        bt[2 * gridDim.x + blockIdx.x] = tot[2];
    }
}

// One block: every block's first output slots (M2L and P2P after the
// running totals ctr[1], ctr[2]; the next level from 0), then ctr[0] =
// next-level size and ctr[1], ctr[2] advanced.
__global__ void __launch_bounds__(1024) k_fmm_dtt_scan(const uint32_t* __restrict__ bt, int nb,
                                                       unsigned long long* __restrict__ ctr,
                                                       unsigned long long* __restrict__ base) {
    __shared__ unsigned long long s[1024];
    const int t = threadIdx.x;
    const int per = (nb + 1023) / 1024;    // at most kFmmMaxBlocks / 1024 blocks per thread
    for (int k = 0; k < 3; ++k) {
        unsigned long long mine = 0;
        for (int j = 0; j < per; ++j) {
            const int b = t * per + j;
            if (b < nb) mine += bt[k * nb + b];
        }
        s[t] = mine;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {     // inclusive Hillis-Steele scan
            const unsigned long long y = t >= o ? s[t - o] : 0ull;
            __syncthreads();
            s[t] += y;
            __syncthreads();
        }
        const unsigned long long start = (k == 2 ? 0ull : ctr[k + 1]) + s[t] - mine;
        unsigned long long run = start;
        for (int j = 0; j < per; ++j) {
            const int b = t * per + j;
            if (b < nb) {
                base[k * nb + b] = run;
                run += bt[k * nb + b];
            }
        }
        const unsigned long long total = s[1023];
        __syncthreads();
        if (t == 0) {
            if (k == 2) ctr[0] = total;
            else ctr[k + 1] += total;
        }
        __syncthreads();
    }
}

// Sweep 2: the same classification, written in thread order from the
// block's first slots.
__global__ void __launch_bounds__(kDttBlock) k_fmm_dtt_write(const DttCell* __restrict__ dc, double theta,
                                                             const uint64_t* __restrict__ fin, int64_t nin,
                                                             const unsigned long long* __restrict__ base,
                                                             uint64_t* __restrict__ fout, int64_t capf,
                                                             uint64_t* __restrict__ m2l, int64_t capm,
                                                             uint64_t* __restrict__ p2p, int64_t capp) {
    __shared__ uint32_t sw[kDttWaves][3];
    int64_t begin, end;
    dtt_chunk(nin, begin, end);
    const int64_t iters = (end - begin + kDttBlock - 1) / kDttBlock;
    uint64_t om = base[blockIdx.x], op = base[gridDim.x + blockIdx.x], on = base[2 * gridDim.x + blockIdx.x];
    for (int64_t it = 0; it < iters; ++it) {
        const int64_t i = begin + it * kDttBlock + threadIdx.x;
        DttOut o;
        o.kind = 0;
        o.nch = 0;
        if (i < end) o = dtt_classify(dc, theta, fin[i]);
        uint32_t ex[3], tot[3];
        block_scan3(o.kind == 1, o.kind == 2, dtt_next(o), ex, tot, sw);
        if (o.kind == 1 || o.kind == 2) {
            const uint64_t key = ((uint64_t)(uint32_t)dc[o.B].pre << 32) | (uint32_t)dc[o.A].pre;
            if (o.kind == 1) {
                const uint64_t s = om + ex[0];
                if ((int64_t)s < capm) m2l[s] = key;
            } else {
                const uint64_t s = op + ex[1];
                if ((int64_t)s < capp) p2p[s] = key;
            }
        } else if (o.kind == 3) {
            uint64_t s = on + ex[2];
            for (int x = 0; x < o.nch; ++x)
                for (int y = 0; y < o.nch; ++y, ++s)
                    if ((int64_t)s < capf) fout[s] = pair_key((uint32_t)(o.child + x), (uint32_t)(o.child + y));
        } else if (o.kind == 4) {
            const uint64_t s = on + ex[2];
            for (int j = 0; j < o.nch; ++j)
                if ((int64_t)(s + j) < capf) fout[s + j] = pair_key((uint32_t)(o.child + j), o.B);
        } else if (o.kind == 5) {
            const uint64_t s = on + ex[2];
            for (int j = 0; j < o.nch; ++j)
                if ((int64_t)(s + j) < capf) fout[s + j] = pair_key(o.A, (uint32_t)(o.child + j));
        }
        om += tot[0];
        op += tot[1];
        on += tot[2];
    }
}

// Start of every target's run in the keys sorted by target (the low 32
// bits): off[t] = the first key whose target is >= t, for t = 0..C
// (off[C] = n).
__global__ void __launch_bounds__(256) k_fmm_offsets(const uint64_t* __restrict__ keys, int64_t n, int64_t C,
                                                     uint32_t* __restrict__ off) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t <= C; t += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if ((int64_t)(uint32_t)keys[mid] < t) lo = mid + 1;
            else hi = mid;
        }
        off[t] = (uint32_t)lo;
    }
}

// ---- expansions, FP64

// Add the expansion of a source (M, traceless Q at its centre of mass) at
// R = centre - source to lam.
__device__ __forceinline__ void m2l_add(double M, const double* Q, double x, double y, double z, double eps2,
                                        double* lam) {
    const double r2 = ((x * x + y * y) + z * z) + eps2;
    const double s = 1.0 / sqrt(r2);
    const double s2 = s * s, s3 = s2 * s, s5 = s3 * s2, s7 = s5 * s2;
    const double Qxx = Q[0], Qyy = Q[1], Qzz = Q[2], Qxy = Q[3], Qxz = Q[4], Qyz = Q[5];
    const double qx = Qxx * x + Qxy * y + Qxz * z;
    const double qy = Qxy * x + Qyy * y + Qyz * z;
    const double qz = Qxz * x + Qyz * y + Qzz * z;
    const double rqr = qx * x + qy * y + qz * z;
    const double trq = Qxx + Qyy + Qzz;
    // Lam_0: M D0 + (1/6) Q:D2, with Q:D2 = 3 RQR s^5 - tr(Q) s^3
    lam[0] += M * s + (3.0 * rqr * s5 - trq * s3) / 6.0;
    // Lam_1: M D1 + (1/6) Q:D3, with (Q:D3)_a = -15 R_a RQR s^7 + 3 (2 (QR)_a + R_a tr Q) s^5
    const double k7 = -15.0 * rqr * s7, k5 = 3.0 * trq * s5;
    lam[1] += -M * x * s3 + (x * k7 + 6.0 * qx * s5 + x * k5) / 6.0;
    lam[2] += -M * y * s3 + (y * k7 + 6.0 * qy * s5 + y * k5) / 6.0;
    lam[3] += -M * z * s3 + (z * k7 + 6.0 * qz * s5 + z * k5) / 6.0;
    // Lam_2 = M D2: 3 R_a R_b s^5 - delta_ab s^3
    const double m5 = 3.0 * M * s5, m3 = M * s3;
    lam[4] += m5 * x * x - m3;
    lam[5] += m5 * y * y - m3;
    lam[6] += m5 * z * z - m3;
    lam[7] += m5 * x * y;
    lam[8] += m5 * x * z;
    lam[9] += m5 * y * z;
    // Lam_3 = M D3: -15 R_a R_b R_c s^7 + 3 (delta_ab R_c + delta_ac R_b + delta_bc R_a) s^5
    const double m7 = -15.0 * M * s7;
    lam[10] += m7 * x * x * x + 3.0 * m5 * x;
    lam[11] += m7 * y * y * y + 3.0 * m5 * y;
    lam[12] += m7 * z * z * z + 3.0 * m5 * z;
    lam[13] += m7 * x * x * y + m5 * y;
    lam[14] += m7 * x * x * z + m5 * z;
    lam[15] += m7 * x * y * y + m5 * x;
    lam[16] += m7 * y * y * z + m5 * z;
    lam[17] += m7 * x * z * z + m5 * x;
    lam[18] += m7 * y * z * z + m5 * y;
    lam[19] += m7 * x * y * z;
}

// Full-tensor views of the packed coefficients.
__device__ __forceinline__ double t2(const double* lam, int a, int b) {
    if (a == b) return lam[4 + a];
    const int s = a + b;   // (0,1) -> xy, (0,2) -> xz, (1,2) -> yz
    return lam[s == 1 ? 7 : s == 2 ? 8 : 9];
}

__device__ __forceinline__ double t3(const double* lam, int a, int b, int c) {
    int n[3] = {0, 0, 0};
    ++n[a];
    ++n[b];
    ++n[c];
    if (n[0] == 3) return lam[10];
    if (n[1] == 3) return lam[11];
    if (n[2] == 3) return lam[12];
    if (n[0] == 2) return n[1] == 1 ? lam[13] : lam[14];
    if (n[1] == 2) return n[0] == 1 ? lam[15] : lam[16];
    if (n[2] == 2) return n[0] == 1 ? lam[17] : lam[18];
    return lam[19];
}

// (acc / G, -pot / G) of an expansion at offset dl: g_a = Lam1_a + Lam2_ab dl_b
// + (1/2) Lam3_abc dl_b dl_c and p = Lam0 + Lam1.dl + (1/2) dl.Lam2.dl +
// (1/6) Lam3[dl, dl, dl].
__device__ __forceinline__ void l2p(const double* lam, const double* dl, double* g, double& p) {
    p = lam[0];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double ga = lam[1 + a];
        p += lam[1 + a] * dl[a];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            ga += t2(lam, a, b) * dl[b];
            p += 0.5 * t2(lam, a, b) * dl[a] * dl[b];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                ga += 0.5 * t3(lam, a, b, c) * dl[b] * dl[c];
                p += t3(lam, a, b, c) * dl[a] * dl[b] * dl[c] / 6.0;
            }
        }
        g[a] = ga;
    }
}

// M2L: one wave per target cell; lane k takes the target's sorted sources
// k, k + 64, ...; the lanes' sums are added by a fixed butterfly.
// Overwrites lam.
__global__ void __launch_bounds__(256) k_fmm_m2l(const Moments* __restrict__ mom, const FmmGeo* __restrict__ geo,
                                                 const DevParams* __restrict__ prm, int64_t cmax,
                                                 const uint64_t* __restrict__ keys, const uint32_t* __restrict__ off,
                                                 double eps2, double* __restrict__ lam_out) {
    int64_t C = prm->ncells;
    if (C > cmax) C = cmax;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t t = blockIdx.x * (int64_t)(blockDim.x / kWave) + (threadIdx.x / kWave); t < C; t += nwaves) {
        double lam[kNL];
#pragma unroll
        for (int k = 0; k < kNL; ++k) lam[k] = 0.0;
        const FmmGeo g = geo[t];
        for (uint32_t q = off[t] + lane; q < off[t + 1]; q += kWave) {
            const uint32_t b = (uint32_t)(keys[q] >> 32);
            const Moments& mb = mom[b];
            m2l_add(mb.M, mb.Q, g.z[0] - mb.com[0], g.z[1] - mb.com[1], g.z[2] - mb.com[2], eps2, lam);
        }
#pragma unroll
        for (int k = 0; k < kNL; ++k) {
            double v = lam[k];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
            lam[k] = v;
        }
        if (lane < kNL) {
            double v = lam[0];
#pragma unroll
            for (int k = 1; k < kNL; ++k)
                if (lane == k) v = lam[k];
            lam_out[t * kNL + lane] = v;
        }
    }
}

// L2L for the cells of one level (level-order range [lo, hi)): each adds its
// parent's expansion moved to its own centre.
__global__ void __launch_bounds__(256) k_fmm_l2l(const Cell* __restrict__ cells, const FmmGeo* __restrict__ geo,
                                                 const uint32_t* __restrict__ bfs2pre,
                                                 const uint32_t* __restrict__ lvl_off, int level,
                                                 double* __restrict__ lam) {
    const int64_t lo = lvl_off[level], hi = lvl_off[level + 1];
    for (int64_t k = lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < hi;
         k += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t c = bfs2pre[k];
        const int32_t p = cells[c].parent;
        if (p < 0) continue;
        double P[kNL];
#pragma unroll
        for (int j = 0; j < kNL; ++j) P[j] = lam[(int64_t)p * kNL + j];
        double t[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) t[a] = geo[c].z[a] - geo[p].z[a];
        double* out = lam + (int64_t)c * kNL;
        // Lam'_0 and Lam'_1 are the potential and its gradient at t
        double g[3], p0;
        l2p(P, t, g, p0);
        out[0] += p0;
        out[1] += g[0];
        out[2] += g[1];
        out[3] += g[2];
        // Lam'_2 = Lam2 + Lam3 . t
        const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            double v = P[4 + j];
#pragma unroll
            for (int c3 = 0; c3 < 3; ++c3) v += t3(P, ia[j], ib[j], c3) * t[c3];
            out[4 + j] += v;
        }
#pragma unroll
        for (int j = 10; j < kNL; ++j) out[j] += P[j];
    }
}

constexpr int kFmmList = 256;
constexpr int kFmmWaves = 4;

// A target leaf whose partner list is longer than kFmmChunk leaves is cut
// into chunks of kFmmChunk partners, one task each, so that no single wave
// carries a far-spread leaf's whole direct sum; the chunks' sums go to
// partial slots and k_fmm_leaf_finish adds them in chunk order.
constexpr uint32_t kFmmChunk = 256;

// Tasks per cell (leaves: chunks of the partner list; other cells: none)
// and partial slots (chunks x bodies, for leaves cut into several chunks).
__global__ void __launch_bounds__(256) k_fmm_tasks_count(const Cell* __restrict__ cells,
                                                         const uint32_t* __restrict__ poff,
                                                         const DevParams* __restrict__ prm, int64_t cmax,
                                                         uint32_t* __restrict__ ntask, uint32_t* __restrict__ nslot) {
    int64_t C = prm->ncells;
    if (C > cmax) C = cmax;
    for (int64_t A = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; A < C; A += (int64_t)gridDim.x * blockDim.x) {
        const Cell ca = cells[A];
        uint32_t nt = 0, ns = 0;
        if (is_leaf(ca)) {
            const uint32_t np = poff[A + 1] - poff[A];
            nt = np > kFmmChunk ? (np + kFmmChunk - 1) / kFmmChunk : 1u;
            ns = nt > 1 ? nt * (uint32_t)ca.count : 0u;
        }
        ntask[A] = nt;
        nslot[A] = ns;
    }
}

__global__ void __launch_bounds__(256) k_fmm_tasks_fill(const uint32_t* __restrict__ toff,
                                                        const DevParams* __restrict__ prm, int64_t cmax,
                                                        uint32_t* __restrict__ task) {
    int64_t C = prm->ncells;
    if (C > cmax) C = cmax;
    for (int64_t A = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; A < C; A += (int64_t)gridDim.x * blockDim.x)
        for (uint32_t k = toff[A]; k < toff[A + 1]; ++k) task[k] = (uint32_t)A;
}

// L2P + P2P: one wave per task (a target leaf, or one chunk of a long
// leaf's partner list).  Lanes are (target body, slice):
// with nA target bodies, 64/P lanes per slice where P is the smallest power
// of two >= nA (at most 64), and slice k sums list entries k, k + S, ...
// (S slices); the slices' sums are added in FP64 in a fixed order.  The
// partner leaves' bodies are gathered 64 at a time: 64 partner cells are
// loaded together, their body counts scanned, and each lane finds its
// body's partner by a binary search over the scan.
__global__ void __launch_bounds__(256) k_fmm_leaf(const Cell* __restrict__ cells, const Body* __restrict__ bodies,
                                                  const float4* __restrict__ bodies32, const uint32_t* __restrict__ perm,
                                                  const FmmGeo* __restrict__ geo, const double* __restrict__ lam,
                                                  const uint64_t* __restrict__ pkeys, const uint32_t* __restrict__ poff,
                                                  const uint32_t* __restrict__ task, const uint32_t* __restrict__ toff,
                                                  const uint32_t* __restrict__ soff, int64_t ntasks, double* __restrict__ part,
                                                  float G, float eps2, float* __restrict__ acc, float* __restrict__ pot) {
    __shared__ float4 s_list[kFmmWaves][kFmmList];
    __shared__ uint32_t s_off[kFmmWaves][kWave];
    __shared__ int32_t s_beg[kFmmWaves][kWave];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    float4* L = s_list[wv];
    uint32_t* SO = s_off[wv];
    int32_t* SB = s_beg[wv];
    const int64_t nwaves = (int64_t)gridDim.x * kFmmWaves;
    for (int64_t tk = blockIdx.x * (int64_t)kFmmWaves + wv; tk < ntasks; tk += nwaves) {
        const uint32_t A = task[tk];
        const uint32_t chunk = (uint32_t)tk - toff[A], nchunks = toff[A + 1] - toff[A];
        const Cell ca = cells[A];
        const FmmGeo ga = geo[A];
        const uint32_t q0 = poff[A] + chunk * kFmmChunk;
        const uint32_t q1 = nchunks > 1 ? min(poff[A + 1], q0 + kFmmChunk) : poff[A + 1];
        for (int t0 = 0; t0 < ca.count; t0 += kWave) {
            const int nA = min(kWave, ca.count - t0);
            int P = 1;
            while (P < nA) P <<= 1;
            const int S = kWave / P;              // slices
            const int t = lane & (P - 1), sl = lane / P;
            const bool tv = t < nA;
            const int64_t i = (int64_t)ca.begin + t0 + (tv ? t : 0);
            const Body me = bodies[i];
            // the far field first: the leaf's expansion at the body (a leaf
            // cut into chunks gets it in k_fmm_leaf_finish)
            double g[3] = {0.0, 0.0, 0.0}, p = 0.0;
            if (sl == 0 && tv && nchunks == 1) {
                double lamA[kNL];
                for (int k = 0; k < kNL; ++k) lamA[k] = lam[A * kNL + k];
                const double dl[3] = {me.x - ga.z[0], me.y - ga.z[1], me.z - ga.z[2]};
                l2p(lamA, dl, g, p);
            }
            const float xi = (float)(me.x - ga.z[0]), yi = (float)(me.y - ga.z[1]), zi = (float)(me.z - ga.z[2]);
            float sx = 0.f, sy = 0.f, sz = 0.f, sp = 0.f, cx = 0.f, cy = 0.f, cz = 0.f, cp = 0.f;
            int len = 0;
            auto flush = [&](int cnt) {
                wave_lds_sync();
                for (int e = 0; e < cnt; e += kWave) {
                    const int lim = min(cnt, e + kWave);
                    float ax = 0.f, ay = 0.f, az = 0.f, ap = 0.f;
                    for (int k = e + sl; k < lim; k += S) {
                        const float4 q = L[k];
                        const float dx = q.x - xi, dy = q.y - yi, dz = q.z - zi;
                        const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
                        const float s = __builtin_amdgcn_rsqf(r2);
                        const float ms = q.w * s;
                        const float ms3 = ms * (s * s);
                        ap -= ms;
                        ax = fmaf(ms3, dx, ax);
                        ay = fmaf(ms3, dy, ay);
                        az = fmaf(ms3, dz, az);
                    }
                    comp_add(sx, cx, ax);
                    comp_add(sy, cy, ay);
                    comp_add(sz, cz, az);
                    comp_add(sp, cp, ap);
                }
                wave_lds_sync();
            };
            for (uint32_t qb = q0; qb < q1; qb += kWave) {
                const int nq = (int)min((uint32_t)kWave, q1 - qb);
                int32_t pb = 0;
                uint32_t pc = 0;
                if (lane < nq) {
                    const Cell cb = cells[(uint32_t)(pkeys[qb + lane] >> 32)];
                    pb = cb.begin;
                    pc = (uint32_t)cb.count;
                }
                uint32_t incl = pc;
#pragma unroll
                for (int o = 1; o < kWave; o <<= 1) {
                    const uint32_t y = __shfl_up(incl, o, kWave);
                    if (lane >= o) incl += y;
                }
                const uint32_t total = __shfl(incl, kWave - 1, kWave);
                SO[lane] = incl - pc;              // first slot of partner `lane`
                SB[lane] = pb;
                wave_lds_sync();
                for (uint32_t base = 0; base < total; base += kWave) {
                    const int m = (int)min((uint32_t)kWave, total - base);
                    if (len + m > kFmmList) {
                        flush(len);
                        len = 0;
                    }
                    if (lane < m) {
                        const uint32_t slot = base + lane;
                        int lo = 0, hi = nq - 1;          // last partner whose first slot <= slot
                        while (lo < hi) {
                            const int mid = (lo + hi + 1) >> 1;
                            if (SO[mid] <= slot) lo = mid;
                            else hi = mid - 1;
                        }
                        const int64_t j = (int64_t)SB[lo] + (slot - SO[lo]);
                        float4 e;
                        if (bodies32) {
                            const float4 b = bodies32[j];
                            e = make_float4((float)((double)b.x - ga.z[0]), (float)((double)b.y - ga.z[1]),
                                            (float)((double)b.z - ga.z[2]), b.w);
                        } else {
                            const Body b = bodies[j];
                            e = make_float4((float)(b.x - ga.z[0]), (float)(b.y - ga.z[1]), (float)(b.z - ga.z[2]),
                                            (float)b.m);
                        }
                        L[len + lane] = e;
                    }
                    len += m;
                }
                wave_lds_sync();
            }
            flush(len);
            // slices' sums in FP64, in slice order
            double v[4] = {(double)sx + (double)cx, (double)sy + (double)cy, (double)sz + (double)cz,
                           (double)sp + (double)cp};
            for (int o = P; o < kWave; o <<= 1) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const double w = __shfl_down(v[k], o, kWave);
                    if ((lane & o) == 0) v[k] += w;
                }
            }
            if (sl == 0 && tv && nchunks > 1) {
                double* o = part + 4 * ((int64_t)soff[A] + (int64_t)chunk * ca.count + t0 + t);
                o[0] = v[0];
                o[1] = v[1];
                o[2] = v[2];
                o[3] = v[3];
            } else if (sl == 0 && tv) {
                // the body met itself in its own leaf: no force, a -m/eps
                // potential term removed as it was formed
                const float mself = (float)me.m;
                const double self = (double)(mself * __builtin_amdgcn_rsqf(eps2));
                const int64_t o = perm[i];
                acc[o * 3 + 0] = (float)((double)G * (g[0] + v[0]));
                acc[o * 3 + 1] = (float)((double)G * (g[1] + v[1]));
                acc[o * 3 + 2] = (float)((double)G * (g[2] + v[2]));
                pot[o] = (float)((double)G * (-p + v[3] + self));
            }
        }
    }
}

// Bodies of the leaves cut into chunks: the chunks' sums in chunk order,
// the leaf's expansion and the self term, as in k_fmm_leaf.  One wave per
// cell, lanes over its bodies.
__global__ void __launch_bounds__(256) k_fmm_leaf_finish(const Cell* __restrict__ cells, const Body* __restrict__ bodies,
                                                         const uint32_t* __restrict__ perm,
                                                         const FmmGeo* __restrict__ geo, const double* __restrict__ lam,
                                                         const uint32_t* __restrict__ toff,
                                                         const uint32_t* __restrict__ soff,
                                                         const double* __restrict__ part,
                                                         const DevParams* __restrict__ prm, int64_t cmax, float G,
                                                         float eps2, float* __restrict__ acc, float* __restrict__ pot) {
    int64_t C = prm->ncells;
    if (C > cmax) C = cmax;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t A = blockIdx.x * (int64_t)(blockDim.x / kWave) + (threadIdx.x / kWave); A < C; A += nwaves) {
        const uint32_t nchunks = toff[A + 1] - toff[A];
        if (nchunks < 2) continue;
        const Cell ca = cells[A];
        const FmmGeo ga = geo[A];
        for (int t = lane; t < ca.count; t += kWave) {
            const int64_t i = (int64_t)ca.begin + t;
            const Body me = bodies[i];
            double v[4] = {0.0, 0.0, 0.0, 0.0};
            for (uint32_t j = 0; j < nchunks; ++j) {
                const double* q = part + 4 * ((int64_t)soff[A] + (int64_t)j * ca.count + t);
                v[0] += q[0];
                v[1] += q[1];
                v[2] += q[2];
                v[3] += q[3];
            }
            double lamA[kNL];
            for (int k = 0; k < kNL; ++k) lamA[k] = lam[A * kNL + k];
            const double dl[3] = {me.x - ga.z[0], me.y - ga.z[1], me.z - ga.z[2]};
            double g[3], p;
            l2p(lamA, dl, g, p);
            const float mself = (float)me.m;
            const double self = (double)(mself * __builtin_amdgcn_rsqf(eps2));
            const int64_t o = perm[i];
            acc[o * 3 + 0] = (float)((double)G * (g[0] + v[0]));
            acc[o * 3 + 1] = (float)((double)G * (g[1] + v[1]));
            acc[o * 3 + 2] = (float)((double)G * (g[2] + v[2]));
            pot[o] = (float)((double)G * (-p + v[3] + self));
        }
    }
}

// Pairs as (target, source) pre-order indices.
__global__ void __launch_bounds__(256) k_fmm_unpack(const uint64_t* __restrict__ keys, int64_t n,
                                                    int32_t* __restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        out[2 * i] = (int32_t)(uint32_t)keys[i];
        out[2 * i + 1] = (int32_t)(keys[i] >> 32);
    }
}

__global__ void __launch_bounds__(256) k_fill_u32(uint32_t* __restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

}  // namespace

hipError_t launch_fmm_geo(const Cell* cells, const Moments* mom, const WalkCell* walk, const uint32_t* pre2bfs,
                          const DevParams* prm, int64_t cmax, FmmGeo* geo, DttCell* dc, hipStream_t s) {
    hipLaunchKernelGGL(k_fmm_geo, dim3(grid_for(cmax)), dim3(256), 0, s, cells, mom, walk, pre2bfs, prm, cmax, geo,
                       dc);
    return hipGetLastError();
}

hipError_t launch_fmm_radii(const Cell* cells, const Moments* mom, const Body* bodies, const WalkCell* walk,
                            const uint32_t* bfs2pre, const uint32_t* lvl_off, int level, int64_t count, FmmGeo* geo,
                            DttCell* dc, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fmm_radii, dim3(grid_for(count)), dim3(256), 0, s, cells, mom, bodies, walk, bfs2pre, lvl_off,
                       level, geo, dc);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_fmm_dtt(const DttCell* dc, double theta, const uint64_t* fin, int64_t nin, uint64_t* fout,
                          int64_t capf, uint64_t* m2l, int64_t capm, uint64_t* p2p, int64_t capp,
                          unsigned long long* ctr, uint32_t* bt, unsigned long long* base, hipStream_t s) {
    if (nin <= 0) return hipSuccess;
    const unsigned nb = grid_for(nin, kFmmMaxBlocks);
    hipLaunchKernelGGL(k_fmm_dtt_count, dim3(nb), dim3(kDttBlock), 0, s, dc, theta, fin, nin, bt);
    hipLaunchKernelGGL(k_fmm_dtt_scan, dim3(1), dim3(1024), 0, s, (const uint32_t*)bt, (int)nb, ctr, base);
    hipLaunchKernelGGL(k_fmm_dtt_write, dim3(nb), dim3(kDttBlock), 0, s, dc, theta, fin, nin,
                       (const unsigned long long*)base, fout, capf, m2l, capm, p2p, capp);
    return hipGetLastError();
}

hipError_t launch_fmm_offsets(const uint64_t* keys, int64_t n, int64_t C, uint32_t* off, hipStream_t s) {
    hipLaunchKernelGGL(k_fmm_offsets, dim3(grid_for(C + 1)), dim3(256), 0, s, keys, n, C, off);
    return hipGetLastError();
}

hipError_t launch_fmm_m2l(const Moments* mom, const FmmGeo* geo, const DevParams* prm, int64_t cmax,
                          const uint64_t* keys, const uint32_t* off, double eps2, double* lam,
                          hipStream_t s) {
    int64_t blocks = (cmax + 3) / 4;   // one wave per cell
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fmm_m2l, dim3((unsigned)blocks), dim3(256), 0, s, mom, geo, prm, cmax, keys, off, eps2,
                       lam);
    return hipGetLastError();
}

hipError_t launch_fmm_l2l(const Cell* cells, const FmmGeo* geo, const uint32_t* bfs2pre, const uint32_t* lvl_off,
                          int level, int64_t count, double* lam, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fmm_l2l, dim3(grid_for(count)), dim3(256), 0, s, cells, geo, bfs2pre, lvl_off, level, lam);
    return hipGetLastError();
}

hipError_t launch_fmm_tasks(const Cell* cells, const uint32_t* poff, const DevParams* prm, int64_t cmax,
                            uint32_t* ntask, uint32_t* nslot, hipStream_t s) {
    hipLaunchKernelGGL(k_fmm_tasks_count, dim3(grid_for(cmax)), dim3(256), 0, s, cells, poff, prm, cmax, ntask, nslot);
    return hipGetLastError();
}

hipError_t launch_fmm_tasks_fill(const uint32_t* toff, const DevParams* prm, int64_t cmax, uint32_t* task,
                                 hipStream_t s) {
    hipLaunchKernelGGL(k_fmm_tasks_fill, dim3(grid_for(cmax)), dim3(256), 0, s, toff, prm, cmax, task);
    return hipGetLastError();
}

hipError_t launch_fmm_leaf(const Cell* cells, const Body* bodies, const float4* bodies32, const uint32_t* perm,
                           const FmmGeo* geo, const double* lam, const uint64_t* pkeys, const uint32_t* poff,
                           const uint32_t* task, const uint32_t* toff, const uint32_t* soff, int64_t ntasks,
                           double* part, const DevParams* prm, int64_t cmax, float G, float eps2, float* acc,
                           float* pot, hipStream_t s) {
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (ntasks > 0) {
        int64_t blocks = (ntasks + kFmmWaves - 1) / kFmmWaves;
        const int64_t cap = (int64_t)ncu * 16;
        if (blocks > cap) blocks = cap;
        hipLaunchKernelGGL(k_fmm_leaf, dim3((unsigned)blocks), dim3(256), 0, s, cells, bodies, bodies32, perm, geo,
                           lam, pkeys, poff, task, toff, soff, ntasks, part, G, eps2, acc, pot);
    }
    int64_t fb = (cmax + 3) / 4;
    if (fb > 65536) fb = 65536;
    hipLaunchKernelGGL(k_fmm_leaf_finish, dim3((unsigned)fb), dim3(256), 0, s, cells, bodies, perm, geo, lam, toff,
                       soff, (const double*)part, prm, cmax, G, eps2, acc, pot);
    return hipGetLastError();
}

hipError_t launch_fmm_unpack(const uint64_t* keys, int64_t n, int32_t* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fmm_unpack, dim3(grid_for(n)), dim3(256), 0, s, keys, n, out);
    return hipGetLastError();
}

}  // namespace tc
