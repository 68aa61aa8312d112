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
//     / theta, with rho_A = (sqrt 3 / 2) s_A and rho_B = (sqrt 3 / 2) s_B +
//     |com_B - z_B| bounding their bodies; two leaves that are not sum
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
// The pairs are sorted by (target, source) cell index before use, so every
// sum runs in a fixed order and the results do not depend on the order the
// traversal found the pairs in.
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
                                                 const DevParams* __restrict__ prm, int64_t cmax,
                                                 FmmGeo* __restrict__ geo) {
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
        g.rhoA = kHalfSqrt3 * s;
        g.rhoB = kHalfSqrt3 * s + sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
        g.pad[0] = g.pad[1] = g.pad[2] = 0.0;
        geo[k] = g;
    }
}

// Reserve n slots of a counter for this lane, one atomic per wave.  Every
// lane of the wave must call it (n = 0 for lanes with nothing to write).
__device__ __forceinline__ uint64_t wave_reserve(unsigned long long* ctr, uint32_t n) {
    const int lane = threadIdx.x & (kWave - 1);
    uint32_t x = n;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    const uint32_t total = __shfl(x, kWave - 1, kWave);
    unsigned long long base = 0;
    if (lane == kWave - 1 && total) base = atomicAdd(ctr, (unsigned long long)total);
    base = __shfl(base, kWave - 1, kWave);
    return base + x - n;
}

__device__ __forceinline__ uint64_t pair_key(uint32_t a, uint32_t b) { return ((uint64_t)a << 32) | b; }

// One level of the traversal: every input pair becomes an M2L pair, a P2P
// pair, or pairs of the next level.  Counters: [0] next level, [1] M2L,
// [2] P2P; a slot at or beyond a capacity is counted but not written.
__global__ void __launch_bounds__(256) k_fmm_dtt(const Cell* __restrict__ cells, const Moments* __restrict__ mom,
                                                 const FmmGeo* __restrict__ geo, double theta,
                                                 const uint64_t* __restrict__ fin, int64_t nin,
                                                 uint64_t* __restrict__ fout, int64_t capf,
                                                 uint64_t* __restrict__ m2l, int64_t capm,
                                                 uint64_t* __restrict__ p2p, int64_t capp,
                                                 unsigned long long* __restrict__ ctr,
                                                 uint32_t* __restrict__ m2l_per, uint32_t* __restrict__ p2p_per) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t iters = (nin + stride - 1) / stride;   // the same for every lane
    for (int64_t it = 0; it < iters; ++it) {
        const int64_t i = it * stride + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
        const bool valid = i < nin;
        uint32_t A = 0, B = 0;
        if (valid) {
            const uint64_t pr = fin[i];
            A = (uint32_t)(pr >> 32);
            B = (uint32_t)pr;
        }
        // 0: nothing, 1: M2L, 2: P2P, 3: children of A x children of A,
        // 4: children of A x B, 5: A x children of B
        int kind = 0;
        Cell ca, cb;
        if (valid) {
            ca = cells[A];
            if (A == B) {
                kind = is_leaf(ca) ? 2 : 3;
            } else {
                bool acc = false;
                if (theta != 0.0) {
                    const FmmGeo ga = geo[A], gb = geo[B];
                    double d[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) d[a] = ga.z[a] - mom[B].com[a];
                    const double d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
                    const double r = (ga.rhoA + gb.rhoB) / theta;
                    acc = d2 > r * r;
                }
                if (acc) {
                    kind = 1;
                } else {
                    cb = cells[B];
                    if (is_leaf(ca) && is_leaf(cb)) kind = 2;
                    else if (!is_leaf(ca) && (is_leaf(cb) || ca.level <= cb.level)) kind = 4;
                    else kind = 5;
                }
            }
        }
        const int na = (kind >= 3 && kind <= 4) ? nchildren(ca) : 0;
        const int nb = kind == 5 ? nchildren(cb) : 0;
        const uint32_t nnext = kind == 3 ? (uint32_t)(na * na) : kind == 4 ? (uint32_t)na : (uint32_t)nb;
        const uint64_t om = wave_reserve(&ctr[1], kind == 1 ? 1u : 0u);
        const uint64_t op = wave_reserve(&ctr[2], kind == 2 ? 1u : 0u);
        const uint64_t on = wave_reserve(&ctr[0], nnext);
        if (kind == 1) {
            if ((int64_t)om < capm) m2l[om] = pair_key(A, B);
            atomicAdd(&m2l_per[A], 1u);
        } else if (kind == 2) {
            if ((int64_t)op < capp) p2p[op] = pair_key(A, B);
            atomicAdd(&p2p_per[A], 1u);
        } else if (kind == 3) {
            uint32_t ch[8];
            uint32_t c = A + 1;
            for (int j = 0; j < na && j < 8; ++j) {
                ch[j] = c;
                c = (uint32_t)cells[c].skip;
            }
            uint64_t o = on;
            for (int x = 0; x < na && x < 8; ++x)
                for (int y = 0; y < na && y < 8; ++y, ++o)
                    if ((int64_t)o < capf) fout[o] = pair_key(ch[x], ch[y]);
        } else if (kind == 4) {
            uint32_t c = A + 1;
            for (int j = 0; j < na; ++j) {
                if ((int64_t)(on + j) < capf) fout[on + j] = pair_key(c, B);
                c = (uint32_t)cells[c].skip;
            }
        } else if (kind == 5) {
            uint32_t c = B + 1;
            for (int j = 0; j < nb; ++j) {
                if ((int64_t)(on + j) < capf) fout[on + j] = pair_key(A, c);
                c = (uint32_t)cells[c].skip;
            }
        }
    }
}

// Pack (target, source) into a key of 2*bits bits for the radix sort.
__global__ void __launch_bounds__(256) k_fmm_pack(uint64_t* __restrict__ keys, uint32_t* __restrict__ idx, int64_t n,
                                                  int bits) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = keys[i];
        keys[i] = ((k >> 32) << bits) | (k & 0xffffffffull);
        idx[i] = (uint32_t)i;
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

// M2L: one thread per target cell over its sorted sources; overwrites lam.
__global__ void __launch_bounds__(256) k_fmm_m2l(const Moments* __restrict__ mom, const FmmGeo* __restrict__ geo,
                                                 const DevParams* __restrict__ prm, int64_t cmax,
                                                 const uint64_t* __restrict__ keys, const uint32_t* __restrict__ off,
                                                 int bits, double eps2, double* __restrict__ lam_out) {
    int64_t C = prm->ncells;
    if (C > cmax) C = cmax;
    const uint64_t mask = ((uint64_t)1 << bits) - 1;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < C; t += (int64_t)gridDim.x * blockDim.x) {
        double lam[kNL];
#pragma unroll
        for (int k = 0; k < kNL; ++k) lam[k] = 0.0;
        const FmmGeo g = geo[t];
        for (uint32_t q = off[t]; q < off[t + 1]; ++q) {
            const uint32_t b = (uint32_t)(keys[q] & mask);
            const Moments& mb = mom[b];
            m2l_add(mb.M, mb.Q, g.z[0] - mb.com[0], g.z[1] - mb.com[1], g.z[2] - mb.com[2], eps2, lam);
        }
#pragma unroll
        for (int k = 0; k < kNL; ++k) lam_out[t * kNL + k] = lam[k];
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

// L2P + P2P: one wave per target leaf.  Lanes are (target body, slice):
// with nA target bodies, 64/P lanes per slice where P is the smallest power
// of two >= nA (at most 64), and slice k sums list entries k, k + S, ...
// (S slices); the slices' sums are added in FP64 in a fixed order.
__global__ void __launch_bounds__(256) k_fmm_leaf(const Cell* __restrict__ cells, const Body* __restrict__ bodies,
                                                  const float4* __restrict__ bodies32, const uint32_t* __restrict__ perm,
                                                  const FmmGeo* __restrict__ geo, const double* __restrict__ lam,
                                                  const uint64_t* __restrict__ pkeys, const uint32_t* __restrict__ poff,
                                                  int bits, const DevParams* __restrict__ prm, int64_t cmax, float G,
                                                  float eps2, float* __restrict__ acc, float* __restrict__ pot) {
    __shared__ float4 s_list[kFmmWaves][kFmmList];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    float4* L = s_list[wv];
    int64_t C = prm->ncells;
    if (C > cmax) C = cmax;
    const uint64_t mask = ((uint64_t)1 << bits) - 1;
    const int64_t nwaves = (int64_t)gridDim.x * kFmmWaves;
    for (int64_t A = blockIdx.x * (int64_t)kFmmWaves + wv; A < C; A += nwaves) {
        const Cell ca = cells[A];
        if (!is_leaf(ca)) continue;
        const FmmGeo ga = geo[A];
        const uint32_t q0 = poff[A], q1 = poff[A + 1];
        for (int t0 = 0; t0 < ca.count; t0 += kWave) {
            const int nA = min(kWave, ca.count - t0);
            int P = 1;
            while (P < nA) P <<= 1;
            const int S = kWave / P;              // slices
            const int t = lane & (P - 1), sl = lane / P;
            const bool tv = t < nA;
            const int64_t i = (int64_t)ca.begin + t0 + (tv ? t : 0);
            const Body me = bodies[i];
            const float xi = (float)(me.x - ga.z[0]), yi = (float)(me.y - ga.z[1]), zi = (float)(me.z - ga.z[2]);
            float sx = 0.f, sy = 0.f, sz = 0.f, sp = 0.f, cx = 0.f, cy = 0.f, cz = 0.f, cp = 0.f;
            int len = 0;
            auto flush = [&](int cnt) {
                wave_lds_sync();
                for (int e = 0; e < cnt; e += kWave) {
                    const int lim = min(cnt, e + kWave);
                    float ax = 0.f, ay = 0.f, az = 0.f, ap = 0.f;
                    for (int k = e + sl; k < lim; k += S) {
                        const float4 p = L[k];
                        const float dx = p.x - xi, dy = p.y - yi, dz = p.z - zi;
                        const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
                        const float s = __builtin_amdgcn_rsqf(r2);
                        const float ms = p.w * s;
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
            for (uint32_t q = q0; q < q1; ++q) {
                const Cell cb = cells[(uint32_t)(pkeys[q] & mask)];
                for (int o = 0; o < cb.count; o += kWave) {
                    const int m = min(kWave, cb.count - o);
                    if (len + m > kFmmList) {
                        flush(len);
                        len = 0;
                    }
                    if (lane < m) {
                        const int64_t j = (int64_t)cb.begin + o + lane;
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
            if (sl == 0 && tv) {
                double lamA[kNL];
#pragma unroll
                for (int k = 0; k < kNL; ++k) lamA[k] = lam[A * kNL + k];
                const double dl[3] = {me.x - ga.z[0], me.y - ga.z[1], me.z - ga.z[2]};
                double g[3], p;
                l2p(lamA, dl, g, p);
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

// Pairs as (target, source) pre-order indices.
__global__ void __launch_bounds__(256) k_fmm_unpack(const uint64_t* __restrict__ keys, int64_t n, int bits,
                                                    int32_t* __restrict__ out) {
    const uint64_t mask = ((uint64_t)1 << bits) - 1;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        out[2 * i] = (int32_t)(keys[i] >> bits);
        out[2 * i + 1] = (int32_t)(keys[i] & mask);
    }
}

__global__ void __launch_bounds__(256) k_fill_u32(uint32_t* __restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

}  // namespace

hipError_t launch_fmm_geo(const Cell* cells, const Moments* mom, const DevParams* prm, int64_t cmax, FmmGeo* geo,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_fmm_geo, dim3(grid_for(cmax)), dim3(256), 0, s, cells, mom, prm, cmax, geo);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_fmm_dtt(const Cell* cells, const Moments* mom, const FmmGeo* geo, double theta,
                          const uint64_t* fin, int64_t nin, uint64_t* fout, int64_t capf, uint64_t* m2l, int64_t capm,
                          uint64_t* p2p, int64_t capp, unsigned long long* ctr, uint32_t* m2l_per, uint32_t* p2p_per,
                          hipStream_t s) {
    if (nin <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fmm_dtt, dim3(grid_for(nin, 8192)), dim3(256), 0, s, cells, mom, geo, theta, fin, nin, fout,
                       capf, m2l, capm, p2p, capp, ctr, m2l_per, p2p_per);
    return hipGetLastError();
}

hipError_t launch_fmm_pack(uint64_t* keys, uint32_t* idx, int64_t n, int bits, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fmm_pack, dim3(grid_for(n)), dim3(256), 0, s, keys, idx, n, bits);
    return hipGetLastError();
}

hipError_t launch_fmm_m2l(const Moments* mom, const FmmGeo* geo, const DevParams* prm, int64_t cmax,
                          const uint64_t* keys, const uint32_t* off, int bits, double eps2, double* lam,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_fmm_m2l, dim3(grid_for(cmax)), dim3(256), 0, s, mom, geo, prm, cmax, keys, off, bits, eps2,
                       lam);
    return hipGetLastError();
}

hipError_t launch_fmm_l2l(const Cell* cells, const FmmGeo* geo, const uint32_t* bfs2pre, const uint32_t* lvl_off,
                          int level, int64_t count, double* lam, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fmm_l2l, dim3(grid_for(count)), dim3(256), 0, s, cells, geo, bfs2pre, lvl_off, level, lam);
    return hipGetLastError();
}

hipError_t launch_fmm_leaf(const Cell* cells, const Body* bodies, const float4* bodies32, const uint32_t* perm,
                           const FmmGeo* geo, const double* lam, const uint64_t* pkeys, const uint32_t* poff,
                           int bits, const DevParams* prm, int64_t cmax, float G, float eps2, float* acc, float* pot,
                           hipStream_t s) {
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    int64_t blocks = (cmax + kFmmWaves - 1) / kFmmWaves;
    const int64_t cap = (int64_t)ncu * 16;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_fmm_leaf, dim3((unsigned)blocks), dim3(256), 0, s, cells, bodies, bodies32, perm, geo, lam,
                       pkeys, poff, bits, prm, cmax, G, eps2, acc, pot);
    return hipGetLastError();
}

hipError_t launch_fmm_unpack(const uint64_t* keys, int64_t n, int bits, int32_t* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fmm_unpack, dim3(grid_for(n)), dim3(256), 0, s, keys, n, bits, out);
    return hipGetLastError();
}

}  // namespace tc
