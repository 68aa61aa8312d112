// Learned closure of the treecode: training data, the network, training.
//
// The paper's treecode represents an accepted cell by its monopole (§3.1).
// The closure adds, for a body x and an accepted cell c (centre of mass C,
// mass M, side s, traceless quadrupole Q), a correction predicted by a small
// network from features of the pair:
//   f = [(x - C)/s (3), Q/(M s^2) (6), ln(M/mbar) (1)],  mbar = total mass / n,
//   yhat = MLP(f) (3),  a += G [ a_mono + (M s^2/|x - C|^4) yhat ].
// The training target is the residual in units of the quadrupole scale
//   y = (a_exact - a_mono) |x - C|^4 / (M s^2)   (G = 1),
// where a_exact sums the cell's bodies directly.  The network is
// 10-64-64-3 with GELU (tanh form); its products run on BF16 matrix-core
// instructions with FP32 accumulation (training: 16x16x16 tiles through
// LDS; inference: net_tile in closure.h) with FP32 master weights, trained
// by mean squared error and Adam.
//
// This file: residual generation (one wave per target body; the walk is the
// batched level-order walk of the force kernel with the box shrunk to the
// body), the network's forward and backward passes, the Adam update.
#include "tc_internal.h"
#include "closure.h"

#include <math.h>

namespace tc {

namespace {

// ------------------------------------------------------------ residuals ----

constexpr int kStack = 320;                       // range stack per wave (bound as in force.hip)

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Walk for one body (the box shrunk to a point) at the prepared opening
// radii; on_accept(b) runs with the whole wave for every accepted cell, b
// its level-order index.  3D.
template <typename F>
__device__ void walk_point(const WalkCell* __restrict__ walk, uint32_t* S, double px, double py, double pz,
                           F&& on_accept) {
    constexpr int R = 8, RP = kWave / R;
    constexpr int kReserve = (R - 1) * 21 + R;
    static_assert(kStack >= kWave + kReserve + kWave, "stack bound");
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    if (lane == 0) S[0] = 0u;
    wave_lds_sync();
    int top = 1;
    while (top > 0) {
        const int nr = (top + kWave + kReserve <= kStack) ? min(top, RP) : 1;
        const int rr = lane / R, j = lane % R;
        uint32_t packed = 0;
        if (rr < nr) packed = S[top - 1 - rr];
        top -= nr;
        const int rlen = (int)(packed & 7u) + 1;
        const bool vc = rr < nr && j < rlen;
        const uint32_t b = (packed >> 3) + (uint32_t)j;
        wave_lds_sync();
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
        const double dx = wc.cx - px, dy = wc.cy - py, dz = wc.cz - pz;
        const double d2 = (dx * dx + dy * dy) + dz * dz;
        const bool leaf = vc && wc.b < 0;
        const bool accept = vc && d2 > wc.rcrit2;
        const bool opened = vc && !accept && !leaf;
        const uint64_t O = __ballot(opened);
        if (opened) S[top + __popcll(O & below)] = ((uint32_t)wc.a << 3) | (uint32_t)(wc.b - 1);
        top += __popcll(O);
        wave_lds_sync();
        uint64_t A = __ballot(accept);
        while (A) {
            const int l = __builtin_ctzll(A);
            A &= A - 1;
            on_accept((uint32_t)__builtin_amdgcn_readlane((int)b, l));
        }
    }
}

// count pass: pairs per target; write pass: the pairs at the scanned offsets
template <bool WRITE>
__global__ void __launch_bounds__(256) k_residuals(const WalkCell* __restrict__ walk, const Body* __restrict__ bodies,
                                                   const Cell* __restrict__ cells, const Moments* __restrict__ mom,
                                                   const uint32_t* __restrict__ bfs2pre,
                                                   const uint32_t* __restrict__ inv_perm,
                                                   DevParams* __restrict__ prm, int64_t n,
                                                   const int32_t* __restrict__ targets, int nt, double eps2,
                                                   uint32_t* __restrict__ counts, const uint32_t* __restrict__ offs,
                                                   int64_t cap, float* __restrict__ feat, float* __restrict__ yout,
                                                   int32_t* __restrict__ cell_out) {
    __shared__ uint32_t s_stack[4][kStack];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    const int t = blockIdx.x * 4 + wv;
    if (t >= nt) return;
    const int64_t o = targets[t];
    if (o < 0 || o >= n) {                     // no pairs for an index outside the bodies
        if (lane == 0) {
            atomicOr(&prm->status, kFlagBadIndex);
            if (!WRITE) counts[t] = 0u;
        }
        return;
    }
    const int64_t p = inv_perm[o];
    const Body me = bodies[p];
    const double mbar = mom[0].M / (double)n;
    const double size = prm->size;
    int64_t k = WRITE ? (int64_t)offs[t] : 0;
    walk_point(walk, s_stack[wv], me.x, me.y, me.z, [&](uint32_t b) {
        if (WRITE && k < cap) {
            const int64_t kc = bfs2pre[b];
            const Cell c = cells[kc];
            const Moments& mo = mom[kc];
            // exact softened sum over the cell's bodies, FP64, fixed order
            double ex = 0.0, ey = 0.0, ez = 0.0;
            for (int64_t j = c.begin + lane; j < (int64_t)c.begin + c.count; j += kWave) {
                const Body q = bodies[j];
                const double dx = q.x - me.x, dy = q.y - me.y, dz = q.z - me.z;
                const double r2 = ((eps2 + dx * dx) + dy * dy) + dz * dz;
                const double inv = 1.0 / sqrt(r2);
                const double w3 = q.m * inv * inv * inv;
                ex += w3 * dx;
                ey += w3 * dy;
                ez += w3 * dz;
            }
            ex = wsum(ex);
            ey = wsum(ey);
            ez = wsum(ez);
            if (lane == 0) {
                const double M = mo.M;
                const double dcx = mo.com[0] - me.x, dcy = mo.com[1] - me.y, dcz = mo.com[2] - me.z;
                const double d2 = (dcx * dcx + dcy * dcy) + dcz * dcz;
                const double inv = 1.0 / sqrt(d2 + eps2);
                const double w3 = M * inv * inv * inv;
                const double s = ldexp(size, -c.level);
                // residual in units of the quadrupole scale M s^2 / d^4
                const double nrm = (d2 * d2) / (M * s * s);
                float* y = yout + k * 3;
                y[0] = (float)((ex - w3 * dcx) * nrm);
                y[1] = (float)((ey - w3 * dcy) * nrm);
                y[2] = (float)((ez - w3 * dcz) * nrm);
                float* f = feat + k * 10;
                f[0] = (float)((me.x - mo.com[0]) / s);
                f[1] = (float)((me.y - mo.com[1]) / s);
                f[2] = (float)((me.z - mo.com[2]) / s);
                const double qs = M * s * s;
                for (int q = 0; q < 6; ++q) f[3 + q] = (float)(mo.Q[q] / qs);
                f[9] = (float)log(M / mbar);
                cell_out[k] = (int32_t)kc;
            }
        }
        ++k;
    });
    if (!WRITE && lane == 0) counts[t] = (uint32_t)k;
}

__global__ void k_inverse_perm(const uint32_t* __restrict__ perm, int64_t n, uint32_t* __restrict__ inv) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        inv[perm[i]] = (uint32_t)i;
}

// --------------------------------------------------------------- network ----

__device__ __forceinline__ uint16_t f2bf(float f) {        // round to nearest, ties to even
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}

__device__ __forceinline__ float gelu(float z) { return gelu_f(z); }

__device__ __forceinline__ float gelu_grad(float z) { return gelu_grad_f(z); }

// One 16x16 output tile of a product of BF16 matrices held in LDS:
//   D(i, j) = sum_k A(i0 + i, k) B(k, j0 + j),  k < K (a multiple of 16),
// with A(i, k) = A[i*sai + k*sak] and B(k, j) = B[k*sbk + j*sbj].  Lane l
// supplies A rows l%16, columns 4(l/16)..+3 of each 16-wide k step and the
// matching B entries, and receives D rows 4(l/16)+q, column l%16 (q < 4).
__device__ __forceinline__ float4_t mm_tile(const uint16_t* A, int sai, int sak, int i0, const uint16_t* B, int sbk,
                                            int sbj, int j0, int K) {
    const int l = threadIdx.x & (kWave - 1);
    const int r = l & 15, kq = 4 * (l >> 4);
    float4_t acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        short4_t a, b;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            a[q] = (short)A[(i0 + r) * sai + (k0 + kq + q) * sak];
            b[q] = (short)B[(k0 + kq + q) * sbk + (j0 + r) * sbj];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    return acc;
}

struct NetLds {
    uint16_t w1[16 * kNHid], w2[kNHid * kNHid], w3[kNHid * 16];
    float b1[kNHid], b2[kNHid], b3[16];
    uint16_t x[kMlpBlock * 16], h1[kMlpBlock * kNHid], h2[kMlpBlock * kNHid];
    float z1[kMlpBlock * kNHid], z2[kMlpBlock * kNHid];
    float yh[kMlpBlock * 16];
};

__device__ void load_net(const MlpState* __restrict__ st, NetLds& L) {
    const int l = threadIdx.x;
    for (int i = l; i < 16 * kNHid; i += kWave) L.w1[i] = st->w1[i];
    for (int i = l; i < kNHid * kNHid; i += kWave) L.w2[i] = st->w2[i];
    for (int i = l; i < kNHid * 16; i += kWave) L.w3[i] = st->w3[i];
    L.b1[l] = st->b1[l];
    L.b2[l] = st->b2[l];
    if (l < 16) L.b3[l] = st->b3[l];
}

// Forward pass for the 64 samples whose BF16 features sit in L.x.
__device__ void net_forward(NetLds& L) {
    const int l = threadIdx.x & (kWave - 1);
    const int col = l & 15, rq = 4 * (l >> 4);
    for (int rt = 0; rt < 4; ++rt)
        for (int ct = 0; ct < 4; ++ct) {
            const float4_t d = mm_tile(L.x, 16, 1, 16 * rt, L.w1, kNHid, 1, 16 * ct, 16);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 16 * rt + rq + q, c = 16 * ct + col;
                const float z = d[q] + L.b1[c];
                L.z1[row * kNHid + c] = z;
                L.h1[row * kNHid + c] = f2bf(gelu(z));
            }
        }
    __syncthreads();
    for (int rt = 0; rt < 4; ++rt)
        for (int ct = 0; ct < 4; ++ct) {
            const float4_t d = mm_tile(L.h1, kNHid, 1, 16 * rt, L.w2, kNHid, 1, 16 * ct, kNHid);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 16 * rt + rq + q, c = 16 * ct + col;
                const float z = d[q] + L.b2[c];
                L.z2[row * kNHid + c] = z;
                L.h2[row * kNHid + c] = f2bf(gelu(z));
            }
        }
    __syncthreads();
    for (int rt = 0; rt < 4; ++rt) {
        const float4_t d = mm_tile(L.h2, kNHid, 1, 16 * rt, L.w3, 16, 1, 0, kNHid);
#pragma unroll
        for (int q = 0; q < 4; ++q) L.yh[(16 * rt + rq + q) * 16 + col] = d[q] + L.b3[col];
    }
    __syncthreads();
}

__device__ void load_features(const float* __restrict__ feat, int64_t nrows, const int32_t* __restrict__ idx,
                              int64_t nb, int64_t s0, NetLds& L, int64_t& src, bool& valid, uint32_t* status) {
    const int l = threadIdx.x;
    const int64_t s = s0 + l;
    valid = s < nb;
    src = valid ? (idx ? (int64_t)idx[s] : s) : 0;
    if (valid && (src < 0 || src >= nrows)) {  // a row outside feat: left out, flagged
        atomicOr(status, kFlagBadIndex);
        valid = false;
        src = 0;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) L.x[l * 16 + q] = (valid && q < kNIn) ? f2bf(feat[src * kNIn + q]) : (uint16_t)0;
}

// Inference on rows of stored features, with the matrix-core routine of
// the learned walk (net_tile): one wave per 64 samples, 16 at a time.
__global__ void __launch_bounds__(256) k_mlp_forward(const float* __restrict__ feat, int64_t nrows,
                                                     const int32_t* __restrict__ idx, int64_t nb,
                                                     const MlpState* __restrict__ st, float* __restrict__ yhat,
                                                     uint32_t* status) {
    __shared__ NetF N;
    load_net_frags(st, N, threadIdx.x, blockDim.x);
    __syncthreads();
    const int wv = threadIdx.x >> 6, l = threadIdx.x & (kWave - 1), g = l >> 4, r = l & 15;
    const int64_t s0 = ((int64_t)blockIdx.x * 4 + wv) * kWave;
    if (s0 >= nb) return;
    for (int tile = 0; tile < 4; ++tile) {
        const int64_t s = s0 + 16 * tile + r;
        bool valid = s < nb;
        int64_t src = valid ? (idx ? (int64_t)idx[s] : s) : 0;
        if (valid && (src < 0 || src >= nrows)) {  // a row outside feat: left out, flagged
            atomicOr(status, kFlagBadIndex);
            valid = false;
            src = 0;
        }
        short4_t x;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 4 * g + j;
            x[j] = (valid && k < kNIn) ? bf16_bits(feat[src * kNIn + k]) : (short)0;
        }
        const float4_t y = net_tile(N, x);
        if (g == 0 && valid)
            for (int q = 0; q < kNOut; ++q) yhat[s * kNOut + q] = y[q];
    }
}

// One training block: forward, squared error, backward for 64 samples;
// writes this block's gradient sums (canonical order) and squared error.
__global__ void __launch_bounds__(64) k_mlp_train(const float* __restrict__ feat, const float* __restrict__ ytrue,
                                                  int64_t nrows, const int32_t* __restrict__ idx, int64_t nb,
                                                  MlpState* __restrict__ st, uint32_t* status) {
    __shared__ NetLds L;
    __shared__ uint16_t dy[kMlpBlock * 16], dz2[kMlpBlock * kNHid], dz1[kMlpBlock * kNHid];
    load_net(st, L);
    int64_t src;
    bool valid;
    const int64_t s0 = (int64_t)blockIdx.x * kMlpBlock;
    load_features(feat, nrows, idx, nb, s0, L, src, valid, status);
    __syncthreads();
    net_forward(L);
    const int l = threadIdx.x;
    const int col = l & 15, rq = 4 * (l >> 4);
    float* part = st->partials[blockIdx.x];
    // loss gradient, one lane per sample
    const float scale = 2.0f / (float)(nb * kNOut);
    float se = 0.f;
    float dyf[kNOut];
#pragma unroll
    for (int q = 0; q < kNOut; ++q) {
        const float d = valid ? L.yh[l * 16 + q] - ytrue[src * kNOut + q] : 0.f;
        se += d * d;
        dyf[q] = d * scale;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) dy[l * 16 + q] = q < kNOut ? f2bf(dyf[q]) : (uint16_t)0;
    __syncthreads();
    // b3 and the squared error: column sums over the 64 samples, fixed order
    L.yh[l * 16 + 0] = dyf[0];
    L.yh[l * 16 + 1] = dyf[1];
    L.yh[l * 16 + 2] = dyf[2];
    L.yh[l * 16 + 3] = se;
    __syncthreads();
    if (l < kNOut + 1) {
        float acc = 0.f;
        for (int s = 0; s < kMlpBlock; ++s) acc += L.yh[s * 16 + l];
        part[l < kNOut ? kOffB3 + l : kNParam] = acc;
    }
    // dW3 = h2^T dy  [64 x 3]
    for (int rt = 0; rt < 4; ++rt) {
        const float4_t d = mm_tile(L.h2, 1, kNHid, 16 * rt, dy, 16, 1, 0, kMlpBlock);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (col < kNOut) part[kOffW3 + (16 * rt + rq + q) * kNOut + col] = d[q];
    }
    // dz2 = (dy W3^T) * gelu'(z2)  [64 samples x 64]
    for (int rt = 0; rt < 4; ++rt)
        for (int ct = 0; ct < 4; ++ct) {
            const float4_t d = mm_tile(dy, 16, 1, 16 * rt, L.w3, 1, 16, 16 * ct, 16);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 16 * rt + rq + q, c = 16 * ct + col;
                const float g = d[q] * gelu_grad(L.z2[row * kNHid + c]);
                L.z2[row * kNHid + c] = g;                 // z2 now holds dz2 (FP32)
                dz2[row * kNHid + c] = f2bf(g);
            }
        }
    __syncthreads();
    {   // b2: column sums of dz2
        float acc = 0.f;
        for (int s = 0; s < kMlpBlock; ++s) acc += L.z2[s * kNHid + l];
        part[kOffB2 + l] = acc;
    }
    // dW2 = h1^T dz2  [64 x 64]
    for (int rt = 0; rt < 4; ++rt)
        for (int ct = 0; ct < 4; ++ct) {
            const float4_t d = mm_tile(L.h1, 1, kNHid, 16 * rt, dz2, kNHid, 1, 16 * ct, kMlpBlock);
#pragma unroll
            for (int q = 0; q < 4; ++q) part[kOffW2 + (16 * rt + rq + q) * kNHid + 16 * ct + col] = d[q];
        }
    // dz1 = (dz2 W2^T) * gelu'(z1)
    for (int rt = 0; rt < 4; ++rt)
        for (int ct = 0; ct < 4; ++ct) {
            const float4_t d = mm_tile(dz2, kNHid, 1, 16 * rt, L.w2, 1, kNHid, 16 * ct, kNHid);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 16 * rt + rq + q, c = 16 * ct + col;
                const float g = d[q] * gelu_grad(L.z1[row * kNHid + c]);
                L.z1[row * kNHid + c] = g;                 // z1 now holds dz1 (FP32)
                dz1[row * kNHid + c] = f2bf(g);
            }
        }
    __syncthreads();
    {   // b1
        float acc = 0.f;
        for (int s = 0; s < kMlpBlock; ++s) acc += L.z1[s * kNHid + l];
        part[kOffB1 + l] = acc;
    }
    // dW1 = x^T dz1  [16 (10 used) x 64]
    for (int ct = 0; ct < 4; ++ct) {
        const float4_t d = mm_tile(L.x, 1, 16, 0, dz1, kNHid, 1, 16 * ct, kMlpBlock);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (rq + q < kNIn) part[kOffW1 + (rq + q) * kNHid + 16 * ct + col] = d[q];
    }
}

// Refresh the padded BF16 weights and the biases from the FP32 masters.
__device__ void refresh_copy(MlpState* st, int p) {
    const float w = st->master[p];
    if (p < kOffB1) {
        st->w1[(p / kNHid) * kNHid + p % kNHid] = f2bf(w);
    } else if (p < kOffW2) {
        st->b1[p - kOffB1] = w;
    } else if (p < kOffB2) {
        st->w2[p - kOffW2] = f2bf(w);
    } else if (p < kOffW3) {
        st->b2[p - kOffB2] = w;
    } else if (p < kOffB3) {
        const int q = p - kOffW3;
        st->w3[(q / kNOut) * 16 + q % kNOut] = f2bf(w);
    } else {
        st->b3[p - kOffB3] = w;
    }
}

// Sum the blocks' gradients in block order, then one Adam step on the
// masters (step counts from 1) and a refresh of the BF16 copies.
__global__ void __launch_bounds__(256) k_mlp_adam(MlpState* __restrict__ st, int nblocks, int64_t nb, float lr,
                                                  int step, float* __restrict__ grad_out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kNParam) return;
    float g = 0.f;
    for (int b = 0; b < nblocks; ++b) g += st->partials[b][p];
    if (p == kNParam) {
        st->loss = g / (float)(nb * kNOut);
        return;
    }
    if (grad_out) grad_out[p] = g;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float m = b1 * st->m[p] + (1.f - b1) * g;
    const float v = b2 * st->v[p] + (1.f - b2) * g * g;
    st->m[p] = m;
    st->v[p] = v;
    const float mh = m / (1.f - powf(b1, (float)step));
    const float vh = v / (1.f - powf(b2, (float)step));
    st->master[p] = st->master[p] - lr * mh / (sqrtf(vh) + eps);
    refresh_copy(st, p);
}

__global__ void __launch_bounds__(256) k_mlp_load(MlpState* __restrict__ st, const float* __restrict__ params) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) st->loss = 0.f;
    if (p >= kNParam) return;
    st->master[p] = params[p];
    st->m[p] = 0.f;
    st->v[p] = 0.f;
    refresh_copy(st, p);
    // padding of the BF16 tiles and b3
    if (p < (16 - kNIn) * kNHid) st->w1[kNIn * kNHid + p] = 0;
    if (p < kNHid * 16) {
        const int c = p % 16;
        if (c >= kNOut) st->w3[p] = 0;
    }
    if (p < 16 - kNOut) st->b3[kNOut + p] = 0.f;
}

__global__ void __launch_bounds__(256) k_mlp_get(const MlpState* __restrict__ st, float* __restrict__ params) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kNParam) params[p] = st->master[p];
}

}  // namespace

// ------------------------------------------------------------ launchers ----

hipError_t launch_inverse_perm(const uint32_t* perm, int64_t n, uint32_t* inv, hipStream_t s) {
    hipLaunchKernelGGL(k_inverse_perm, dim3(grid_for(n)), dim3(256), 0, s, perm, n, inv);
    return hipGetLastError();
}

hipError_t launch_residuals(bool write, const WalkCell* walk, const Body* bodies, const Cell* cells,
                            const Moments* mom, const uint32_t* bfs2pre, const uint32_t* inv_perm,
                            DevParams* prm, int64_t n, const int32_t* targets, int nt, double eps2,
                            uint32_t* counts, const uint32_t* offs, int64_t cap, float* feat, float* y,
                            int32_t* cell_out, hipStream_t s) {
    const unsigned nb = (unsigned)((nt + 3) / 4);
    if (write)
        hipLaunchKernelGGL(k_residuals<true>, dim3(nb), dim3(256), 0, s, walk, bodies, cells, mom, bfs2pre, inv_perm,
                           prm, n, targets, nt, eps2, counts, offs, cap, feat, y, cell_out);
    else
        hipLaunchKernelGGL(k_residuals<false>, dim3(nb), dim3(256), 0, s, walk, bodies, cells, mom, bfs2pre, inv_perm,
                           prm, n, targets, nt, eps2, counts, offs, cap, feat, y, cell_out);
    return hipGetLastError();
}

hipError_t launch_mlp_load(MlpState* st, const float* params, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_load, dim3((kNParam + 255) / 256), dim3(256), 0, s, st, params);
    return hipGetLastError();
}

hipError_t launch_mlp_get(const MlpState* st, float* params, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_get, dim3((kNParam + 255) / 256), dim3(256), 0, s, st, params);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const MlpState* st, const float* feat, int64_t nrows, const int32_t* idx, int64_t nb,
                              float* yhat, uint32_t* status, hipStream_t s) {
    const unsigned blocks = (unsigned)((nb + 4 * kWave - 1) / (4 * kWave));
    hipLaunchKernelGGL(k_mlp_forward, dim3(blocks), dim3(256), 0, s, feat, nrows, idx, nb, st, yhat, status);
    return hipGetLastError();
}

hipError_t launch_mlp_step(MlpState* st, const float* feat, const float* y, int64_t nrows, const int32_t* idx,
                           int64_t nb, float lr, int step, float* grad_out, uint32_t* status, hipStream_t s) {
    const int blocks = (int)((nb + kMlpBlock - 1) / kMlpBlock);
    hipLaunchKernelGGL(k_mlp_train, dim3(blocks), dim3(kMlpBlock), 0, s, feat, y, nrows, idx, nb, st, status);
    hipLaunchKernelGGL(k_mlp_adam, dim3((kNParam + 1 + 255) / 256), dim3(256), 0, s, st, blocks, nb, lr, step,
                       grad_out);
    return hipGetLastError();
}

}  // namespace tc
