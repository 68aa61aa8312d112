// Tree construction and cell moments (§3.1 of the paper: recursive 4-/8-way
// subdivision until a subspace holds at most leaf_cap bodies; each cell is
// its bodies' total mass at their centre of mass).
//
// Pipeline, one stream, no host synchronisation:
//   bbox     root cube: per-axis minimum corner, power-of-two side (FP64);
//            the same pass packs the input as (x, y, z, m) records
//   keys     Morton key of FP64-quantised coordinates, index iota
//   sort     stable LSD radix sort of (key, index), 8 bits per pass (large
//            sorts rank each tile in LDS before writing it out)
//   gather   bodies into key order, FP64, one packed record per body
//   topology all cells at once from the sorted keys (no per-level launches):
//            body i starts the cells of levels a_i..l*_i, where a_i is one
//            more than its common-prefix length with body i-1 and l*_i is
//            one below the deepest level at which a run of leaf_cap+1
//            consecutive keys around i still shares a prefix; their
//            exclusive scan is the depth-first pre-order index; the level
//            order is one more radix pass, keyed by level, and the walk
//            groups one more scan
//   moments  FP64, leaves over bodies in order (one launch), then internal
//            cells level by level from the deepest up, each over its
//            children in digit order read from level-order copies (the top
//            and the deepest levels each in one single-block launch)
//   mac      opening radius per cell for the current theta
//
// Every expression that decides an integer (keys, topology, opening radii)
// is compiled without floating-point contraction.
#include "tc_internal.h"

#include <math.h>

namespace tc {
namespace {

__device__ __forceinline__ int wave_lane() { return threadIdx.x & (kWave - 1); }

// ---------------------------------------------------------------- bbox ----

// The input's bodies packed four values to a record, (x, y, z, m) with z = 0
// in 2D, in the input's order: the gather then reads one record per body
// instead of a position and a mass from two places.
template <typename T> struct Packed;
template <> struct Packed<float> { using type = float4; };
template <> struct Packed<double> { using type = double4; };

template <typename T, int D>
__global__ void __launch_bounds__(256) k_bbox_part(const T* __restrict__ pos, const T* __restrict__ mass,
                                                   int64_t n, double* __restrict__ part,
                                                   typename Packed<T>::type* __restrict__ packed) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        T c[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int a = 0; a < D; ++a) {
            c[a] = pos[i * D + a];
            const double v = (double)c[a];
            if (!isfinite(v)) { bad = 1; continue; }
            lo[a] = fmin(lo[a], v);
            hi[a] = fmax(hi[a], v);
        }
        const T mt = mass[i];
        const double m = (double)mt;
        if (!(isfinite(m) && m > 0.0)) bad = 1;
        typename Packed<T>::type r;
        r.x = c[0];
        r.y = c[1];
        r.z = c[2];
        r.w = mt;
        packed[i] = r;
    }
    __shared__ double s_lo[3][256], s_hi[3][256];
    __shared__ int s_bad[256];
    const int t = threadIdx.x;
#pragma unroll
    for (int a = 0; a < 3; ++a) { s_lo[a][t] = lo[a]; s_hi[a][t] = hi[a]; }
    s_bad[t] = bad;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                s_lo[a][t] = fmin(s_lo[a][t], s_lo[a][t + w]);
                s_hi[a][t] = fmax(s_hi[a][t], s_hi[a][t + w]);
            }
            s_bad[t] |= s_bad[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        double* o = part + blockIdx.x * 7;
        for (int a = 0; a < 3; ++a) { o[a] = s_lo[a][0]; o[3 + a] = s_hi[a][0]; }
        o[6] = (double)s_bad[0];
    }
}

__global__ void __launch_bounds__(256) k_bbox_final(const double* __restrict__ part, int nb, int dim,
                                                    DevParams* prm) {
    __shared__ double s_lo[3][256], s_hi[3][256];
    __shared__ int s_bad[256];
    const int t = threadIdx.x;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int bad = 0;
    for (int b = t; b < nb; b += 256) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = fmin(lo[a], part[b * 7 + a]);
            hi[a] = fmax(hi[a], part[b * 7 + 3 + a]);
        }
        bad |= part[b * 7 + 6] != 0.0;
    }
    for (int a = 0; a < 3; ++a) { s_lo[a][t] = lo[a]; s_hi[a][t] = hi[a]; }
    s_bad[t] = bad;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            for (int a = 0; a < 3; ++a) {
                s_lo[a][t] = fmin(s_lo[a][t], s_lo[a][t + w]);
                s_hi[a][t] = fmax(s_hi[a][t], s_hi[a][t + w]);
            }
            s_bad[t] |= s_bad[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        const int L = dim == 3 ? 21 : 31;
        double ext = 0.0;
        for (int a = 0; a < dim; ++a) {
            double l = s_lo[a][0];
            if (!isfinite(l)) l = 0.0;            // no finite coordinate on this axis
            prm->lo[a] = l;
            const double e = s_hi[a][0] - s_lo[a][0];
            if (e > ext) ext = e;
        }
        for (int a = dim; a < 3; ++a) prm->lo[a] = 0.0;
        double size = 1.0;
        if (ext > 0.0 && isfinite(ext)) {
            int e2;
            const double f = frexp(ext, &e2);     // ext = f 2^e2, f in [0.5, 1)
            size = (f == 0.5) ? ext : ldexp(1.0, e2);
        }
        int e2;
        frexp(size, &e2);                         // size = 2^(e2-1)
        prm->size = size;
        prm->scale = ldexp(1.0, L - (e2 - 1));
        prm->status = s_bad[0] ? kFlagNonFinite : 0u;
        prm->ncells = 0;
    }
}

// ---------------------------------------------------------------- keys ----

__device__ __forceinline__ uint64_t spread3(uint64_t x) {   // bit b -> bit 3b (21 bits)
    x &= 0x1fffffull;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}

__device__ __forceinline__ uint64_t spread2(uint64_t x) {   // bit b -> bit 2b (32 bits)
    x &= 0xffffffffull;
    x = (x | x << 16) & 0x0000ffff0000ffffull;
    x = (x | x << 8) & 0x00ff00ff00ff00ffull;
    x = (x | x << 4) & 0x0f0f0f0f0f0f0f0full;
    x = (x | x << 2) & 0x3333333333333333ull;
    x = (x | x << 1) & 0x5555555555555555ull;
    return x;
}

template <int D>
__device__ __forceinline__ uint64_t quantise(double x, double lo, double scale) {
    constexpr int L = D == 3 ? 21 : 31;
    const double top = (double)((1ull << L) - 1ull);
    double f = floor((x - lo) * scale);
    if (!(f >= 0.0)) f = 0.0;                     // also catches NaN
    if (f > top) f = top;
    return (uint64_t)f;
}

template <typename T, int D>
__global__ void __launch_bounds__(256) k_keys(const T* __restrict__ pos, int64_t n,
                                              const DevParams* __restrict__ prm,
                                              uint64_t* __restrict__ keys, uint32_t* __restrict__ idx) {
    const double scale = prm->scale;
    const double lo0 = prm->lo[0], lo1 = prm->lo[1], lo2 = prm->lo[2];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t key;
        if (D == 3) {
            const uint64_t qx = quantise<3>((double)pos[i * 3 + 0], lo0, scale);
            const uint64_t qy = quantise<3>((double)pos[i * 3 + 1], lo1, scale);
            const uint64_t qz = quantise<3>((double)pos[i * 3 + 2], lo2, scale);
            key = (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
        } else {
            const uint64_t qx = quantise<2>((double)pos[i * 2 + 0], lo0, scale);
            const uint64_t qy = quantise<2>((double)pos[i * 2 + 1], lo1, scale);
            key = (spread2(qx) << 1) | spread2(qy);
        }
        keys[i] = key;
        idx[i] = (uint32_t)i;
    }
}

// ---------------------------------------------------------------- sort ----
// Reduce-then-scan LSD radix sort: per tile digit counts, a scan of the
// counts in digit-major order, then a stable scatter in which each wave
// ranks its keys with ballot-based digit matching.  The scatter loads all
// of a thread's keys before ranking any (one block per tile leaves few
// waves per CU, and a load per round of 256 keys waited on memory round
// after round: 20.2 us per pass of 1M keys, 16.0 us with the loads first).
// Recording every round's per-wave digit counts and placing all keys after
// one prefix pass (three barriers per tile instead of three per round) took
// 18.4 us.  Copies of the running places (two) and counts (three) let a
// round place its keys while the next round's places are advanced and a
// later round's counts cleared: one barrier per round instead of three
// (1M keys: 0.191 against 0.201 ms per sort; 16.7M: 1.57 against 1.64).
// PER keys per thread, tiles of 256 PER keys (sort_per).
// Placing each key straight at its output place writes about one key per
// digit per round of 256, so a line of the output is written in many
// pieces; large sorts (STAGE, from kSortStageMin keys) first rank the whole
// tile into LDS in output order and then write each digit's run with
// consecutive threads (16.7M keys: 2.36 to 1.64 ms for the eight passes,
// 4M: 0.56 to 0.46; 1M keys, whose passes stay in the caches, 0.20 to 0.22,
// so smaller sorts do not stage; the same at 1.5M).
//
// Where a pass's pairs come from and go to.  A plain pass reads keys and
// values (nullable) and writes both at their places.  The level pass sorts
// the cells by level (pre-order within a level, so the children of a cell
// stay adjacent): it reads each cell's level as its key and its pre-order
// index as its value, writes the level order both ways, and the first tile
// writes where each level starts (its digit bases: no tile precedes it).
struct PairsIn {
    const uint64_t* __restrict__ k;
    const uint32_t* __restrict__ v;
    __device__ uint64_t key(int64_t i) const { return k[i]; }
    __device__ uint32_t val(int64_t i) const { return v ? v[i] : 0u; }
};
struct PairsOut {
    uint64_t* __restrict__ k;
    uint32_t* __restrict__ v;
    __device__ void put(uint32_t p, uint64_t key, uint32_t val) const {
        k[p] = key;
        if (v) v[p] = val;
    }
    __device__ void starts(int, uint32_t) const {}
};
struct LevelsIn {
    const Cell* __restrict__ cells;
    __device__ uint64_t key(int64_t i) const { return (uint64_t)cells[i].level; }
    __device__ uint32_t val(int64_t i) const { return (uint32_t)i; }
};
struct LevelsOut {
    uint32_t* __restrict__ bfs2pre;
    uint32_t* __restrict__ pre2bfs;
    uint32_t* __restrict__ lvl_off;   // levels 0..L and the end
    int L;
    __device__ void put(uint32_t p, uint64_t, uint32_t val) const {
        bfs2pre[p] = val;
        pre2bfs[val] = p;
    }
    __device__ void starts(int d, uint32_t base) const {
        if (d <= L + 1) lvl_off[d] = base;
    }
};

// Tiles of `tile` keys that hold the first n keys (at least one, so that
// the first tile always writes the digit starts).
__device__ __forceinline__ int64_t live_tiles(int64_t n, int64_t tile) {
    return n > 0 ? (n + tile - 1) / tile : 1;
}

template <int PER, class In>
// n_live (nullable, device): sort only the first min(n, *n_live) keys; the
// tiles past them (a pass over the cells is sized for the most cells a tree
// can have) count, scan and scatter nothing.
__global__ void __launch_bounds__(256) k_sort_hist(In in, int64_t n, const uint32_t* __restrict__ n_live, int shift,
                                                   uint32_t* __restrict__ hist, int64_t tiles) {
    if (n_live && (int64_t)*n_live < n) n = *n_live;
    const int64_t tile = blockIdx.x;
    if (tile >= live_tiles(n, 256 * PER)) return;   // nothing reads the counts of later tiles
    __shared__ uint32_t cnt[4][256];
    const int t = threadIdx.x, w = t >> 6;
    for (int a = 0; a < 4; ++a) cnt[a][t] = 0;
    __syncthreads();
    const int64_t base = tile * (256 * PER);
#pragma unroll 4
    for (int j = 0; j < PER; ++j) {
        const int64_t i = base + j * 256 + t;
        if (i < n) atomicAdd(&cnt[w][(unsigned)(in.key(i) >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)t * tiles + tile] = cnt[0][t] + cnt[1][t] + cnt[2][t] + cnt[3][t];
}

// Exclusive block scan of one value per thread (256 threads); returns the
// prefix, writes the block total into *total (shared).
__device__ __forceinline__ uint32_t block_exscan_u32(uint32_t v, uint32_t* s_w, uint32_t* total) {
    const int lane = wave_lane(), w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) s_w[w] = x;
    __syncthreads();
    uint32_t wbase = 0;
    for (int k = 0; k < w; ++k) wbase += s_w[k];
    if (threadIdx.x == 255) *total = wbase + x;
    __syncthreads();
    return wbase + x - v;
}

template <int PER>
__global__ void __launch_bounds__(256) k_sort_scan(uint32_t* __restrict__ hist, int64_t tiles, int64_t n,
                                                   const uint32_t* __restrict__ n_live,
                                                   uint32_t* __restrict__ digit_tot) {
    __shared__ uint32_t s_w[4];
    __shared__ uint32_t s_tot;
    if (n_live && (int64_t)*n_live < n) n = *n_live;
    const int64_t tl = live_tiles(n, 256 * PER);
    uint32_t* h = hist + (int64_t)blockIdx.x * tiles;
    uint32_t carry = 0;
    for (int64_t c = 0; c < tl; c += 256) {
        const int64_t i = c + threadIdx.x;
        const uint32_t v = i < tl ? h[i] : 0u;
        const uint32_t ex = block_exscan_u32(v, s_w, &s_tot);
        if (i < tl) h[i] = carry + ex;
        carry += s_tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) digit_tot[blockIdx.x] = carry;
}

// SCAN: hist holds the raw per-tile counts (no k_sort_scan before it), and
// each block sums its digit's row itself: the earlier tiles' counts and the
// total, which block 0 also stores in digit_tot.  For a few tiles (at most
// kSortScanInScatter) this costs less than the scan's own launch.
constexpr int64_t kSortScanInScatter = 128;
// Sorts of at least kSortStageMin keys stage each tile in LDS (STAGE).
constexpr int64_t kSortStageMin = (int64_t)1 << 21;
constexpr int kSortStagePer = 16;

template <int PER, bool SCAN, bool STAGE, class In, class Out>
__global__ void __launch_bounds__(256) k_sort_scatter(In in, Out out, int64_t n, const uint32_t* __restrict__ n_live,
                                                      int shift, const uint32_t* __restrict__ hist,
                                                      uint32_t* __restrict__ digit_tot, int64_t tiles) {
    if (n_live && (int64_t)*n_live < n) n = *n_live;
    constexpr int kTile = 256 * PER;
    constexpr int kStage = STAGE ? kTile : 1;
    const int64_t tl = live_tiles(n, kTile);
    if ((int64_t)blockIdx.x >= tl) return;
    __shared__ uint32_t s_base[256];   // where the tile's keys of each digit start in the output
    // running place of each digit (staged: in the tile, else in the output)
    // in two copies, and each wave's count of each digit in a round in three:
    // round r reads place copy r % 2 and count copy r % 3, writes place copy
    // (r + 1) % 2 and clears count copy (r + 2) % 3, so one barrier per round
    // separates every write of a copy from its reads
    __shared__ uint32_t s_pos[2][256];
    __shared__ uint32_t s_lstart[256]; // staged: where each digit's keys start in the tile
    __shared__ uint32_t s_wcnt[3][4][256];
    __shared__ uint32_t s_w[4];
    __shared__ uint32_t s_tot;
    __shared__ uint64_t s_key[kStage];
    __shared__ uint32_t s_val[kStage];
    const int t = threadIdx.x, w = t >> 6, lane = wave_lane();
    const int64_t tile = blockIdx.x;
    uint32_t own = 0;   // this tile's count of digit t (staged only)
    if (SCAN) {
        const uint32_t* row = hist + (int64_t)t * tiles;
        uint32_t pre = 0, tot = 0;
#pragma unroll 8
        for (int64_t k = 0; k < tl; ++k) {
            const uint32_t v = row[k];
            tot += v;
            if (k < tile) pre += v;
        }
        if (tile == 0) digit_tot[t] = tot;
        if (STAGE) own = row[tile];
        s_base[t] = block_exscan_u32(tot, s_w, &s_tot) + pre;
    } else {
        const uint32_t tot = digit_tot[t];
        const uint32_t here = hist[(int64_t)t * tiles + tile];
        if (STAGE) own = (tile + 1 < tl ? hist[(int64_t)t * tiles + tile + 1] : tot) - here;
        s_base[t] = block_exscan_u32(tot, s_w, &s_tot) + here;
    }
    if (tile == 0) out.starts(t, s_base[t]);
    if (STAGE) {
        const uint32_t l = block_exscan_u32(own, s_w, &s_tot);
        s_lstart[t] = l;
        s_pos[0][t] = l;
    } else {
        s_pos[0][t] = s_base[t];
    }
    for (int a = 0; a < 4; ++a) s_wcnt[0][a][t] = s_wcnt[1][a][t] = 0;
    uint64_t kr[PER];
    uint32_t vr[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int64_t i = tile * kTile + r * 256 + t;
        kr[r] = i < n ? in.key(i) : 0ull;
        vr[r] = i < n ? in.val(i) : 0u;
    }
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const bool valid = tile * kTile + r * 256 + t < n;
        const uint64_t k = kr[r];
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const uint64_t before = peers & lt;
        const int cur = r & 1, nxt = cur ^ 1, cc = r % 3, cz = (r + 2) % 3;
        if (valid && before == 0) s_wcnt[cc][w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t p = s_pos[cur][d] + (uint32_t)__popcll(before);
            for (int a = 0; a < w; ++a) p += s_wcnt[cc][a][d];
            if (STAGE) {
                s_key[p] = k;
                s_val[p] = vr[r];
            } else {
                out.put(p, k, vr[r]);
            }
        }
        // the next round's places, advanced by this round's counts, and the
        // counts of the round after it cleared (last read by the previous round)
        s_pos[nxt][t] = s_pos[cur][t] + s_wcnt[cc][0][t] + s_wcnt[cc][1][t] + s_wcnt[cc][2][t] +
                        s_wcnt[cc][3][t];
        for (int a = 0; a < 4; ++a) s_wcnt[cz][a][t] = 0;
    }
    if (STAGE) {
        __syncthreads();
        // The tile's keys now sit in LDS in output order, digit by digit:
        // consecutive threads write consecutive places of a digit's run.
        const int64_t left = n - tile * kTile;
        const int live = left < kTile ? (int)left : kTile;
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int l = r * 256 + t;
            if (l < live) {
                const uint64_t k = s_key[l];
                const uint32_t d = (uint32_t)(k >> shift) & 255u;
                out.put(s_base[d] + (uint32_t)l - s_lstart[d], k, s_val[l]);
            }
        }
    }
}

// -------------------------------------------------------------- gather ----

template <typename T>
__global__ void __launch_bounds__(256) k_gather(const typename Packed<T>::type* __restrict__ packed,
                                                const uint32_t* __restrict__ perm, int64_t n,
                                                Body* __restrict__ bodies, float4* __restrict__ bodies32) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const typename Packed<T>::type r = packed[perm[i]];
        Body b;
        b.x = (double)r.x;
        b.y = (double)r.y;
        b.z = (double)r.z;
        b.m = (double)r.w;
        bodies[i] = b;
        // FP32 inputs also get a compact copy (exactly the input values)
        if (bodies32) bodies32[i] = make_float4((float)b.x, (float)b.y, (float)b.z, (float)b.m);
    }
}

// ---------------------------------------------------------------- scan ----
// Exclusive scan of u32 values: out[i] = sum_{j<i} in[j], out[n] = total.
// With n_live (device, nullable) only the first m = min(n, *n_live) values
// are read and written, and the total also goes to out[m]; the grids cover
// n.

__device__ __forceinline__ int64_t live_count(int64_t n, const uint32_t* n_live) {
    return (n_live && (int64_t)*n_live < n) ? (int64_t)*n_live : n;
}

__global__ void __launch_bounds__(256) k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                     const uint32_t* __restrict__ n_live,
                                                     uint32_t* __restrict__ part) {
    __shared__ uint32_t s_w[4];
    __shared__ uint32_t s_tot;
    n = live_count(n, n_live);
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    if (base >= n) {                       // the whole tile is past the live values
        if (threadIdx.x == 0) part[blockIdx.x] = 0u;
        return;
    }
    uint32_t s = 0;
    for (int j = 0; j < kScanTile / 256; ++j) {
        const int64_t i = base + j * 256 + threadIdx.x;
        if (i < n) s += in[i];
    }
    block_exscan_u32(s, s_w, &s_tot);
    if (threadIdx.x == 0) part[blockIdx.x] = s_tot;
}

// The tiles' sums in one block of 1024 threads, four consecutive tiles per
// thread, over the tiles that hold live values only.
__global__ void __launch_bounds__(1024) k_scan_part(uint32_t* __restrict__ part, int64_t tiles,
                                                    uint32_t* __restrict__ out, int64_t n,
                                                    const uint32_t* __restrict__ n_live) {
    __shared__ uint32_t s_w[16];
    const int64_t m = live_count(n, n_live);
    int64_t tl = (m + kScanTile - 1) / kScanTile;
    if (tl > tiles) tl = tiles;
    const int t = threadIdx.x, lane = wave_lane(), w = t >> 6;
    uint32_t carry = 0;
    for (int64_t c = 0; c < tl; c += 4 * 1024) {
        const int64_t i = c + 4 * t;
        const uint32_t v0 = i < tl ? part[i] : 0u, v1 = i + 1 < tl ? part[i + 1] : 0u;
        const uint32_t v2 = i + 2 < tl ? part[i + 2] : 0u, v3 = i + 3 < tl ? part[i + 3] : 0u;
        const uint32_t own = v0 + v1 + v2 + v3;
        uint32_t x = own;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, kWave);
            if (lane >= o) x += y;
        }
        if (lane == kWave - 1) s_w[w] = x;
        __syncthreads();
        uint32_t wbase = 0, tot = 0;
        for (int k = 0; k < 16; ++k) {
            if (k < w) wbase += s_w[k];
            tot += s_w[k];
        }
        uint32_t e = carry + wbase + x - own;
        if (i < tl) part[i] = e;
        e += v0;
        if (i + 1 < tl) part[i + 1] = e;
        e += v1;
        if (i + 2 < tl) part[i + 2] = e;
        e += v2;
        if (i + 3 < tl) part[i + 3] = e;
        carry += tot;
        __syncthreads();    // s_w is rewritten by the next round
    }
    if (t == 0) {
        out[n] = carry;
        out[m] = carry;
    }
}

// A tile is kScanTile / 1024 rows of 1024 values; thread t takes values
// 4t..4t+3 of each row (one 16-byte load and store when VEC: in and out
// 16-byte aligned), so a wave's accesses are contiguous.  (One thread per 16
// consecutive values, each loaded alone, took 100 us for 16.7M values; the
// rows take about 23.)
template <bool VEC>
__global__ void __launch_bounds__(256) k_scan_apply(const uint32_t* __restrict__ in, int64_t n,
                                                    const uint32_t* __restrict__ n_live,
                                                    const uint32_t* __restrict__ part,
                                                    uint32_t* __restrict__ out) {
    constexpr int kRows = kScanTile / 1024;
    static_assert(kScanTile % 1024 == 0, "scan tiles are whole rows of 1024 values");
    __shared__ uint32_t s_w[kRows][4];
    n = live_count(n, n_live);
    const int64_t tile0 = (int64_t)blockIdx.x * kScanTile;
    if (tile0 >= n) return;
    const int t = threadIdx.x, lane = wave_lane(), w = t >> 6;
    uint4 q[kRows];
    uint32_t own[kRows], x[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const int64_t i = tile0 + r * 1024 + 4 * t;
        if (VEC && i + 3 < n) {
            q[r] = *reinterpret_cast<const uint4*>(in + i);
        } else {
            q[r].x = i < n ? in[i] : 0u;
            q[r].y = i + 1 < n ? in[i + 1] : 0u;
            q[r].z = i + 2 < n ? in[i + 2] : 0u;
            q[r].w = i + 3 < n ? in[i + 3] : 0u;
        }
        own[r] = q[r].x + q[r].y + q[r].z + q[r].w;
        x[r] = own[r];
    }
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const uint32_t y = __shfl_up(x[r], o, kWave);
            if (lane >= o) x[r] += y;
        }
    }
    if (lane == kWave - 1) {
#pragma unroll
        for (int r = 0; r < kRows; ++r) s_w[r][w] = x[r];
    }
    __syncthreads();
    uint32_t run = part[blockIdx.x];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        uint32_t wbase = 0;
        for (int k = 0; k < w; ++k) wbase += s_w[r][k];
        uint4 e;
        e.x = run + wbase + x[r] - own[r];
        e.y = e.x + q[r].x;
        e.z = e.y + q[r].y;
        e.w = e.z + q[r].z;
        const int64_t i = tile0 + r * 1024 + 4 * t;
        if (VEC && i + 3 < n) {
            *reinterpret_cast<uint4*>(out + i) = e;
        } else {
            if (i < n) out[i] = e.x;
            if (i + 1 < n) out[i + 1] = e.y;
            if (i + 2 < n) out[i + 2] = e.z;
            if (i + 3 < n) out[i + 3] = e.w;
        }
        run += s_w[r][0] + s_w[r][1] + s_w[r][2] + s_w[r][3];
    }
}

// Short arrays in one block of 1024 threads, one launch instead of three.
// A segment is kScanSmallRows rows of 4096 values; thread t loads values
// 4t..4t+3 of each row with one 16-byte load, and the rows of a segment are
// scanned together between one pair of barriers, with a running carry from
// segment to segment.  in and out must be 16-byte aligned.
constexpr int kScanSmallRows = 4;
constexpr int64_t kScanSmallSeg = kScanSmallRows * 4096;
constexpr int64_t kScanSmallMax = 8 * kScanSmallSeg;   // longest array sent here

__global__ void __launch_bounds__(1024) k_scan_small(const uint32_t* __restrict__ in, int64_t n,
                                                     const uint32_t* __restrict__ n_live,
                                                     uint32_t* __restrict__ out) {
    __shared__ uint32_t s_w[kScanSmallRows][16];
    const int64_t m = live_count(n, n_live);
    const int t = threadIdx.x, lane = wave_lane(), w = t >> 6;
    uint32_t carry = 0;
    for (int64_t c = 0; c < m; c += kScanSmallSeg) {
        uint4 q[kScanSmallRows];
        uint32_t x[kScanSmallRows], sum[kScanSmallRows];
#pragma unroll
        for (int r = 0; r < kScanSmallRows; ++r) {
            const int64_t i = c + r * 4096 + 4 * t;
            if (i + 3 < m) {
                q[r] = *reinterpret_cast<const uint4*>(in + i);
            } else {
                q[r].x = i < m ? in[i] : 0u;
                q[r].y = i + 1 < m ? in[i + 1] : 0u;
                q[r].z = i + 2 < m ? in[i + 2] : 0u;
                q[r].w = 0u;
            }
            sum[r] = q[r].x + q[r].y + q[r].z + q[r].w;
            x[r] = sum[r];
        }
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
#pragma unroll
            for (int r = 0; r < kScanSmallRows; ++r) {
                const uint32_t y = __shfl_up(x[r], o, kWave);
                if (lane >= o) x[r] += y;
            }
        }
        if (lane == kWave - 1) {
#pragma unroll
            for (int r = 0; r < kScanSmallRows; ++r) s_w[r][w] = x[r];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kScanSmallRows; ++r) {
            uint32_t pre = 0, tot = 0;
            for (int k = 0; k < 16; ++k) {
                const uint32_t v = s_w[r][k];
                if (k < w) pre += v;
                tot += v;
            }
            const int64_t i = c + r * 4096 + 4 * t;
            uint4 e;
            e.x = carry + pre + x[r] - sum[r];
            e.y = e.x + q[r].x;
            e.z = e.y + q[r].y;
            e.w = e.z + q[r].z;
            if (i + 3 < m) {
                *reinterpret_cast<uint4*>(out + i) = e;
            } else {
                if (i < m) out[i] = e.x;
                if (i + 1 < m) out[i + 1] = e.y;
                if (i + 2 < m) out[i + 2] = e.z;
            }
            carry += tot;
        }
        __syncthreads();    // s_w is rewritten by the next segment
    }
    if (t == 0) {
        out[n] = carry;
        out[m] = carry;
    }
}

// Exclusive scan of n values (the first min(n, *n_live) with n_live) into
// out, with out[n] and out[live] the total; part holds `tiles` partial sums.
static void scan_u32(const uint32_t* in, int64_t n, const uint32_t* n_live, uint32_t* out, uint32_t* part,
                     int64_t tiles, hipStream_t s) {
    if (n <= kScanSmallMax && (reinterpret_cast<uintptr_t>(in) & 15) == 0 &&
        (reinterpret_cast<uintptr_t>(out) & 15) == 0) {
        hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, s, in, n, n_live, out);
        return;
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)tiles), dim3(256), 0, s, in, n, n_live, part);
    hipLaunchKernelGGL(k_scan_part, dim3(1), dim3(1024), 0, s, part, tiles, out, n, n_live);
    if ((reinterpret_cast<uintptr_t>(in) & 15) == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0)
        hipLaunchKernelGGL(k_scan_apply<true>, dim3((unsigned)tiles), dim3(256), 0, s, in, n, n_live,
                           (const uint32_t*)part, out);
    else
        hipLaunchKernelGGL(k_scan_apply<false>, dim3((unsigned)tiles), dim3(256), 0, s, in, n, n_live,
                           (const uint32_t*)part, out);
}

// ------------------------------------------------------------ topology ----

// Number of leading Morton digits two keys share (L if equal).
template <int D>
__device__ __forceinline__ int common_digits(uint64_t a, uint64_t b) {
    const uint64_t x = a ^ b;
    if (x == 0) return D == 3 ? 21 : 31;
    const int z = __clzll(x);
    return D == 3 ? (z - 1) / 3 : (z - 2) / 2;
}

// Per body i: a = the shallowest level at which a cell starts at i (one
// past the digits i shares with i - 1), lstar = the deepest level of a cell
// containing i that is not a leaf, plus one (leaf_cap + 1 consecutive
// bodies sharing c digits put an internal cell at level c).  The window
// depths c_j = common digits of bodies j and j + leaf_cap are computed once
// per block tile into LDS, and each body takes the maximum over the windows
// that contain it.
constexpr int kTopoTile = 256;

template <int D>
__global__ void __launch_bounds__(kTopoTile) k_topo_count(const uint64_t* __restrict__ keys, int64_t n, int leaf_cap,
                                                          uint32_t* __restrict__ range, uint32_t* __restrict__ nper) {
    constexpr int L = D == 3 ? 21 : 31;
    __shared__ int8_t s_c[kTopoTile + kMaxLeafCap];   // c_j for j = i0 - leaf_cap .. i0 + kTopoTile - 1
    const int t = threadIdx.x;
    for (int64_t i0 = (int64_t)blockIdx.x * kTopoTile; i0 < n; i0 += (int64_t)gridDim.x * kTopoTile) {
        for (int q = t; q < kTopoTile + leaf_cap; q += kTopoTile) {
            const int64_t j = i0 - leaf_cap + q;
            s_c[q] = (j >= 0 && j + leaf_cap < n) ? (int8_t)common_digits<D>(keys[j], keys[j + leaf_cap]) : (int8_t)-1;
        }
        __syncthreads();
        const int64_t i = i0 + t;
        if (i < n) {
            const int a = (i == 0) ? 0 : common_digits<D>(keys[i - 1], keys[i]) + 1;
            // windows j = i - leaf_cap .. i (those out of range hold -1)
            int deep = -1;
            for (int q = t; q <= t + leaf_cap; ++q) deep = s_c[q] > deep ? s_c[q] : deep;
            int lstar = 0;
            if (deep >= 0) lstar = (deep < L - 1 ? deep : L - 1) + 1;
            range[i] = (uint32_t)a | ((uint32_t)lstar << 8);
            nper[i] = lstar >= a ? (uint32_t)(lstar - a + 1) : 0u;
        }
        __syncthreads();
    }
}

// The cells that start at body i (levels a_i..l*_i) at their pre-order
// indices cstart[i] + (l - a_i): prefix, first body, level, parent and the
// leaf mark.  Their ends (count and skip) come from k_topo_ends, one lane
// per cell: a body that starts many cells would otherwise run their
// searches one after another while the other lanes of its wave, most of
// which start none, wait.
template <int D>
__global__ void __launch_bounds__(256) k_topo_emit(const uint64_t* __restrict__ keys, int64_t n,
                                                   const uint32_t* __restrict__ range,
                                                   const uint32_t* __restrict__ cstart, Cell* __restrict__ cells,
                                                   int64_t cmax, DevParams* prm) {
    constexpr int L = D == 3 ? 21 : 31;
    const uint32_t C = cstart[n];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // C never exceeds the bound (internal cells are disjoint per level
        // and hold > leaf_cap bodies); clamp anyway so no reader can run off
        prm->ncells = (int64_t)C > cmax ? (uint32_t)cmax : C;
        if ((int64_t)C > cmax) atomicOr(&prm->status, kFlagOverflow);
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int a = (int)(range[i] & 255u), lstar = (int)(range[i] >> 8);
        if (lstar < a) continue;
        const uint32_t base = cstart[i];
        const uint64_t key = keys[i];
        for (int l = a; l <= lstar; ++l) {
            const int64_t k = (int64_t)base + (l - a);
            if (k >= cmax) break;
            Cell c;
            c.prefix = l == 0 ? 0ull : key >> (D * (L - l));
            c.begin = (int32_t)i;
            c.count = 0;                           // k_topo_ends
            c.skip = 0;
            c.parent = (l == 0) ? -1 : (l > a ? (int32_t)(k - 1) : -2);
            c.level = l;
            c.leaf_nch = (l == lstar) ? (int32_t)0x80000000u : 0;
            cells[k] = c;
        }
    }
}

// Each cell's end: the first body after its first whose prefix at the
// cell's level differs (a galloping search, then bisection over the sorted
// keys; the root ends at n), giving its body count and its skip (the
// pre-order index of the cell that starts there).
template <int D>
__global__ void __launch_bounds__(256) k_topo_ends(const uint64_t* __restrict__ keys, int64_t n,
                                                   const uint32_t* __restrict__ cstart, Cell* __restrict__ cells,
                                                   const DevParams* __restrict__ prm, int64_t cmax) {
    constexpr int L = D == 3 ? 21 : 31;
    int64_t C = prm->ncells;
    if (C > cmax) C = cmax;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < C;
         k += (int64_t)gridDim.x * blockDim.x) {
        const Cell c = cells[k];
        const int64_t i = c.begin;
        const int l = c.level;
        int64_t end = n;
        if (l > 0) {
            const int shift = D * (L - l);
            const uint64_t prefix = c.prefix;
            int64_t lo = i, step = 1, hi = i + 1;
            while (hi < n && (keys[hi] >> shift) == prefix) {
                lo = hi;
                step <<= 1;
                hi = i + step;
            }
            if (hi > n) hi = n;
            while (hi - lo > 1) {
                const int64_t mid = lo + ((hi - lo) >> 1);
                if ((keys[mid] >> shift) == prefix) lo = mid; else hi = mid;
            }
            end = hi;
        }
        cells[k].count = (int32_t)(end - i);
        cells[k].skip = (int32_t)cstart[end];
    }
}

__global__ void __launch_bounds__(256) k_topo_link(Cell* __restrict__ cells,
                                                   const DevParams* __restrict__ prm, int64_t cmax) {
    int64_t C = prm->ncells;
    if (C > cmax) C = cmax;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < C;
         k += (int64_t)gridDim.x * blockDim.x) {
        const Cell c = cells[k];
        if (c.leaf_nch < 0) continue;          // leaf
        int nch = 0;
        int64_t ch = k + 1;
        const int64_t end = c.skip < C ? c.skip : C;
        while (ch < end) {
            cells[ch].parent = (int32_t)k;
            ++nch;
            const int64_t nx = cells[ch].skip;
            ch = nx > ch ? nx : end;           // defensive: the skip chain only moves forward
        }
        cells[k].leaf_nch = nch;
    }
}

// ------------------------------------------------------------- moments ----

template <int D>
__device__ void leaf_moments(const Cell& c, const Body* __restrict__ bodies, Moments& mo) {
    double M = 0.0, S0 = 0.0, S1 = 0.0, S2 = 0.0;
#pragma unroll 4
    for (int32_t j = c.begin; j < c.begin + c.count; ++j) {
        const Body b = bodies[j];
        M = M + b.m;
        S0 = S0 + b.m * b.x;
        S1 = S1 + b.m * b.y;
        if (D == 3) S2 = S2 + b.m * b.z;
    }
    mo.M = M;
    mo.S[0] = S0; mo.S[1] = S1; mo.S[2] = S2;
    mo.com[0] = S0 / M; mo.com[1] = S1 / M; mo.com[2] = D == 3 ? S2 / M : 0.0;
    double Q[6] = {0, 0, 0, 0, 0, 0};
    if (D == 3) {
#pragma unroll 4
        for (int32_t j = c.begin; j < c.begin + c.count; ++j) {
            const Body b = bodies[j];
            const double d0 = b.x - mo.com[0], d1 = b.y - mo.com[1], d2 = b.z - mo.com[2];
            const double r2 = (d0 * d0 + d1 * d1) + d2 * d2;
            Q[0] = Q[0] + b.m * ((3.0 * d0) * d0 - r2);
            Q[1] = Q[1] + b.m * ((3.0 * d1) * d1 - r2);
            Q[2] = Q[2] + b.m * ((3.0 * d2) * d2 - r2);
            Q[3] = Q[3] + b.m * ((3.0 * d0) * d1);
            Q[4] = Q[4] + b.m * ((3.0 * d0) * d2);
            Q[5] = Q[5] + b.m * ((3.0 * d1) * d2);
        }
    }
    for (int q = 0; q < 6; ++q) mo.Q[q] = Q[q];
    mo.pad = 0.0;
}

// An internal cell's moments from its children's, in digit order.  The
// children are contiguous in level order from the level-order index
// `first`, and kid points at their level-order copies.
template <int D>
__device__ void internal_moments(const Moments* __restrict__ kid, int nch, Moments& mo) {
    // fixed trip counts (predicated) let all children's loads issue together
    double M = 0.0, S0 = 0.0, S1 = 0.0, S2 = 0.0;
#pragma unroll
    for (int i = 0; i < (1 << D); ++i) {
        if (i >= nch) continue;
        M = M + kid[i].M;
        S0 = S0 + kid[i].S[0];
        S1 = S1 + kid[i].S[1];
        if (D == 3) S2 = S2 + kid[i].S[2];
    }
    mo.M = M;
    mo.S[0] = S0; mo.S[1] = S1; mo.S[2] = S2;
    mo.com[0] = S0 / M; mo.com[1] = S1 / M; mo.com[2] = D == 3 ? S2 / M : 0.0;
    double Q[6] = {0, 0, 0, 0, 0, 0};
    if (D == 3) {
#pragma unroll
        for (int i = 0; i < (1 << D); ++i) {
            if (i >= nch) continue;
            const double s0 = kid[i].com[0] - mo.com[0];
            const double s1 = kid[i].com[1] - mo.com[1];
            const double s2 = kid[i].com[2] - mo.com[2];
            const double r2 = (s0 * s0 + s1 * s1) + s2 * s2;
            const double Mc = kid[i].M;
            Q[0] = Q[0] + (kid[i].Q[0] + Mc * ((3.0 * s0) * s0 - r2));
            Q[1] = Q[1] + (kid[i].Q[1] + Mc * ((3.0 * s1) * s1 - r2));
            Q[2] = Q[2] + (kid[i].Q[2] + Mc * ((3.0 * s2) * s2 - r2));
            Q[3] = Q[3] + (kid[i].Q[3] + Mc * ((3.0 * s0) * s1));
            Q[4] = Q[4] + (kid[i].Q[4] + Mc * ((3.0 * s0) * s2));
            Q[5] = Q[5] + (kid[i].Q[5] + Mc * ((3.0 * s1) * s2));
        }
    }
    for (int q = 0; q < 6; ++q) mo.Q[q] = Q[q];
    mo.pad = 0.0;
}

__device__ __forceinline__ void store_walk(WalkCell* walk, const uint32_t* __restrict__ pre2bfs, int64_t k,
                                           const Cell& c, const Moments& mo) {
    WalkCell w;
    w.cx = mo.com[0];
    w.cy = mo.com[1];
    w.cz = mo.com[2];
    w.rcrit2 = INFINITY;
    w.m = (float)mo.M;
    if (c.leaf_nch < 0) {
        w.a = c.begin;
        w.b = (c.count & 0x7fffffff) | (int32_t)0x80000000u;
    } else {
        w.a = (int32_t)pre2bfs[k + 1];           // first child, pre-order k + 1
        w.b = c.leaf_nch;
    }
    w.pad = 0;
    walk[pre2bfs[k]] = w;
}

// Leaves first, all levels in one launch (in pre-order, each leaf summing
// its bodies in order), which also records every cell's children in level
// order (first child, count; a leaf gets kLeafKids) and a level-order copy
// of the leaves' moments.  Then one launch per level, deepest first, for
// the internal cells: a cell's children sit one level below it and were
// finished by an earlier launch, so no cross-block synchronisation is
// needed, and with the level-order copies a cell waits on two dependent
// loads (its children's range, then their moments) instead of five.
// Internal cells sum their children in digit order: the result does not
// depend on scheduling.  (Leaves inside the per-level launches and
// children found through the pre-order arrays took 186 us per build of 1M
// bodies; leaves first, 171 us.)
constexpr uint32_t kLeafKids = 0xffffffffu;

template <int D>
__global__ void __launch_bounds__(256) k_leaf_moments(const Cell* __restrict__ cells, const Body* __restrict__ bodies,
                                                      const uint32_t* __restrict__ pre2bfs,
                                                      const DevParams* __restrict__ prm, int64_t cmax,
                                                      Moments* __restrict__ mom, Moments* __restrict__ mom_lvl,
                                                      uint2* __restrict__ kids, WalkCell* __restrict__ walk) {
    int64_t C = prm->ncells;
    if (C > cmax) C = cmax;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < C; k += (int64_t)gridDim.x * blockDim.x) {
        const Cell c = cells[k];
        const uint32_t b = pre2bfs[k];
        if (c.leaf_nch >= 0) {
            kids[b] = make_uint2(pre2bfs[k + 1], (uint32_t)c.leaf_nch);   // first child: pre-order k + 1
            continue;
        }
        kids[b] = make_uint2(0u, kLeafKids);
        Moments mo;
        leaf_moments<D>(c, bodies, mo);
        mom[k] = mo;
        mom_lvl[b] = mo;
        store_walk(walk, pre2bfs, k, c, mo);
    }
}

// The outputs of internal cell b (level order) with children kc.
__device__ __forceinline__ void store_internal(int64_t b, uint2 kc, const Moments& mo,
                                               const uint32_t* __restrict__ bfs2pre, Moments* mom,
                                               Moments* mom_lvl, WalkCell* __restrict__ walk) {
    mom_lvl[b] = mo;
    mom[bfs2pre[b]] = mo;
    WalkCell w;
    w.cx = mo.com[0];
    w.cy = mo.com[1];
    w.cz = mo.com[2];
    w.rcrit2 = INFINITY;
    w.m = (float)mo.M;
    w.a = (int32_t)kc.x;
    w.b = (int32_t)kc.y;
    w.pad = 0;
    walk[b] = w;
}

// One internal cell of the level passes.
template <int D>
__device__ __forceinline__ void moments_of_internal(int64_t b, const uint32_t* __restrict__ bfs2pre,
                                                    const uint2* __restrict__ kids, Moments* mom, Moments* mom_lvl,
                                                    WalkCell* __restrict__ walk) {
    const uint2 kc = kids[b];
    if (kc.y == kLeafKids) return;
    Moments mo;
    internal_moments<D>(mom_lvl + kc.x, (int)kc.y, mo);
    store_internal(b, kc, mo, bfs2pre, mom, mom_lvl, walk);
}

// Levels `deepest` down to top + 1, deepest first, in one block: a launch
// costs a few microseconds even when its level is nearly empty, and most of
// the deepest levels are.  Which levels come here follows from an earlier
// tree, so they usually hold few cells; any cells they do hold are still
// done (in order: a barrier separates the levels, and the block's waves
// share one CU's L1).
constexpr int kDeepThreads = 1024;

template <int D>
__global__ void __launch_bounds__(kDeepThreads) k_moments_deep(const uint32_t* __restrict__ bfs2pre,
                                                               const uint32_t* __restrict__ lvl_off, int top,
                                                               int deepest, const uint2* __restrict__ kids,
                                                               Moments* mom, Moments* mom_lvl,
                                                               WalkCell* __restrict__ walk) {
    for (int l = deepest; l > top; --l) {
        const int64_t b0 = lvl_off[l], b1 = lvl_off[l + 1];
        for (int64_t b = b0 + threadIdx.x; b < b1; b += kDeepThreads)
            moments_of_internal<D>(b, bfs2pre, kids, mom, mom_lvl, walk);
        __syncthreads();
    }
}

template <int D>
__global__ void __launch_bounds__(256) k_moments_level(const uint32_t* __restrict__ bfs2pre,
                                                       const uint32_t* __restrict__ lvl_off, int level,
                                                       const uint2* __restrict__ kids, Moments* mom,
                                                       Moments* mom_lvl, WalkCell* __restrict__ walk) {
    const int64_t b0 = lvl_off[level], b1 = lvl_off[level + 1];
    for (int64_t b = b0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < b1;
         b += (int64_t)gridDim.x * blockDim.x)
        moments_of_internal<D>(b, bfs2pre, kids, mom, mom_lvl, walk);
}

// Levels `head` down to 0 in one block, their moments kept in LDS: these
// levels occupy level-order indices 0 .. lvl_off[head + 1] - 1, so a cell's
// LDS slot is its level-order index, and each level reads its children from
// LDS instead of going round through memory (the head level's children
// come from the level below, done by an earlier launch).  Which levels come
// here follows from an earlier tree; if the current one holds more than
// kHeadCells cells in them, the block reads the children from memory
// instead, as the per-level passes do.
constexpr int kHeadCells = 512;

template <int D>
__global__ void __launch_bounds__(kDeepThreads) k_moments_head(const uint32_t* __restrict__ bfs2pre,
                                                               const uint32_t* __restrict__ lvl_off, int head,
                                                               const uint2* __restrict__ kids, Moments* mom,
                                                               Moments* mom_lvl, WalkCell* __restrict__ walk) {
    __shared__ Moments s_m[kHeadCells];
    const bool fit = lvl_off[head + 1] <= (uint32_t)kHeadCells;
    for (int l = head; l >= 0; --l) {
        const int64_t b0 = lvl_off[l], b1 = lvl_off[l + 1];
        for (int64_t b = b0 + threadIdx.x; b < b1; b += kDeepThreads) {
            const uint2 kc = kids[b];
            if (kc.y == kLeafKids) {
                if (fit) s_m[b] = mom_lvl[b];
                continue;
            }
            Moments mo;
            internal_moments<D>((fit && l < head ? s_m : mom_lvl) + kc.x, (int)kc.y, mo);
            if (fit) s_m[b] = mo;
            store_internal(b, kc, mo, bfs2pre, mom, mom_lvl, walk);
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------- mac ----

template <int D>
__global__ void __launch_bounds__(256) k_mac(const Cell* __restrict__ cells, const Moments* __restrict__ mom,
                                             double theta, const uint32_t* __restrict__ pre2bfs,
                                             WalkCell* __restrict__ walk, double* __restrict__ rc_out,
                                             const DevParams* __restrict__ prm, int64_t cmax) {
    int64_t C = prm->ncells;
    if (C > cmax) C = cmax;
    const double size = prm->size;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < C;
         k += (int64_t)gridDim.x * blockDim.x) {
        if (theta == 0.0) {
            if (rc_out) rc_out[pre2bfs[k]] = INFINITY;
            else walk[pre2bfs[k]].rcrit2 = INFINITY;
            continue;
        }
        const Cell c = cells[k];
        const int l = c.level;
        const double s = ldexp(size, -l);
        uint64_t org[3] = {0, 0, 0};
        for (int j = 1; j <= l; ++j) {
            const unsigned d = (unsigned)((c.prefix >> (D * (l - j))) & ((1u << D) - 1u));
#pragma unroll
            for (int a = 0; a < D; ++a) org[a] = (org[a] << 1) | ((d >> (D - 1 - a)) & 1u);
        }
        double dd[3];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const double centre = prm->lo[a] + ((double)org[a] + 0.5) * s;
            dd[a] = mom[k].com[a] - centre;
        }
        double d2 = dd[0] * dd[0] + dd[1] * dd[1];
        if (D == 3) d2 = d2 + dd[2] * dd[2];
        const double r = s / theta + sqrt(d2);
        if (rc_out) rc_out[pre2bfs[k]] = r * r;
        else walk[pre2bfs[k]].rcrit2 = r * r;
    }
}

// ---------------------------------------------------------- walk groups ----
// A walk group is a run of at most 64 consecutive bodies in key order that
// never straddles a cluster cell (a maximal cell holding at most kCluster
// bodies, or a leaf deeper than that): the group's bounding box then stays
// inside one compact region even where the Morton curve jumps across empty
// space.  Cluster cells are found in pre-order, so groups come out in body
// order.

__device__ __forceinline__ bool small_cell(const Cell& c) { return c.count <= kCluster || c.leaf_nch < 0; }

__global__ void __launch_bounds__(256) k_group_count(const Cell* __restrict__ cells, const DevParams* __restrict__ prm,
                                                     int64_t cmax, uint32_t* __restrict__ gper) {
    int64_t C = prm->ncells;
    if (C > cmax) C = cmax;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < C; k += (int64_t)gridDim.x * blockDim.x) {
        const Cell c = cells[k];
        const bool cluster = small_cell(c) && (k == 0 || !small_cell(cells[c.parent]));
        gper[k] = cluster ? (uint32_t)((c.count + kGroup - 1) / kGroup) : 0u;
    }
}

__global__ void __launch_bounds__(256) k_group_emit(const Cell* __restrict__ cells, const uint32_t* __restrict__ goff,
                                                    DevParams* prm, int64_t cmax, int32_t* __restrict__ gbeg,
                                                    int32_t* __restrict__ gcnt, int64_t gmax) {
    int64_t C = prm->ncells;
    if (C > cmax) C = cmax;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t G = goff[cmax];
        prm->ngroups = (int64_t)G > gmax ? (uint32_t)gmax : G;
        if ((int64_t)G > gmax) atomicOr(&prm->status, kFlagOverflow);
    }
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < C;
         k += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t g0 = goff[k], g1 = goff[k + 1];
        if (g1 == g0) continue;
        const Cell c = cells[k];
        for (uint32_t g = g0; g < g1 && (int64_t)g < gmax; ++g) {
            const int32_t o = (int32_t)(g - g0) * kGroup;
            gbeg[g] = c.begin + o;
            gcnt[g] = min(kGroup, c.count - o);
        }
    }
}

// -------------------------------------------------------------- export ----

__global__ void __launch_bounds__(256) k_export(const Cell* __restrict__ cells, const Moments* __restrict__ mom,
                                                int dim, const DevParams* __restrict__ prm, int64_t cmax,
                                                int32_t* level, uint64_t* prefix, int32_t* begin,
                                                int32_t* count, int32_t* parent, int32_t* skip,
                                                int32_t* nch, int32_t* leaf, double* M, double* com,
                                                double* Q) {
    int64_t C = prm->ncells;
    if (C > cmax) C = cmax;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < C;
         k += (int64_t)gridDim.x * blockDim.x) {
        const Cell c = cells[k];
        if (level) level[k] = c.level;
        if (prefix) prefix[k] = c.prefix;
        if (begin) begin[k] = c.begin;
        if (count) count[k] = c.count;
        if (parent) parent[k] = c.parent;
        if (skip) skip[k] = c.skip;
        if (nch) nch[k] = c.leaf_nch < 0 ? 0 : c.leaf_nch;
        if (leaf) leaf[k] = c.leaf_nch < 0 ? 1 : 0;
        if (M) M[k] = mom[k].M;
        if (com)
            for (int a = 0; a < dim; ++a) com[k * dim + a] = mom[k].com[a];
        if (Q)
            for (int q = 0; q < 6; ++q) Q[k * 6 + q] = mom[k].Q[q];
    }
}

}  // namespace

// ------------------------------------------------------------ launchers ----

hipError_t launch_bbox(const void* pos, const void* mass, int64_t n, int dim, int f64,
                       double* part, void* packed, DevParams* prm, hipStream_t s) {
    const unsigned nb = grid_for(n, 1024);
    if (f64) {
        if (dim == 3) hipLaunchKernelGGL((k_bbox_part<double, 3>), dim3(nb), dim3(256), 0, s, (const double*)pos, (const double*)mass, n, part, (double4*)packed);
        else hipLaunchKernelGGL((k_bbox_part<double, 2>), dim3(nb), dim3(256), 0, s, (const double*)pos, (const double*)mass, n, part, (double4*)packed);
    } else {
        if (dim == 3) hipLaunchKernelGGL((k_bbox_part<float, 3>), dim3(nb), dim3(256), 0, s, (const float*)pos, (const float*)mass, n, part, (float4*)packed);
        else hipLaunchKernelGGL((k_bbox_part<float, 2>), dim3(nb), dim3(256), 0, s, (const float*)pos, (const float*)mass, n, part, (float4*)packed);
    }
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(256), 0, s, part, (int)nb, dim, prm);
    return hipGetLastError();
}

hipError_t launch_keys(const void* pos, int64_t n, int dim, int f64, const DevParams* prm,
                       uint64_t* keys, uint32_t* idx, hipStream_t s) {
    const unsigned nb = grid_for(n);
    if (f64) {
        if (dim == 3) hipLaunchKernelGGL((k_keys<double, 3>), dim3(nb), dim3(256), 0, s, (const double*)pos, n, prm, keys, idx);
        else hipLaunchKernelGGL((k_keys<double, 2>), dim3(nb), dim3(256), 0, s, (const double*)pos, n, prm, keys, idx);
    } else {
        if (dim == 3) hipLaunchKernelGGL((k_keys<float, 3>), dim3(nb), dim3(256), 0, s, (const float*)pos, n, prm, keys, idx);
        else hipLaunchKernelGGL((k_keys<float, 2>), dim3(nb), dim3(256), 0, s, (const float*)pos, n, prm, keys, idx);
    }
    return hipGetLastError();
}

// One pass of the reduce-then-scan sort (2 or 3 launches).
template <int PER, bool STAGE, class In, class Out>
static void sort_pass(In in, Out out, int64_t n, const uint32_t* n_live, int shift, uint32_t* hist,
                      uint32_t* digit_tot, hipStream_t s) {
    const int64_t tiles = (n + 256 * PER - 1) / (256 * PER);
    hipLaunchKernelGGL((k_sort_hist<PER, In>), dim3((unsigned)tiles), dim3(256), 0, s, in, n, n_live, shift, hist,
                       tiles);
    if (tiles <= kSortScanInScatter) {
        hipLaunchKernelGGL((k_sort_scatter<PER, true, STAGE, In, Out>), dim3((unsigned)tiles), dim3(256), 0, s, in, out, n,
                           n_live, shift, (const uint32_t*)hist, digit_tot, tiles);
        return;
    }
    hipLaunchKernelGGL(k_sort_scan<PER>, dim3(256), dim3(256), 0, s, hist, tiles, n, n_live, digit_tot);
    hipLaunchKernelGGL((k_sort_scatter<PER, false, STAGE, In, Out>), dim3((unsigned)tiles), dim3(256), 0, s, in, out, n,
                       n_live, shift, (const uint32_t*)hist, digit_tot, tiles);
}

template <int PER, bool STAGE>
static void sort_passes(uint64_t* keys_a, uint32_t* idx_a, uint64_t* keys_b, uint32_t* idx_b, int64_t n,
                        const uint32_t* n_live, int passes, uint32_t* hist, uint32_t* digit_tot, hipStream_t s) {
    for (int p = 0; p < passes; ++p) {
        const bool even = (p % 2) == 0;
        const PairsIn in{even ? keys_a : keys_b, even ? idx_a : idx_b};
        const PairsOut out{even ? keys_b : keys_a, even ? idx_b : idx_a};
        sort_pass<PER, STAGE>(in, out, n, n_live, 8 * p, hist, digit_tot, s);
    }
}

hipError_t launch_sort(uint64_t* keys_a, uint32_t* idx_a, uint64_t* keys_b, uint32_t* idx_b,
                       int64_t n, int key_bits, uint32_t* hist, uint32_t* digit_tot, hipStream_t s) {
    const int passes = (key_bits + 7) / 8;    // even for 62/63-bit keys: result lands in _a
    if (n >= kSortStageMin) {
        sort_passes<kSortStagePer, true>(keys_a, idx_a, keys_b, idx_b, n, nullptr, passes, hist, digit_tot, s);
        return hipGetLastError();
    }
    switch (sort_per(n)) {
        case 16: sort_passes<16, false>(keys_a, idx_a, keys_b, idx_b, n, nullptr, passes, hist, digit_tot, s); break;
        case 8: sort_passes<8, false>(keys_a, idx_a, keys_b, idx_b, n, nullptr, passes, hist, digit_tot, s); break;
        default: sort_passes<4, false>(keys_a, idx_a, keys_b, idx_b, n, nullptr, passes, hist, digit_tot, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_gather(const void* packed, const uint32_t* perm, int64_t n, int f64, Body* bodies,
                         float4* bodies32, hipStream_t s) {
    const unsigned nb = grid_for(n);
    if (f64) hipLaunchKernelGGL(k_gather<double>, dim3(nb), dim3(256), 0, s, (const double4*)packed, perm, n, bodies, (float4*)nullptr);
    else hipLaunchKernelGGL(k_gather<float>, dim3(nb), dim3(256), 0, s, (const float4*)packed, perm, n, bodies, bodies32);
    return hipGetLastError();
}

hipError_t launch_scan_u32(const uint32_t* in, int64_t n, uint32_t* out, uint32_t* part, int64_t tiles,
                           hipStream_t s) {
    scan_u32(in, n, nullptr, out, part, tiles, s);
    return hipGetLastError();
}

hipError_t launch_topology(const uint64_t* keys, int64_t n, int dim, int leaf_cap,
                           uint32_t* range, uint32_t* nper, uint32_t* cstart,
                           uint32_t* scan_part, int64_t scan_tiles, Cell* cells,
                           int64_t cmax, DevParams* prm, hipStream_t s) {
    const unsigned nb = grid_for(n);
    if (dim == 3) hipLaunchKernelGGL(k_topo_count<3>, dim3(nb), dim3(256), 0, s, keys, n, leaf_cap, range, nper);
    else hipLaunchKernelGGL(k_topo_count<2>, dim3(nb), dim3(256), 0, s, keys, n, leaf_cap, range, nper);
    scan_u32(nper, n, nullptr, cstart, scan_part, scan_tiles, s);
    if (dim == 3) hipLaunchKernelGGL(k_topo_emit<3>, dim3(nb), dim3(256), 0, s, keys, n, (const uint32_t*)range, (const uint32_t*)cstart, cells, cmax, prm);
    else hipLaunchKernelGGL(k_topo_emit<2>, dim3(nb), dim3(256), 0, s, keys, n, (const uint32_t*)range, (const uint32_t*)cstart, cells, cmax, prm);
    const unsigned nc = grid_for(cmax);
    if (dim == 3) hipLaunchKernelGGL(k_topo_ends<3>, dim3(nc), dim3(256), 0, s, keys, n, (const uint32_t*)cstart, cells, (const DevParams*)prm, cmax);
    else hipLaunchKernelGGL(k_topo_ends<2>, dim3(nc), dim3(256), 0, s, keys, n, (const uint32_t*)cstart, cells, (const DevParams*)prm, cmax);
    hipLaunchKernelGGL(k_topo_link, dim3(nc), dim3(256), 0, s, cells, (const DevParams*)prm, cmax);
    return hipGetLastError();
}

hipError_t launch_level_order(const Cell* cells, int64_t cmax, int64_t cells_est, int dim, const DevParams* prm,
                              uint32_t* bfs2pre, uint32_t* hist, uint32_t* digit_tot, uint32_t* pre2bfs,
                              uint32_t* lvl_off, hipStream_t s) {
    // one pass by level over the live cells (their count is on the device,
    // so the tile follows the host's estimate of it: the slots are several
    // times more; 1M bodies: 16 against 27 us per pass with tiles sized for
    // the slots)
    const LevelsIn in{cells};
    const LevelsOut out{bfs2pre, pre2bfs, lvl_off, levels_for(dim)};
    switch (sort_per(cells_est)) {
        case 16: sort_pass<16, false>(in, out, cmax, &prm->ncells, 0, hist, digit_tot, s); break;
        case 8: sort_pass<8, false>(in, out, cmax, &prm->ncells, 0, hist, digit_tot, s); break;
        default: sort_pass<4, false>(in, out, cmax, &prm->ncells, 0, hist, digit_tot, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_groups(const Cell* cells, int64_t cmax, uint32_t* gper, uint32_t* goff, uint32_t* scan_part,
                         int64_t scan_tiles, int32_t* gbeg, int32_t* gcnt, int64_t gmax, DevParams* prm,
                         hipStream_t s) {
    const unsigned nb = grid_for(cmax);
    hipLaunchKernelGGL(k_group_count, dim3(nb), dim3(256), 0, s, cells, (const DevParams*)prm, cmax, gper);
    // over the live cells only (their count is on the device)
    const uint32_t* live = &prm->ncells;
    scan_u32(gper, cmax, live, goff, scan_part, scan_tiles, s);
    hipLaunchKernelGGL(k_group_emit, dim3(nb), dim3(256), 0, s, cells, (const uint32_t*)goff, prm, cmax, gbeg,
                       gcnt, gmax);
    return hipGetLastError();
}

hipError_t launch_moments(const Cell* cells, const Body* bodies, int dim, int64_t cmax,
                          const uint32_t* bfs2pre, const uint32_t* pre2bfs, const uint32_t* lvl_off,
                          const DevParams* prm, Moments* mom, Moments* mom_lvl, uint2* kids, WalkCell* walk,
                          const uint32_t* hint, hipStream_t s) {
    const int L = levels_for(dim);
    // levels L..top+1 go to one single-block launch, top..0 to one launch
    // each.  (The top levels hold few cells too, but there one launch per
    // level is the faster: a level's cost is a chain of dependent loads and
    // stores either way, and the single block adds its barrier waits.)
    int top = L;
    int64_t cnt[66] = {};
    if (hint) {
        for (int l = 0; l <= L; ++l) cnt[l] = (int64_t)hint[l + 1] - (int64_t)hint[l];
        top = 0;
        for (int l = L; l > 0; --l)
            if (cnt[l] > kDeepThreads) {
                top = l;
                break;
            }
    }
    // levels head..0 (at most kHeadCells cells together, and at most down
    // from top) go to one single-block launch with their moments in LDS
    int head = -1;
    if (hint)
        while (head + 1 <= top && (int64_t)hint[head + 2] <= kHeadCells) ++head;
    const unsigned nl = grid_for(cmax);
    if (dim == 3)
        hipLaunchKernelGGL(k_leaf_moments<3>, dim3(nl), dim3(256), 0, s, cells, bodies, pre2bfs, prm, cmax, mom,
                           mom_lvl, kids, walk);
    else
        hipLaunchKernelGGL(k_leaf_moments<2>, dim3(nl), dim3(256), 0, s, cells, bodies, pre2bfs, prm, cmax, mom,
                           mom_lvl, kids, walk);
    if (top < L) {
        if (dim == 3)
            hipLaunchKernelGGL(k_moments_deep<3>, dim3(1), dim3(kDeepThreads), 0, s, bfs2pre, lvl_off, top, L,
                               (const uint2*)kids, mom, mom_lvl, walk);
        else
            hipLaunchKernelGGL(k_moments_deep<2>, dim3(1), dim3(kDeepThreads), 0, s, bfs2pre, lvl_off, top, L,
                               (const uint2*)kids, mom, mom_lvl, walk);
    }
    for (int l = top; l > head; --l) {
        // an earlier count plus a quarter: a grid-stride loop covers any more
        const unsigned nb = hint ? grid_for(cnt[l] + cnt[l] / 4, 2048) : grid_for(cmax, 2048);
        if (dim == 3)
            hipLaunchKernelGGL(k_moments_level<3>, dim3(nb), dim3(256), 0, s, bfs2pre, lvl_off, l, kids, mom, mom_lvl,
                               walk);
        else
            hipLaunchKernelGGL(k_moments_level<2>, dim3(nb), dim3(256), 0, s, bfs2pre, lvl_off, l, kids, mom, mom_lvl,
                               walk);
    }
    if (head >= 0) {
        if (dim == 3)
            hipLaunchKernelGGL(k_moments_head<3>, dim3(1), dim3(kDeepThreads), 0, s, bfs2pre, lvl_off, head,
                               (const uint2*)kids, mom, mom_lvl, walk);
        else
            hipLaunchKernelGGL(k_moments_head<2>, dim3(1), dim3(kDeepThreads), 0, s, bfs2pre, lvl_off, head,
                               (const uint2*)kids, mom, mom_lvl, walk);
    }
    return hipGetLastError();
}

hipError_t launch_mac(const Cell* cells, const Moments* mom, int dim, double theta, int64_t cmax,
                      const uint32_t* pre2bfs, WalkCell* walk, double* rc_out, const DevParams* prm,
                      hipStream_t s) {
    const unsigned nb = grid_for(cmax);
    if (dim == 3) hipLaunchKernelGGL(k_mac<3>, dim3(nb), dim3(256), 0, s, cells, mom, theta, pre2bfs, walk, rc_out, prm, cmax);
    else hipLaunchKernelGGL(k_mac<2>, dim3(nb), dim3(256), 0, s, cells, mom, theta, pre2bfs, walk, rc_out, prm, cmax);
    return hipGetLastError();
}

hipError_t launch_export(const Cell* cells, const Moments* mom, int dim, int64_t cmax,
                         const DevParams* prm, int32_t* level, uint64_t* prefix, int32_t* begin,
                         int32_t* count, int32_t* parent, int32_t* skip, int32_t* nch,
                         int32_t* leaf, double* M, double* com, double* Q, hipStream_t s) {
    hipLaunchKernelGGL(k_export, dim3(grid_for(cmax)), dim3(256), 0, s, cells, mom, dim, prm, cmax, level,
                       prefix, begin, count, parent, skip, nch, leaf, M, com, Q);
    return hipGetLastError();
}

}  // namespace tc
