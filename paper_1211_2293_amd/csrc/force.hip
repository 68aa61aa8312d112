// Fused tree walk and force summation (§3.1: a cell goes on a body's
// interaction list when it is distant enough, otherwise the walk descends
// into its children; the list is then summed to give the force; §3.2: the
// per-body sums are independent of each other).
//
// One wavefront per walk group (at most 64 consecutive bodies in key order,
// never straddling a cluster cell), one lane per body.  The walk tests whole batches of cells at once: a per-wave LDS
// stack holds ranges of sibling cells (the children of one opened cell are
// contiguous in level order), and each round pops up to 8 ranges (4 in 2D),
// gives every lane one cell, and runs the opening test for all of them in
// FP64.  Accepted cells become list entries, leaves that are not accepted
// contribute their bodies (copied by all lanes together, 16 bodies per leaf
// side by side), opened cells push the range of their children.  The list
// lives in LDS; when it is full it is flushed: every lane sums it for its
// own body in FP32, reading each entry as an LDS broadcast.  Coordinates are
// relative to the group's box centre (FP64 difference, then rounded) so FP32
// keeps the significant digits; chunks of 64 entries are summed plainly and
// folded into Neumaier-compensated totals.  Each group's walk also counts
// the cells it tests (the root and every child of an opened cell), a
// measure of the walk's work that is kept per group.
//
// Stack bound: a round pushes at most 64 ranges; popping a single range at a
// time is a depth-first descent that adds at most (R-1) ranges per level
// plus R (R = cells per range, 8 in 3D, 4 in 2D), so full batches are popped
// only while that reserve is free and the stack can never overflow.
#include "tc_internal.h"
#include "walk_common.h"

#include <math.h>

#include <algorithm>

namespace tc {
namespace {

using namespace walk;
constexpr int kWavesPerBlock = 4;

// Walk for one group from the batch of cells [first, first + first_len) (the
// root alone for a whole walk) and sum its list into a, counting the cell
// entries in nm2p and the body entries in np2p.  The group's box is
// [lo, hi], its FP32 origin (rx, ry, rz), this lane's body (xi, yi, zi).
// With NP > 1 (a walk from the root shared by NP waves) this wave walks
// part `part` of it: the cells above the deal level (level-order indices
// below deal_lo) are tested by every part but their entries kept by part 0
// only; the cells of the deal level ([deal_lo, deal_hi) in level order) are
// dealt out by index modulo NP; everything deeper follows its ancestor at
// the deal level.  The parts' lists together are the whole walk's.
// STAGED: the list sums in staged batches (flush).
template <int D, bool PLAIN, bool QUAD, int NP = 1, bool STAGED = false, int STEP = 8>
__device__ __forceinline__ void walk_group(const WalkCell* __restrict__ walk, const float4* __restrict__ walkq,
                                           const Body* __restrict__ bodies, const float4* __restrict__ bodies32,
                                           float4* L, uint32_t* S, float4* LQ, int lpl_log2, float eps2,
                                           double lox, double hix, double loy, double hiy, double loz, double hiz,
                                           double rx, double ry, double rz, float xi, float yi, float zi,
                                           uint32_t first, int first_len, Acc& a, int64_t& nm2p, int64_t& np2p,
                                           int64_t& ntest, int part = 0, uint32_t deal_lo = 0, uint32_t deal_hi = 0) {
    constexpr int R = D == 3 ? 8 : 4;                    // lanes (cells) per popped range
    constexpr int RP = kWave / R;                        // ranges per full round
    constexpr int kReserve = (R - 1) * (D == 3 ? 21 : 31) + R;
    static_assert(kStackCap >= kWave + kReserve + kWave, "stack too small for its bound");
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t lanes_below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    const int lpl = 1 << lpl_log2;                       // lanes per leaf in a copy batch
    const int slot = lane >> lpl_log2, jj = lane & (lpl - 1);
        int len = 0, qlen = 0;

        // The first batch is the range [first, first + first_len).  Each round: opening tests, pushes,
        // then the NEXT batch is popped and its cell loads issued before
        // this round's entries and leaf bodies are staged, so the two
        // memory round trips of a round overlap.
        int top = 0;
        bool vc = lane < first_len;
        uint32_t cidx = first + (uint32_t)lane;              // level-order index of the tested cell
        WalkCell wc = load_cell(walk, first + (uint32_t)lane, vc);
        float4 q0 = make_float4(0.f, 0.f, 0.f, 0.f), q1 = q0;   // quadrupole of the tested cell
        if (QUAD && vc) {
            q0 = walkq[2 * (size_t)(first + lane)];
            q1 = walkq[2 * (size_t)(first + lane) + 1];
        }
        bool more = true;
        while (more) {
            // opening test: squared distance from the centre of mass to the box
            const double dxm = fmax(fmax(lox - wc.cx, 0.0), wc.cx - hix);
            const double dym = fmax(fmax(loy - wc.cy, 0.0), wc.cy - hiy);
            double d2 = dxm * dxm + dym * dym;
            if (D == 3) {
                const double dzm = fmax(fmax(loz - wc.cz, 0.0), wc.cz - hiz);
                d2 = d2 + dzm * dzm;
            }
            const bool own = vc && (NP == 1 || cidx < deal_lo || cidx >= deal_hi || (int)(cidx % NP) == part);
            const bool emit = NP == 1 || cidx >= deal_lo || part == 0;
            const bool leaf = own && wc.b < 0;
            const bool acc0 = own && d2 > wc.rcrit2;
            const bool opened = own && !acc0 && !leaf;
            const bool accept = acc0 && emit;
            const bool direct = leaf && !acc0 && emit;
            ntest += __popcll(__ballot(own && emit));    // each tested cell once over the parts

            // push the children ranges of opened cells
            const uint64_t O = __ballot(opened);
            if (opened) S[top + __popcll(O & lanes_below)] = ((uint32_t)wc.a << 3) | (uint32_t)(wc.b - 1);
            top += __popcll(O);
            wave_lds_sync();

            // pop the next batch (full batches only while the depth-first
            // reserve is free) and start loading its cells
            more = top > 0;
            bool vcn = false;
            uint32_t cidxn = 0;
            WalkCell wcn;
            float4 q0n = make_float4(0.f, 0.f, 0.f, 0.f), q1n = q0n;
            if (more) {
                const int nr = (top + kWave + kReserve <= kStackCap) ? min(top, RP) : 1;
                const int rr = lane / R, j = lane % R;
                uint32_t packed = 0;
                if (rr < nr) packed = S[top - 1 - rr];
                top -= nr;
                const int rlen = (int)(packed & 7u) + 1;
                vcn = rr < nr && j < rlen;
                cidxn = (packed >> 3) + j;
                wcn = load_cell(walk, (packed >> 3) + j, vcn);
                if (QUAD && vcn) {
                    const uint32_t bq = (packed >> 3) + j;
                    q0n = walkq[2 * (size_t)bq];
                    q1n = walkq[2 * (size_t)bq + 1];
                }
            }
            wave_lds_sync();

            // accepted cells: one entry each, at their centre of mass
            const uint64_t A = __ballot(accept);
            const int na = __popcll(A);
            if (QUAD && na) {
                // with their quadrupole: 3 float4 per entry in the second list
                if (qlen + na > kQuadCap) {
                    flush_quad<PLAIN>(LQ, qlen, xi, yi, zi, eps2, a);
                    qlen = 0;
                }
                if (accept) {
                    const int at = 3 * (qlen + __popcll(A & lanes_below));
                    LQ[at] = make_float4((float)(wc.cx - rx), (float)(wc.cy - ry), (float)(wc.cz - rz), wc.m);
                    LQ[at + 1] = q0;
                    LQ[at + 2] = q1;
                }
                qlen += na;
                nm2p += na;
            } else if (na) {
                if (len + na > kListCap) {
                    flush<D, PLAIN, STAGED, STEP>(L, len, xi, yi, zi, eps2, a);
                    len = 0;
                }
                if (accept)
                    L[len + __popcll(A & lanes_below)] =
                        make_float4((float)(wc.cx - rx), (float)(wc.cy - ry), (float)(wc.cz - rz), wc.m);
                len += na;
                nm2p += na;
            }

            // leaves that are not accepted: their bodies, copied cooperatively
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
                        flush<D, PLAIN, STAGED, STEP>(L, len, xi, yi, zi, eps2, a);
                        len = 0;
                    }
                    if (jj < my_cnt)
                        L[len + my_off + jj] = body_entry(bodies, bodies32, my_begin + jj, rx, ry, rz);
                    len += tot;
                    np2p += tot;
                }
                uint64_t bg = big;
                while (bg) {                                   // leaves larger than a batch slot
                    const int l = __builtin_ctzll(bg);
                    bg &= bg - 1;
                    const int cl = __builtin_amdgcn_readlane(cnt, l);
                    const int bl = __builtin_amdgcn_readlane(wc.a, l);
                    for (int o = 0; o < cl; o += kWave) {
                        const int m = min(kWave, cl - o);
                        if (len + m > kListCap) {
                            flush<D, PLAIN, STAGED, STEP>(L, len, xi, yi, zi, eps2, a);
                            len = 0;
                        }
                        if (lane < m) L[len + lane] = body_entry(bodies, bodies32, bl + o + lane, rx, ry, rz);
                        len += m;
                    }
                    np2p += cl;
                }
            }
            wave_lds_sync();
            wc = wcn;
            vc = vcn;
            cidx = cidxn;
            if (QUAD) {
                q0 = q0n;
                q1 = q1n;
            }
        }
        flush<D, PLAIN, STAGED, STEP>(L, len, xi, yi, zi, eps2, a);
        if (QUAD) flush_quad<PLAIN>(LQ, qlen, xi, yi, zi, eps2, a);
}

template <int D, bool PLAIN, bool QUAD, int STEP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(QUAD ? 4 : 5, 8))) k_walk_force(const WalkCell* __restrict__ walk,
                                                    const float4* __restrict__ walkq,
                                                    const Body* __restrict__ bodies,
                                                    const float4* __restrict__ bodies32,
                                                    const uint32_t* __restrict__ perm,
                                                    const int32_t* __restrict__ gbeg,
                                                    const int32_t* __restrict__ gcnt,
                                                    const uint32_t* __restrict__ order, uint32_t* queue,
                                                    uint32_t* __restrict__ bcost,
                                                    int lpl_log2, float G, float eps2,
                                                    const DevParams* __restrict__ prm,
                                                    float* __restrict__ acc, float* __restrict__ pot,
                                                    int64_t* __restrict__ m2p_out,
                                                    int64_t* __restrict__ p2p_out,
                                                    int64_t* __restrict__ tst_out) {
    static_assert(!QUAD || D == 3, "quadrupole terms are 3D");
    __shared__ float4 s_list[kWavesPerBlock][kListCap];
    __shared__ uint32_t s_stack[kWavesPerBlock][kStackCap];
    __shared__ float4 s_qlist[kWavesPerBlock][QUAD ? 3 * kQuadCap : 1];   // accepted cells with Q
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    float4* L = s_list[wv];
    uint32_t* S = s_stack[wv];
    float4* LQ = s_qlist[wv];

    // Persistent waves, scheduled by GroupSched over the positions of
    // order (a permutation of the groups within each XCD share).
    const GroupSched sched = make_sched(queue, prm->ngroups, kWavesPerBlock);
    for (int hop = 0; hop < kXcd; ++hop) {
        const int xq = (sched.home + hop) % kXcd;
        const uint32_t g_hi = sched.share_lo(xq + 1);
        uint32_t g = sched.first(xq, hop);
        while (g < g_hi) {

            const uint32_t gi = order[g];
            const int64_t i0 = gbeg[gi];
            const int gn = gcnt[gi];
            const int64_t i = i0 + lane;
            const bool valid = lane < gn;
            const Body me = bodies[valid ? i : i0];

            // group bounding box (exact) and its centre, the group's FP32 origin
            const double lox = uniform(wave_min(me.x)), hix = uniform(wave_max(me.x));
            const double loy = uniform(wave_min(me.y)), hiy = uniform(wave_max(me.y));
            const double loz = D == 3 ? uniform(wave_min(me.z)) : 0.0;
            const double hiz = D == 3 ? uniform(wave_max(me.z)) : 0.0;
            const double rx = (lox + hix) * 0.5, ry = (loy + hiy) * 0.5, rz = (loz + hiz) * 0.5;
            const float xi = (float)(me.x - rx), yi = (float)(me.y - ry), zi = (float)(me.z - rz);

            Acc a = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            int64_t nm2p = 0, np2p = 0, ntest = 0;
            walk_group<D, PLAIN, QUAD, 1, false, STEP>(walk, walkq, bodies, bodies32, L, S, LQ, lpl_log2, eps2, lox,
                                                       hix, loy, hiy, loz, hiz, rx, ry, rz, xi, yi, zi, 0u, 1, a, nm2p,
                                                       np2p, ntest);

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
                // the list length, for the next evaluation's schedule
                const int64_t lc = nm2p + np2p;
                bcost[o] = lc > 0xffffffffll ? 0xffffffffu : (uint32_t)lc;
            }
            if (lane == 0) {
                m2p_out[gi] = nm2p;
                p2p_out[gi] = np2p;
                tst_out[gi] = ntest;
            }
            g = sched.pop(xq);
        }
    }
}

// Small and mid-size problems: with fewer groups than resident waves, every
// wave walks its group alone on its SIMD and the walk's latency sets the
// time.  Here a block of NW waves takes one group at a time
// (positions of the cost order of k_group_order, strided by the grid):
// each wave walks its part of the tree (walk_group with NP parts, the cells
// of level `deal` dealt out) and sums its own list, and the parts' FP32 sums
// are added in FP64 in wave order.  The interactions and counts are those
// of the one-wave walk; only the summation order differs.  The near field,
// where most of a group's list comes from, lies in a few cells around the
// group, so a shallow deal level leaves one part with most of the work
// (3D Plummer, 65,536 bodies: 1.15x over one wave dealing level 3, 1.7x
// dealing level 5 or 6); one too deep leaves the parts repeating the walk
// above it.  coop_deal_level holds the measured choice, coop_waves the
// number of waves (NW) per group.
template <int D, bool PLAIN, bool QUAD, int NW>
__global__ void __launch_bounds__(NW * kWave) __attribute__((amdgpu_waves_per_eu(QUAD ? 4 : 5, 8))) k_walk_force_coop(
    const WalkCell* __restrict__ walk, const float4* __restrict__ walkq, const Body* __restrict__ bodies,
    const float4* __restrict__ bodies32, const uint32_t* __restrict__ perm, const int32_t* __restrict__ gbeg,
    const int32_t* __restrict__ gcnt, const uint32_t* __restrict__ order, uint32_t* __restrict__ bcost,
    const uint32_t* __restrict__ lvl_off, int deal, int lpl_log2, float G, float eps2,
    const DevParams* __restrict__ prm,
    float* __restrict__ acc, float* __restrict__ pot, int64_t* __restrict__ m2p_out, int64_t* __restrict__ p2p_out,
    int64_t* __restrict__ tst_out) {
    constexpr int kCoopParts = NW;
    __shared__ float4 s_list[NW][kListCap];
    __shared__ uint32_t s_stack[NW][kStackCap];
    __shared__ float4 s_qlist[NW][QUAD ? 3 * kQuadCap : 1];
    __shared__ double s_part[NW - 1][4][kWave];
    __shared__ int64_t s_cnt[NW - 1][3];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    const uint32_t deal_lo = lvl_off[deal], deal_hi = lvl_off[deal + 1];   // the cells dealt out
    // blocks take the positions of order in strides of the grid
    for (uint32_t pos = blockIdx.x; pos < prm->ngroups; pos += gridDim.x) {
        const uint32_t g = order[pos];
        const int64_t i0 = gbeg[g];
        const int gn = gcnt[g];
        const int64_t i = i0 + lane;
        const bool valid = lane < gn;
        const Body me = bodies[valid ? i : i0];
        const double lox = uniform(wave_min(me.x)), hix = uniform(wave_max(me.x));
        const double loy = uniform(wave_min(me.y)), hiy = uniform(wave_max(me.y));
        const double loz = D == 3 ? uniform(wave_min(me.z)) : 0.0;
        const double hiz = D == 3 ? uniform(wave_max(me.z)) : 0.0;
        const double rx = (lox + hix) * 0.5, ry = (loy + hiy) * 0.5, rz = (loz + hiz) * 0.5;
        const float xi = (float)(me.x - rx), yi = (float)(me.y - ry), zi = (float)(me.z - rz);

        Acc a = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        int64_t nm2p = 0, np2p = 0, ntest = 0;
        walk_group<D, PLAIN, QUAD, kCoopParts, true>(walk, walkq, bodies, bodies32, s_list[wv], s_stack[wv], s_qlist[wv],
                                               lpl_log2, eps2, lox, hix, loy, hiy, loz, hiz, rx, ry, rz, xi, yi, zi,
                                               0u, 1, a, nm2p, np2p, ntest, wv, deal_lo, deal_hi);
        double px = (double)a.sx + (double)a.cx, py = (double)a.sy + (double)a.cy;
        double pz = (double)a.sz + (double)a.cz, pp = (double)a.sp + (double)a.cp;
        if (wv > 0) {
            s_part[wv - 1][0][lane] = px;
            s_part[wv - 1][1][lane] = py;
            s_part[wv - 1][2][lane] = pz;
            s_part[wv - 1][3][lane] = pp;
            if (lane == 0) {
                s_cnt[wv - 1][0] = nm2p;
                s_cnt[wv - 1][1] = np2p;
                s_cnt[wv - 1][2] = ntest;
            }
        }
        __syncthreads();
        if (wv == 0) {
            for (int w = 0; w < kCoopParts - 1; ++w) {
                px += s_part[w][0][lane];
                py += s_part[w][1][lane];
                pz += s_part[w][2][lane];
                pp += s_part[w][3][lane];
                nm2p += s_cnt[w][0];
                np2p += s_cnt[w][1];
                ntest += s_cnt[w][2];
            }
            if (valid) {
                // the body met itself once as a direct entry (in one of the
                // parts): its -m/eps potential term is removed as in the
                // one-wave kernel
                const float mself = (float)me.m;
                pp += (double)(mself * __builtin_amdgcn_rsqf(eps2));
                const int64_t o = perm[i];
                acc[o * D + 0] = (float)((double)G * px);
                acc[o * D + 1] = (float)((double)G * py);
                if (D == 3) acc[o * D + 2] = (float)((double)G * pz);
                pot[o] = (float)((double)G * pp);
                const int64_t lc = nm2p + np2p;
                bcost[o] = lc > 0xffffffffll ? 0xffffffffu : (uint32_t)lc;
            }
            if (lane == 0) {
                m2p_out[g] = nm2p;
                p2p_out[g] = np2p;
                tst_out[g] = ntest;
            }
        }
        __syncthreads();                                  // s_part is reused by the next group
    }
}

// Split walks for small N, where the longest single group otherwise bounds
// the kernel: the walk of group g is cut into kSplitTasks<D> tasks, one per
// (level-1 cell k, child slot j).  If cell k is accepted or is a leaf, task
// (k, 0) walks it and the other slots of k do nothing; if k is opened, task
// (k, j) walks its j-th child.  Together the tasks visit exactly the cells
// and bodies of the unsplit walk (the root is never accepted for a group
// inside it).  Each task writes its FP32 sums for the group's bodies to its
// own slice of part; k_split_reduce adds the slices in FP64 in task order.
template <int D>
constexpr int kSplitTasks = D == 3 ? 64 : 16;

template <int D, bool PLAIN, bool QUAD>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(QUAD ? 4 : 5, 8))) k_walk_force_split(
    const WalkCell* __restrict__ walk, const float4* __restrict__ walkq, const Body* __restrict__ bodies,
    const float4* __restrict__ bodies32, const int32_t* __restrict__ gbeg, const int32_t* __restrict__ gcnt,
    int lpl_log2, float eps2, const DevParams* __restrict__ prm, int64_t n, float4* __restrict__ part,
    unsigned long long* __restrict__ m2p_out, unsigned long long* __restrict__ p2p_out) {
    constexpr int R = D == 3 ? 8 : 4;
    constexpr int T = kSplitTasks<D>;
    __shared__ float4 s_list[kWavesPerBlock][kListCap];
    __shared__ uint32_t s_stack[kWavesPerBlock][kStackCap];
    __shared__ float4 s_qlist[kWavesPerBlock][QUAD ? 3 * kQuadCap : 1];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    const int64_t task = (int64_t)blockIdx.x * kWavesPerBlock + wv;
    const int64_t g = task / T;
    const int t = (int)(task % T);
    if (g >= (int64_t)prm->ngroups) return;
    const int64_t i0 = gbeg[g];
    const int gn = gcnt[g];
    const int64_t i = i0 + lane;
    const bool valid = lane < gn;
    const Body me = bodies[valid ? i : i0];
    const double lox = uniform(wave_min(me.x)), hix = uniform(wave_max(me.x));
    const double loy = uniform(wave_min(me.y)), hiy = uniform(wave_max(me.y));
    const double loz = D == 3 ? uniform(wave_min(me.z)) : 0.0;
    const double hiz = D == 3 ? uniform(wave_max(me.z)) : 0.0;
    const double rx = (lox + hix) * 0.5, ry = (loy + hiy) * 0.5, rz = (loz + hiz) * 0.5;
    const float xi = (float)(me.x - rx), yi = (float)(me.y - ry), zi = (float)(me.z - rz);

    // this task's first batch: one cell or nothing
    uint32_t first = 0;
    int first_len = 0;
    const WalkCell root = walk[0];
    if (root.b < 0) {                                    // the root is a leaf
        first_len = t == 0 ? 1 : 0;
    } else {
        const int k = t / R, j = t % R;
        if (k < root.b) {
            const uint32_t c1 = (uint32_t)root.a + (uint32_t)k;
            const WalkCell w1 = walk[c1];
            const double dxm = fmax(fmax(lox - w1.cx, 0.0), w1.cx - hix);
            const double dym = fmax(fmax(loy - w1.cy, 0.0), w1.cy - hiy);
            double d2 = dxm * dxm + dym * dym;
            if (D == 3) {
                const double dzm = fmax(fmax(loz - w1.cz, 0.0), w1.cz - hiz);
                d2 = d2 + dzm * dzm;
            }
            if (d2 > w1.rcrit2 || w1.b < 0) {
                first = c1;
                first_len = j == 0 ? 1 : 0;
            } else if (j < w1.b) {
                first = (uint32_t)w1.a + (uint32_t)j;
                first_len = 1;
            }
        }
    }
    Acc a = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int64_t nm2p = 0, np2p = 0, ntest = 0;   // tested cells are not kept for split walks
    walk_group<D, PLAIN, QUAD>(walk, walkq, bodies, bodies32, s_list[wv], s_stack[wv], s_qlist[wv], lpl_log2, eps2,
                               lox, hix, loy, hiy, loz, hiz, rx, ry, rz, xi, yi, zi, first, first_len, a, nm2p,
                               np2p, ntest);
    if (valid)
        part[(int64_t)t * n + i] = make_float4(a.sx + a.cx, a.sy + a.cy, a.sz + a.cz, a.sp + a.cp);
    if (lane == 0 && (nm2p | np2p)) {
        atomicAdd(&m2p_out[g], (unsigned long long)nm2p);
        atomicAdd(&p2p_out[g], (unsigned long long)np2p);
    }
}

template <int D>
__global__ void __launch_bounds__(256) k_split_reduce(const float4* __restrict__ part, const Body* __restrict__ bodies,
                                                      const uint32_t* __restrict__ perm, int64_t n, float G,
                                                      float eps2, float* __restrict__ acc, float* __restrict__ pot) {
    constexpr int T = kSplitTasks<D>;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double ax = 0.0, ay = 0.0, az = 0.0, ap = 0.0;
        for (int t = 0; t < T; ++t) {
            const float4 v = part[(int64_t)t * n + i];
            ax += v.x;
            ay += v.y;
            az += v.z;
            ap += v.w;
        }
        // the body met itself once as a direct entry: its -m/eps potential
        // term is removed as in the unsplit kernel
        const float mself = (float)bodies[i].m;
        ap += (double)(mself * __builtin_amdgcn_rsqf(eps2));
        const int64_t o = perm[i];
        acc[o * D + 0] = (float)((double)G * ax);
        acc[o * D + 1] = (float)((double)G * ay);
        if (D == 3) acc[o * D + 2] = (float)((double)G * az);
        pot[o] = (float)((double)G * ap);
    }
}

__global__ void k_zero_u64(unsigned long long* __restrict__ a, unsigned long long* __restrict__ b,
                           unsigned long long* __restrict__ c, int64_t k) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < k; i += (int64_t)gridDim.x * blockDim.x) {
        a[i] = 0ull;
        b[i] = 0ull;
        c[i] = 0ull;
    }
}

// FP32 copy of each cell's traceless quadrupole in level order, two float4
// per cell: (xx, yy, zz, xy), (xz, yz, 0, 0).
__global__ void __launch_bounds__(256) k_quad_pack(const Moments* __restrict__ mom,
                                                   const uint32_t* __restrict__ pre2bfs,
                                                   const DevParams* __restrict__ prm, int64_t cmax,
                                                   float4* __restrict__ walkq) {
    int64_t C = prm->ncells;
    if (C > cmax) C = cmax;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < C; k += (int64_t)gridDim.x * blockDim.x) {
        const Moments& mo = mom[k];
        const size_t b = 2 * (size_t)pre2bfs[k];
        walkq[b] = make_float4((float)mo.Q[0], (float)mo.Q[1], (float)mo.Q[2], (float)mo.Q[3]);
        walkq[b + 1] = make_float4((float)mo.Q[4], (float)mo.Q[5], 0.f, 0.f);
    }
}


// The order in which the persistent waves take the groups of each XCD
// share: runs of consecutive groups, by decreasing cost.  A
// group's cost is the list length that its middle body had in the previous
// force evaluation (bodies are named by their input index, so this survives
// a rebuild; group boundaries move from step to step, so neither a group
// index nor a group's first body, often the previous group's last, does as
// well).  Long walks then start first and the walks still running when a
// share drains are short ones.  Longer runs keep more neighbouring groups,
// which read the same cells and bodies, running side by side in one XCD's
// L2, but they lengthen the tail, which matters less the more groups each
// wave takes.  Runs are max(1, groups / (4 waves)) long, and from 16 groups
// per wave on the groups are taken in key order.  Measured: on a 1M-body
// Plummer sphere (3.5 groups per wave) runs of 1, 4, 16, 64 and 256 groups
// fetched 560, 500, 400, 320 and 275 MB from HBM per launch (280 GB/s at
// most: the kernel is ALU-bound) and took 2.0, 2.11, 2.09, 2.16 and
// 2.19 ms (2.2 ms in key order); on 4.2M bodies of two Plummer spheres (14
// groups per wave) runs of 3 took 1% less than key order; on 16.7M
// clustered bodies (57 groups per wave) single groups took 15.7 ms, runs of
// 14, 16 or 64 14.9-15.3 ms, key order 14.7-15.2 ms.  Only the schedule
// depends on the costs: each group's walk and sums are the same in any order, so stale
// or missing costs cost time, never accuracy.  k_group_order gathers the
// costs of one share's groups and sorts its runs, one share per block (and
// zeroes that share's work counter), by the mean cost of a run in buckets
// of 1/16 of an octave (log2 with four fraction bits);
// places within a bucket are taken with LDS atomics, so they may differ
// from run to run.
constexpr int kOrderBuckets = 512;
constexpr int kOrderThreads = 1024;

__device__ __forceinline__ int cost_bucket(uint32_t v) {
    if (v < 1) return 0;
    const int e = 31 - __builtin_clz(v);
    const uint32_t frac = (e >= 4 ? (v >> (e - 4)) : (v << (4 - e))) & 15u;
    const int b = 16 * e + (int)frac;
    return b < kOrderBuckets ? b : kOrderBuckets - 1;
}

__global__ void __launch_bounds__(kOrderThreads) k_group_order(const uint32_t* __restrict__ bcost,
                                                               const uint32_t* __restrict__ perm,
                                                               const int32_t* __restrict__ gbeg,
                                                               const int32_t* __restrict__ gcnt,
                                                               const DevParams* __restrict__ prm,
                                                               uint32_t* __restrict__ gcost,
                                                               uint16_t* __restrict__ ckey,
                                                               uint32_t* __restrict__ order,
                                                               uint32_t* __restrict__ queue, uint32_t waves) {
    __shared__ uint32_t hist[kOrderBuckets];
    __shared__ uint32_t scan[2][kOrderBuckets];
    const uint32_t NG = prm->ngroups;
    const int x = (int)blockIdx.x;
    const uint32_t lo = (uint32_t)(((uint64_t)NG * x) / kXcd), hi = (uint32_t)(((uint64_t)NG * (x + 1)) / kXcd);
    const uint32_t W = max(waves, 1u);
    const int t = (int)threadIdx.x;
    if (t == 0) queue[x * kQueueStride] = 0u;
    if (NG >= 16u * W) {                                 // key order
        for (uint32_t g = lo + (uint32_t)t; g < hi; g += kOrderThreads) order[g] = g;
        return;
    }
    const uint32_t run = max(1u, NG / (4u * W));
    const uint32_t nc = (hi - lo + run - 1) / run;
    if (t < kOrderBuckets) hist[t] = 0u;
    // the share's group costs, four groups per thread with their loads
    // issued together (three dependent loads each)
    for (uint32_t g0 = lo + (uint32_t)t; g0 < hi; g0 += 4 * kOrderThreads) {
        int32_t gb[4], gc[4];
        uint32_t pb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t g = g0 + u * kOrderThreads;
            gb[u] = g < hi ? gbeg[g] : 0;
            gc[u] = g < hi ? gcnt[g] : 0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) pb[u] = g0 + u * kOrderThreads < hi ? perm[gb[u] + gc[u] / 2] : 0u;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t g = g0 + u * kOrderThreads;
            if (g < hi) gcost[g] = bcost[pb[u]];
        }
    }
    __syncthreads();
    // each run's bucket (kept at its first group's key) and the groups per bucket
    for (uint32_t c = (uint32_t)t; c < nc; c += kOrderThreads) {
        const uint32_t c0 = lo + c * run, c1 = min(hi, c0 + run);
        uint64_t sum = 0;
        for (uint32_t g = c0; g < c1; ++g) sum += gcost[g];
        const uint64_t mean = sum / (c1 - c0);
        const int b = cost_bucket(mean > 0xffffffffull ? 0xffffffffu : (uint32_t)mean);
        ckey[c0] = (uint16_t)b;
        atomicAdd(&hist[b], c1 - c0);
    }
    __syncthreads();
    // inclusive scan over the buckets from the most expensive down
    int cur = 0;
    if (t < kOrderBuckets) scan[0][t] = hist[kOrderBuckets - 1 - t];
    __syncthreads();
    for (int d = 1; d < kOrderBuckets; d <<= 1) {
        if (t < kOrderBuckets) scan[cur ^ 1][t] = scan[cur][t] + (t >= d ? scan[cur][t - d] : 0u);
        cur ^= 1;
        __syncthreads();
    }
    // hist becomes the next free place of each bucket
    if (t < kOrderBuckets) {
        const int r = kOrderBuckets - 1 - t;             // bucket of scan position t
        hist[r] = scan[cur][t] - hist[r];
    }
    __syncthreads();
    // the same runs as above, each read back by the thread that keyed it
    for (uint32_t c = (uint32_t)t; c < nc; c += kOrderThreads) {
        const uint32_t c0 = lo + c * run, c1 = min(hi, c0 + run);
        const uint32_t at = lo + atomicAdd(&hist[ckey[c0]], c1 - c0);
        for (uint32_t g = c0; g < c1; ++g) order[at + (g - c0)] = g;
    }
}

}  // namespace

hipError_t launch_quad_pack(const Moments* mom, const uint32_t* pre2bfs, const DevParams* prm, int64_t cmax,
                            float4* walkq, hipStream_t s) {
    int64_t nb = (cmax + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_quad_pack, dim3((unsigned)nb), dim3(256), 0, s, mom, pre2bfs, prm, cmax, walkq);
    return hipGetLastError();
}

hipError_t launch_walk_force_split(const WalkCell* walk, const float4* walkq, const Body* bodies,
                                   const float4* bodies32, const uint32_t* perm, const int32_t* gbeg,
                                   const int32_t* gcnt, int64_t gmax, int64_t n, int dim, int leaf_cap, float G,
                                   float eps2, const DevParams* prm, float4* part, float* acc, float* pot,
                                   int64_t* m2p, int64_t* p2p, int64_t* tests, bool plain, hipStream_t s) {
    int lpl_log2 = 0;
    while ((1 << lpl_log2) < leaf_cap && lpl_log2 < 6) ++lpl_log2;
    unsigned long long* c1 = reinterpret_cast<unsigned long long*>(m2p);
    unsigned long long* c2 = reinterpret_cast<unsigned long long*>(p2p);
    hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)((gmax + 255) / 256)), dim3(256), 0, s, c1, c2,
                       reinterpret_cast<unsigned long long*>(tests), gmax);
    const int T = dim == 3 ? kSplitTasks<3> : kSplitTasks<2>;
    const unsigned nb = (unsigned)((gmax * T + kWavesPerBlock - 1) / kWavesPerBlock);
#define TC_LAUNCH_SPLIT(DIM, PL, QU)                                                                               \
    hipLaunchKernelGGL((k_walk_force_split<DIM, PL, QU>), dim3(nb), dim3(256), 0, s, walk, walkq, bodies, bodies32, \
                       gbeg, gcnt, lpl_log2, eps2, prm, n, part, c1, c2)
    if (dim == 3 && walkq) {
        if (plain) TC_LAUNCH_SPLIT(3, true, true);
        else TC_LAUNCH_SPLIT(3, false, true);
    } else if (dim == 3) {
        if (plain) TC_LAUNCH_SPLIT(3, true, false);
        else TC_LAUNCH_SPLIT(3, false, false);
    } else {
        if (plain) TC_LAUNCH_SPLIT(2, true, false);
        else TC_LAUNCH_SPLIT(2, false, false);
    }
#undef TC_LAUNCH_SPLIT
    const unsigned rb = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    if (dim == 3)
        hipLaunchKernelGGL(k_split_reduce<3>, dim3(rb), dim3(256), 0, s, part, bodies, perm, n, G, eps2, acc, pot);
    else
        hipLaunchKernelGGL(k_split_reduce<2>, dim3(rb), dim3(256), 0, s, part, bodies, perm, n, G, eps2, acc, pot);
    return hipGetLastError();
}

hipError_t launch_walk_force(const WalkCell* walk, const float4* walkq, const Body* bodies, const float4* bodies32,
                             const uint32_t* perm,
                             const int32_t* gbeg, const int32_t* gcnt, int64_t gmax, uint32_t* order,
                             uint32_t* queue, uint32_t* bcost,
                             int64_t n, int dim, int leaf_cap, float G, float eps2,
                             const DevParams* prm, float* acc, float* pot, int64_t* m2p,
                             int64_t* p2p, int64_t* tests, bool plain, bool share, const uint32_t* lvl_off,
                             hipStream_t s) {
    // as many blocks as can be resident at once (the waves are persistent)
    static int resident[3] = {0, 0, 0};                // 2D, 3D, 3D with quadrupoles
    const int kind = dim == 3 ? (walkq ? 2 : 1) : 0;
    int& res = resident[kind];
    if (res == 0) {
        int dev = 0, cus = 0, per_cu = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = kind == 2   ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_walk_force<3, false, true, 8>, 256, 0)
                : kind == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_walk_force<3, false, false, 8>, 256, 0)
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_walk_force<2, false, false, 8>, 256, 0);
        if (e != hipSuccess) return e;
        res = cus * (per_cu > 0 ? per_cu : 1);
    }
    int64_t want = (gmax + kWavesPerBlock - 1) / kWavesPerBlock;
    if (want > res) want = res;
    if (want < kXcd) want = kXcd;
    const unsigned nb = (unsigned)want;
    int lpl_log2 = 0;                                   // lanes per leaf: next power of two, <= 64
    while ((1 << lpl_log2) < leaf_cap && lpl_log2 < 6) ++lpl_log2;
    // the group order: costs and run keys after the gmax places of order
    // (as the layout reserves), then the counting sort of each share
    uint32_t* gcost = order + gmax;
    uint16_t* ckey = reinterpret_cast<uint16_t*>(order + 2 * gmax);
    hipLaunchKernelGGL(k_group_order, dim3(kXcd), dim3(kOrderThreads), 0, s, (const uint32_t*)bcost, perm, gbeg,
                       gcnt, prm, gcost, ckey, order, queue, (uint32_t)(nb * kWavesPerBlock));
    if (share && n <= coop_max_n(dim)) {
        // one block per group at a time, as many blocks as can be resident
        const int deal = coop_deal_level(n, dim);
        const int nw = coop_waves(n, dim);
#define TC_LAUNCH_COOP_NW(DIM, PL, QU, NW)                                                                          \
    hipLaunchKernelGGL((k_walk_force_coop<DIM, PL, QU, NW>), dim3(nb), dim3(NW * kWave), 0, s, walk, walkq, bodies,  \
                       bodies32, perm, gbeg, gcnt, order, bcost, lvl_off, deal, lpl_log2, G, eps2, prm, acc, pot,  \
                       m2p, p2p, tests)
#define TC_LAUNCH_COOP(DIM, PL, QU)                                                                                 \
    do {                                                                                                            \
        if (nw == 8) TC_LAUNCH_COOP_NW(DIM, PL, QU, 8);                                                             \
        else TC_LAUNCH_COOP_NW(DIM, PL, QU, 4);                                                                     \
    } while (0)
        if (dim == 3 && walkq) {    // quadrupole lists: four waves (eight would take 82 KB of LDS)
            if (plain) TC_LAUNCH_COOP_NW(3, true, true, 4);
            else TC_LAUNCH_COOP_NW(3, false, true, 4);
        } else if (dim == 3) {
            if (plain) TC_LAUNCH_COOP(3, true, false);
            else TC_LAUNCH_COOP(3, false, false);
        } else {
            if (plain) TC_LAUNCH_COOP(2, true, false);
            else TC_LAUNCH_COOP(2, false, false);
        }
#undef TC_LAUNCH_COOP
#undef TC_LAUNCH_COOP_NW
        return hipGetLastError();
    }
    // With two to four groups per resident wave (counting n/64 groups) the
    // list sums go in rounds of 4 entries, else 8: the same sums either
    // way, and measured per force kernel (3D Plummer, rounds of 4 against
    // 8): 1.89 against 1.94 ms at 1M bodies, 2.29 against 2.32 at 1.25M,
    // but 0.86 against 0.85 at 400,000, 7.89 against 7.86 at 4M, 16.45
    // against 16.19 at 16.7M and 0.1145 against 0.1140 ms for the
    // 262,144-body disk.
    const int64_t groups_lo = (n + kGroup - 1) / kGroup, waves_all = (int64_t)nb * kWavesPerBlock;
    const bool short_rounds = groups_lo > 2 * waves_all && groups_lo <= 4 * waves_all;
#define TC_LAUNCH_WF_STEP(DIM, PL, QU, ST)                                                                           \
    hipLaunchKernelGGL((k_walk_force<DIM, PL, QU, ST>), dim3(nb), dim3(256), 0, s, walk, walkq, bodies, bodies32,  \
                       perm, gbeg, gcnt, order, queue, bcost, lpl_log2, G, eps2, prm, acc, pot, m2p, p2p, tests)
#define TC_LAUNCH_WF(DIM, PL, QU)                                                                                \
    do {                                                                                                         \
        if (short_rounds) TC_LAUNCH_WF_STEP(DIM, PL, QU, 4);                                                     \
        else TC_LAUNCH_WF_STEP(DIM, PL, QU, 8);                                                                  \
    } while (0)
    if (dim == 3 && walkq) {
        if (plain) TC_LAUNCH_WF(3, true, true);
        else TC_LAUNCH_WF(3, false, true);
    } else if (dim == 3) {
        if (plain) TC_LAUNCH_WF(3, true, false);
        else TC_LAUNCH_WF(3, false, false);
    } else {
        if (plain) TC_LAUNCH_WF(2, true, false);
        else TC_LAUNCH_WF(2, false, false);
    }
#undef TC_LAUNCH_WF
#undef TC_LAUNCH_WF_STEP
    return hipGetLastError();
}

}  // namespace tc
