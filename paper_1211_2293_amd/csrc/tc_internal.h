// Internal declarations shared by the HIP translation units of libtc.
// Not part of the public ABI (include/tc.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace tc {

constexpr int kWave = 64;           // CDNA wavefront width
constexpr int kGroup = 64;          // bodies per walk group = one wave
constexpr int kMaxLeafCap = 256;    // the largest leaf_cap (TC_MAX_LEAF_CAP)
// Radix-sort tiles: 256 threads x sort_per(n) keys.  One block per tile
// and few blocks leave the passes latency-bound, so smaller sorts use
// smaller tiles (measured per pass: 1M keys 16.0 us with 4096-key tiles,
// 16.6 with 2048, 18.6 with 1024; 262k keys 14.2 us with 4096, 9.4 with
// 2048, 7.3 with 1024): the largest tile that still gives 256 tiles.
inline int sort_per(int64_t n) { return n >= (int64_t)256 * 4096 ? 16 : n >= (int64_t)256 * 2048 ? 8 : 4; }
inline int64_t sort_tiles(int64_t n) { return (n + 256 * sort_per(n) - 1) / (256 * sort_per(n)); }
// Tiles a histogram buffer must hold for any sort of at most n keys.
inline int64_t sort_tiles_max(int64_t n) { return (n + 1023) / 1024; }
constexpr int kScanTile = 4096;     // elements per scan tile
constexpr int kDiagBlocks = 512;    // fixed partial count of the FP64 diagnostics
constexpr int kCluster = 1024;      // walk groups never straddle a cell of <= kCluster bodies
constexpr int kXcd = 8;             // XCDs per MI355X: one work queue each
constexpr int kQueueStride = 64;    // work-queue counters 256 B apart (own cache lines)

// Status bits raised by kernels into the workspace's status word.
constexpr uint32_t kFlagNonFinite = 1u;
constexpr uint32_t kFlagOverflow = 2u;   // cell bound exceeded (never expected)
constexpr uint32_t kFlagBadIndex = 4u;   // an index argument outside its array

inline int levels_for(int dim) { return dim == 3 ? 21 : 31; }

// A body in key order: FP64 position and mass (z = 0 in 2D).
struct __align__(32) Body {
    double x, y, z, m;
};

// Topology of one cell (pre-order index k).
struct __align__(16) Cell {
    uint64_t prefix;   // key prefix: the top level*dim bits of its bodies' keys
    int32_t begin;     // first sorted body
    int32_t count;     // number of bodies
    int32_t skip;      // pre-order index just past the subtree
    int32_t parent;    // -1 for the root
    int32_t level;
    int32_t leaf_nch;  // bit 31: leaf; low bits: number of children
};

// FP64 moments of one cell: total mass, mass-weighted position sum, centre
// of mass and traceless quadrupole (xx, yy, zz, xy, xz, yz).
struct __align__(16) Moments {
    double M;
    double S[3];
    double com[3];
    double Q[6];
    double pad;
};

// What the walk reads per cell, in level order (breadth-first: all cells of
// level 0, then level 1, ...; within a level in pre-order), so that the
// children of every cell are contiguous.  48 bytes, one lane per cell.
//   a = leaf ? first sorted body : level-order index of the first child
//   b = leaf ? (body count | 0x80000000) : number of children
struct __align__(16) WalkCell {
    double cx, cy, cz;   // centre of mass (FP64)
    double rcrit2;       // squared opening radius for the current theta
    float m;             // total mass, FP32
    int32_t a;
    int32_t b;
    int32_t pad;
};

// Device-side scalars computed by the kernels.
struct DevParams {
    double lo[3];        // root cube corner
    double size;         // root cube side (a power of two)
    double scale;        // 2^L / size
    uint32_t ncells;
    uint32_t status;     // kFlag* bits, sticky until the next build
    uint32_t ngroups;    // walk groups of the current tree
    uint32_t pad;
};

// Carve-up of the caller's workspace.
struct Layout {
    int64_t n;
    int dim, leaf_cap;
    int64_t cmax;        // cell bound
    int64_t groups;      // ceil(n / 64)
    int64_t sort_tiles;
    int64_t scan_tiles;
    size_t off_params, off_keys_a, off_keys_b, off_idx_a, off_idx_b, off_bodies, off_range,
        off_nper, off_cstart, off_scan_part, off_hist, off_digit_tot, off_cells, off_mom,
        off_walk, off_mom_lvl, off_kids, off_bodies32, off_acc, off_pot, off_m2p, off_p2p, off_bbox_part, off_diag_part,
        off_diag_out, off_lvl_idx_b, off_pre2bfs,
        off_lvl_hist, off_gper, off_goff, off_gscan_part, off_gbeg, off_gcnt, off_queue, off_gorder, off_bcost, off_lvl_off, off_inv_perm, off_rcount, off_roffs,
        off_rscan_part, off_mlp, off_rcp2, off_nlearn, off_nfall, off_pb_cnt, off_pb_off, off_pb_part, off_walkq, off_split, off_tests, total;
    int64_t lvl_tiles;   // radix tiles over cmax cells (level sort)
    int64_t gmax;        // bound on walk groups
    int64_t cscan_tiles; // scan tiles over cmax cells
};

Layout make_layout(int64_t n, int dim, int leaf_cap);

// ---- launchers (all enqueue on `s`, return hipSuccess or the launch error)
// build.hip
// Also packs the input into (x, y, z, m) records (float4, or double4 for FP64
// input; n of them at `packed`) for launch_gather.
hipError_t launch_bbox(const void* pos, const void* mass, int64_t n, int dim, int f64,
                       double* part, void* packed, DevParams* prm, hipStream_t s);
hipError_t launch_keys(const void* pos, int64_t n, int dim, int f64, const DevParams* prm,
                       uint64_t* keys, uint32_t* idx, hipStream_t s);
// LSD radix sort (stable) of the low key_bits bits; idx_a / idx_b may both be
// null for keys without a payload.
// hist holds 256 x sort_tiles_max(n) counts.
hipError_t launch_sort(uint64_t* keys_a, uint32_t* idx_a, uint64_t* keys_b, uint32_t* idx_b,
                       int64_t n, int key_bits, uint32_t* hist, uint32_t* digit_tot, hipStream_t s);
hipError_t launch_gather(const void* packed, const uint32_t* perm, int64_t n, int f64, Body* bodies,
                         float4* bodies32, hipStream_t s);
hipError_t launch_topology(const uint64_t* keys, int64_t n, int dim, int leaf_cap,
                           uint32_t* range, uint32_t* nper, uint32_t* cstart,
                           uint32_t* scan_part, int64_t scan_tiles, Cell* cells,
                           int64_t cmax, DevParams* prm, hipStream_t s);
// Level order (one radix pass by level over the live cells): bfs2pre and
// pre2bfs, and lvl_off, where each level starts (levels 0..L and the end).
// cells_est, an estimate of the live cells (any value works), sets the tile.
hipError_t launch_level_order(const Cell* cells, int64_t cmax, int64_t cells_est, int dim, const DevParams* prm, uint32_t* bfs2pre,
                              uint32_t* hist, uint32_t* digit_tot, uint32_t* pre2bfs, uint32_t* lvl_off,
                              hipStream_t s);
hipError_t launch_groups(const Cell* cells, int64_t cmax, uint32_t* gper, uint32_t* goff, uint32_t* scan_part,
                         int64_t scan_tiles, int32_t* gbeg, int32_t* gcnt, int64_t gmax, DevParams* prm,
                         hipStream_t s);
hipError_t launch_moments(const Cell* cells, const Body* bodies, int dim, int64_t cmax,
                          const uint32_t* bfs2pre, const uint32_t* pre2bfs, const uint32_t* lvl_off,
                          const DevParams* prm, Moments* mom, Moments* mom_lvl, uint2* kids, WalkCell* walk,
                          const uint32_t* hint, hipStream_t s);
// hint (host, nullable): the level offsets (levels 0..L and the end) of an
// earlier tree.  They shape the launches only: the deepest levels that held
// few cells go to one single-block launch, the others get grids sized by
// their earlier counts.  Any tree is still done in full.
hipError_t launch_mac(const Cell* cells, const Moments* mom, int dim, double theta, int64_t cmax,
                      const uint32_t* pre2bfs, WalkCell* walk, double* rc_out, const DevParams* prm,
                      hipStream_t s);
hipError_t launch_export(const Cell* cells, const Moments* mom, int dim, int64_t cmax,
                         const DevParams* prm, int32_t* level, uint64_t* prefix, int32_t* begin,
                         int32_t* count, int32_t* parent, int32_t* skip, int32_t* nch,
                         int32_t* leaf, double* M, double* com, double* Q, hipStream_t s);
// force.hip
// order: room for 2 gmax uint32 (places, costs) and gmax uint16 keys; bcost:
// n uint32 per-body list lengths, written for the next call's schedule.
hipError_t launch_walk_force(const WalkCell* walk, const float4* walkq, const Body* bodies, const float4* bodies32,
                             const uint32_t* perm,
                             const int32_t* gbeg, const int32_t* gcnt, int64_t gmax, uint32_t* order,
                             uint32_t* queue, uint32_t* bcost, int64_t n, int dim, int leaf_cap, float G, float eps2,
                             const DevParams* prm, float* acc, float* pot, int64_t* m2p,
                             int64_t* p2p, int64_t* tests, bool plain, bool share, const uint32_t* lvl_off,
                             hipStream_t s);
hipError_t launch_scan_u32(const uint32_t* in, int64_t n, uint32_t* out, uint32_t* part, int64_t tiles,
                           hipStream_t s);
// closure.hip
struct MlpState;
hipError_t launch_direct64(const Body* bodies, const uint32_t* inv_perm, int64_t n, const int32_t* targets, int nt,
                           double eps2, double G, DevParams* prm, double* acc, double* pot, hipStream_t s);
// Split walks pay off for small n only (measured on 3D Plummer spheres:
// 1.6x faster force evaluations at 2,000 bodies, 1.14x at 10,000, 0.64x at
// 16,384; on 2D disks 1.25x at 16,384, 0.90x at 32,768).  The shared walks
// below are faster still, so split walks are used only when asked for
// (tc_set_split(ctx, 2)), for n at most split_max_n(dim); the workspace holds
// their partial sums.
constexpr int64_t kSplitMaxN3 = 12288;
constexpr int64_t kSplitMaxN2 = 24576;
inline int64_t split_max_n(int dim) { return dim == 3 ? kSplitMaxN3 : kSplitMaxN2; }
// Up to coop_max_n(dim), one block of waves shares each group's walk
// (k_walk_force_coop), dealing out the cells of level coop_deal_level;
// beyond, one wave per group.  Measured (force evaluation, one wave / shared):
// 3D Plummer 0.160 / 0.073 ms at 2,000 bodies, 0.402 / 0.168 at 10,000,
// 0.473 / 0.278 at 65,536, 0.494 / 0.450 at 131,072, 0.663 / 0.807 at
// 262,144; 2D disk 0.111 / 0.052 at 5,000, 0.098 / 0.049 at 32,768,
// 0.118 / 0.103 at 131,072, 0.125 / 0.179 at 262,144.  tc_set_split(ctx, 0)
// turns it off; tc_set_split(ctx, 2) uses the split walks (above) for
// n <= split_max_n(dim) instead.
constexpr int64_t kCoopMaxN3 = 163840;
constexpr int64_t kCoopMaxN2 = 163840;
inline int64_t coop_max_n(int dim) { return dim == 3 ? kCoopMaxN3 : kCoopMaxN2; }
// Waves sharing each group's walk: eight for the smaller systems, where
// even a block per group leaves most of the GPU idle, else four.  Measured
// (force kernel, four / eight waves): 3D Plummer 0.175 / 0.123 ms at 10,000
// bodies, 0.196 / 0.147 at 20,000, 0.213 / 0.183 at 30,000, 0.238 / 0.258
// at 50,000, 0.536 / 0.690 at 163,840; 2D disk 0.046 / 0.038 at 20,000,
// 0.048 / 0.044 at 30,000, 0.063 / 0.063 at 50,000, 0.121 / 0.159 at
// 163,840.  Walks with quadrupole lists always use four (eight would need
// 82 KB of LDS).
inline int coop_waves(int64_t n, int dim) { return n <= 36000 ? 8 : 4; }
inline int coop_deal_level(int64_t n, int dim) {
    if (dim == 3) return n < 8192 ? 5 : 6;
    return n < 8192 ? 5 : n < 65536 ? 6 : 7;
}
hipError_t launch_walk_force_split(const WalkCell* walk, const float4* walkq, const Body* bodies,
                                   const float4* bodies32, const uint32_t* perm, const int32_t* gbeg,
                                   const int32_t* gcnt, int64_t gmax, int64_t n, int dim, int leaf_cap, float G,
                                   float eps2, const DevParams* prm, float4* part, float* acc, float* pot,
                                   int64_t* m2p, int64_t* p2p, int64_t* tests, bool plain, hipStream_t s);
hipError_t launch_quad_pack(const Moments* mom, const uint32_t* pre2bfs, const DevParams* prm, int64_t cmax,
                            float4* walkq, hipStream_t s);
// perbody.hip
hipError_t launch_pb_count(const WalkCell* walk, const Body* bodies, int64_t n, int dim, uint32_t* counts,
                           uint64_t* offs, uint64_t* part, hipStream_t s);
hipError_t launch_pb_write_sum(const WalkCell* walk, const Body* bodies, const uint32_t* perm, int64_t n, int dim,
                               const uint64_t* offs, uint32_t* lists, int64_t cap, int64_t cbound, float G,
                               float eps2, float* acc, float* pot, hipStream_t s);
hipError_t launch_inverse_perm(const uint32_t* perm, int64_t n, uint32_t* inv, hipStream_t s);
hipError_t launch_residuals(bool write, const WalkCell* walk, const Body* bodies, const Cell* cells,
                            const Moments* mom, const uint32_t* bfs2pre, const uint32_t* inv_perm,
                            DevParams* prm, int64_t n, const int32_t* targets, int nt, double eps2,
                            uint32_t* counts, const uint32_t* offs, int64_t cap, float* feat, float* y,
                            int32_t* cell_out, hipStream_t s);
hipError_t launch_mlp_load(MlpState* st, const float* params, hipStream_t s);
hipError_t launch_mlp_get(const MlpState* st, float* params, hipStream_t s);
hipError_t launch_mlp_forward(const MlpState* st, const float* feat, int64_t nrows, const int32_t* idx, int64_t nb,
                              float* yhat, uint32_t* status, hipStream_t s);
hipError_t launch_mlp_step(MlpState* st, const float* feat, const float* y, int64_t nrows, const int32_t* idx,
                           int64_t nb, float lr, int step, float* grad_out, uint32_t* status, hipStream_t s);
// learned.hip
hipError_t launch_walk_force_learned(const WalkCell* walk, const double* rcp2, const Body* bodies,
                                     const float4* bodies32, const Cell* cells, const Moments* mom,
                                     const uint32_t* bfs2pre, const uint32_t* perm, const int32_t* gbeg,
                                     const int32_t* gcnt, int64_t gmax, uint32_t* queue, const MlpState* st,
                                     int leaf_cap, float G, float eps2, float tau, int64_t n,
                                     const DevParams* prm, float* acc, float* pot, int64_t* m2p, int64_t* p2p,
                                     int64_t* learned, int64_t* fallback, hipStream_t s);
// fmm.hip
// Geometry of a cell for the fast multipole method: its geometric centre
// (the local expansion's centre) and the radii bounding its bodies about
// that centre (rhoA) and about its centre of mass (rhoB).
struct __align__(16) FmmGeo {
    double z[3];
    double rhoA, rhoB;
    double pad[3];
};
// What the traversal reads of a cell, in level order: centre, centre of
// mass, the two radii, its first child (level order; children are
// contiguous there), child count with bit 31 set for a leaf, and level.
constexpr int kFmmMaxBlocks = 4096;   // blocks per traversal launch
struct __align__(16) DttCell {
    double z[3];
    double com[3];
    double rhoA, rhoB;
    int32_t child, nch_leaf, level, pre;   // pre: the cell's pre-order index
};
hipError_t launch_fmm_geo(const Cell* cells, const Moments* mom, const WalkCell* walk, const uint32_t* pre2bfs,
                          const DevParams* prm, int64_t cmax, FmmGeo* geo, DttCell* dc, hipStream_t s);
hipError_t launch_fmm_radii(const Cell* cells, const Moments* mom, const Body* bodies, const WalkCell* walk,
                            const uint32_t* bfs2pre, const uint32_t* lvl_off, int level, int64_t count, FmmGeo* geo,
                            DttCell* dc, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, hipStream_t s);
hipError_t launch_fmm_dtt(const DttCell* dc, double theta, const uint64_t* fin, int64_t nin, uint64_t* fout,
                          int64_t capf, uint64_t* m2l, int64_t capm, uint64_t* p2p, int64_t capp,
                          unsigned long long* ctr, uint32_t* bt, unsigned long long* base, hipStream_t s);
hipError_t launch_fmm_offsets(const uint64_t* keys, int64_t n, int64_t C, uint32_t* off, hipStream_t s);
hipError_t launch_fmm_m2l(const Moments* mom, const FmmGeo* geo, const DevParams* prm, int64_t cmax,
                          const uint64_t* keys, const uint32_t* off, double eps2, double* lam,
                          hipStream_t s);
hipError_t launch_fmm_l2l(const Cell* cells, const FmmGeo* geo, const uint32_t* bfs2pre, const uint32_t* lvl_off,
                          int level, int64_t count, double* lam, hipStream_t s);
hipError_t launch_fmm_tasks(const Cell* cells, const uint32_t* poff, const DevParams* prm, int64_t cmax,
                            uint32_t* ntask, uint32_t* nslot, hipStream_t s);
hipError_t launch_fmm_tasks_fill(const uint32_t* toff, const DevParams* prm, int64_t cmax, uint32_t* task,
                                 hipStream_t s);
hipError_t launch_fmm_leaf(const Cell* cells, const Body* bodies, const float4* bodies32, const uint32_t* perm,
                           const FmmGeo* geo, const double* lam, const uint64_t* pkeys, const uint32_t* poff,
                           const uint32_t* task, const uint32_t* toff, const uint32_t* soff, int64_t ntasks,
                           double* part, const DevParams* prm, int64_t cmax, float G, float eps2, float* acc,
                           float* pot, hipStream_t s);
hipError_t launch_fmm_unpack(const uint64_t* keys, int64_t n, int32_t* out, hipStream_t s);
// step.hip
hipError_t launch_kick_drift(void* pos, void* vel, const float* acc, int64_t n, int dim, int f64,
                             double dt, hipStream_t s);
hipError_t launch_kick(void* vel, const float* acc, int64_t n, int dim, int f64, double dt,
                       hipStream_t s);
hipError_t launch_diag(const void* mass, const void* vel, const float* acc, const float* pot,
                       int64_t n, int dim, int f64, double* part, double* out, hipStream_t s);

// Grid size for grid-stride loops over `work` items with 256-thread blocks.
inline unsigned grid_for(int64_t work, int64_t cap = 16384) {
    int64_t b = (work + 255) / 256;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

}  // namespace tc
