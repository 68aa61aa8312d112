// C ABI of the treecode library (declared in include/tc.h): argument and
// call-order checks, the carve-up of the caller's workspace, and the
// sequence of launches for each call.  The call order mirrors the client
// program of §3.2 (construct the tree, build the lists, compute the forces,
// move the bodies).
#include "tc.h"
#include "tc_internal.h"
#include "closure.h"

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

using namespace tc;

// Device scratch for tc_forces_noalloc: the workspace of callers that cannot
// allocate device memory.  Every GPU the library runs on holds its own copy
// until the process ends.  In host code this name is only a handle for
// hipGetSymbolAddress; its device address is looked up once per device.
static __device__ __align__(256) uint8_t scratch[TC_NOALLOC_SCRATCH_BYTES];

namespace {

enum State { kNone = 0, kBuilt = 1, kMoments = 2, kWalked = 3, kForced = 4 };

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

thread_local char g_errbuf[256];

}  // namespace

namespace tc {

Layout make_layout(int64_t n, int dim, int leaf_cap) {
    Layout l;
    memset(&l, 0, sizeof(l));
    l.n = n;
    l.dim = dim;
    l.leaf_cap = leaf_cap;
    l.cmax = (int64_t)levels_for(dim) * (n / (leaf_cap + 1)) + n + 1;
    l.groups = (n + kGroup - 1) / kGroup;
    l.sort_tiles = sort_tiles_max(n);
    l.scan_tiles = (n + kScanTile - 1) / kScanTile;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    l.off_params = take(sizeof(DevParams));
    l.off_keys_a = take(8 * (size_t)n);
    l.off_keys_b = take(8 * (size_t)n);
    l.off_idx_a = take(4 * (size_t)n);
    l.off_idx_b = take(4 * (size_t)n);
    l.off_bodies = take(sizeof(Body) * (size_t)n);
    l.off_bodies32 = take(16 * (size_t)n);
    l.off_range = take(4 * (size_t)n);
    l.off_nper = take(4 * (size_t)n);
    l.off_cstart = take(4 * (size_t)(n + 1));
    l.off_scan_part = take(4 * (size_t)l.scan_tiles);
    l.off_hist = take(4 * 256 * (size_t)l.sort_tiles);
    l.off_digit_tot = take(4 * 256);
    l.off_cells = take(sizeof(Cell) * (size_t)l.cmax);
    l.off_mom = take(sizeof(Moments) * (size_t)l.cmax);
    l.off_walk = take(sizeof(WalkCell) * (size_t)l.cmax);
    l.off_mom_lvl = take(sizeof(Moments) * (size_t)l.cmax);   // level-order copy for the moments pass
    // ... and, earlier in each build, the packed input records (cmax > n)
    static_assert(sizeof(Moments) >= sizeof(double4), "packed records must fit the level-order buffer");
    l.off_kids = take(8 * (size_t)l.cmax);
    l.off_acc = take(4 * (size_t)n * dim);
    l.off_pot = take(4 * (size_t)n);
    l.off_m2p = 0;   // placed after the group bound is known
    l.off_p2p = 0;
    l.off_bbox_part = take(7 * 8 * 1024);
    l.off_diag_part = take(8 * 8 * (size_t)kDiagBlocks);
    l.off_diag_out = take(8 * 8);
    l.lvl_tiles = sort_tiles_max(l.cmax);
    l.off_lvl_idx_b = take(4 * (size_t)l.cmax);
    l.off_pre2bfs = take(4 * (size_t)l.cmax);
    l.off_lvl_hist = take(4 * 256 * (size_t)l.lvl_tiles);
    // walk groups: at most ceil(n/64) + (number of cluster cells); a cluster
    // cell's parent holds > kCluster bodies, and such parents are disjoint
    // within a level
    const int64_t clusters = (int64_t)(1 << dim) * levels_for(dim) * (n / (kCluster + 1)) + 1;
    l.gmax = (n + kGroup - 1) / kGroup + (clusters < n ? clusters : n);
    l.cscan_tiles = (l.cmax + kScanTile - 1) / kScanTile;
    l.off_gper = take(4 * (size_t)l.cmax);
    l.off_goff = take(4 * (size_t)(l.cmax + 1));
    l.off_gscan_part = take(4 * (size_t)l.cscan_tiles);
    l.off_gbeg = take(4 * (size_t)l.gmax);
    l.off_gcnt = take(4 * (size_t)l.gmax);
    l.off_queue = take(4 * kQueueStride * kXcd);
    l.off_gorder = take(10 * (size_t)l.gmax);   // order and costs (u32), run keys (u16)
    l.off_bcost = take(4 * (size_t)n);
    l.off_lvl_off = take(4 * 64);
    l.off_inv_perm = take(4 * (size_t)n);
    l.off_rcount = take(4 * (size_t)kResidMaxTargets);
    l.off_roffs = take(4 * (size_t)(kResidMaxTargets + 1));
    l.off_rscan_part = take(4 * (size_t)((kResidMaxTargets + kScanTile - 1) / kScanTile));
    l.off_mlp = take(sizeof(MlpState));
    l.off_rcp2 = take(8 * (size_t)l.cmax);
    l.off_m2p = take(8 * (size_t)l.gmax);
    l.off_p2p = take(8 * (size_t)l.gmax);
    l.off_tests = take(8 * (size_t)l.gmax);
    l.off_nlearn = take(8 * (size_t)l.gmax);
    l.off_nfall = take(8 * (size_t)l.gmax);
    l.off_pb_cnt = take(4 * (size_t)n);
    l.off_pb_off = take(8 * (size_t)(n + 1));
    l.off_pb_part = take(8 * (size_t)((n + 4095) / 4096));
    l.off_walkq = take(32 * (size_t)l.cmax);
    // partial sums of the split walk (64 tasks per group in 3D, 16 in 2D)
    l.off_split = n <= split_max_n(dim) ? take(16 * (size_t)(dim == 3 ? 64 : 16) * (size_t)n) : 0;
    l.total = off;
    return l;
}

}  // namespace tc

struct tc_ctx {
    int dim = 3;
    hipStream_t stream = nullptr;
    uint8_t* ws = nullptr;
    size_t ws_bytes = 0;
    Layout lay;
    int state = kNone;
    const void* mass = nullptr;
    int dtype = TC_F32;
    int64_t n = 0;
    int leaf_cap = 0;
    double theta = 0.0, G = 1.0, eps = 0.0;
    bool theta_set = false;    // a tc_walk fixed theta (the plain walk's)
    bool radii_plain = false;  // the walk records hold the opening radii of theta
    // the learned walk in tc_leapfrog (tc_set_closure)
    bool closure = false;
    double cl_theta_l = 0.0, cl_theta_p = 0.0, cl_tau = 0.0;
    bool timing = false;
    std::vector<hipEvent_t> ev_pending;   // (start, stop) pairs not yet summed
    // per-stage timing (tc_set_stage_timing): events around each stage
    struct StageEv {
        int stage;
        hipEvent_t a, b;
    };
    bool stage_timing = false;
    std::vector<StageEv> st_pending;
    double st_ms[TC_NSTAGES] = {};
    int64_t st_count[TC_NSTAGES] = {};
    std::vector<hipEvent_t> ev_pool;
    double t_total_ms = 0.0;
    int64_t t_launches = 0;
    hipError_t last_hip = hipSuccess;
    int mlp_step = 0;          // Adam steps since the last tc_mlp_load
    bool mlp_loaded = false;
    // the pre-force part of tc_leapfrog as a replayed graph (see tc_leapfrog)
    bool use_graph = false;
    bool capturing = false;    // inside the graph capture of the pre-force part
    bool no_alloc = false;     // inside tc_forces_noalloc: no host copies that need pinned memory
    // Level sizes of an earlier tree, for the moments pass: each build copies
    // its level offsets to pinned host memory behind an event; a later call
    // takes them once the event has completed.  Only launch shapes depend
    // on them, never results.
    uint32_t* lvl_host = nullptr;
    hipEvent_t lvl_ev = nullptr;
    bool lvl_pending = false;
    bool have_hint = false;    // lvl_hint holds the last harvested build's level offsets
    uint32_t lvl_hint[64] = {};
    bool plain_acc = false;    // uncompensated running sums (precision study)
    int mp_order = 1;          // 1: monopole cells, 2: with quadrupole terms (3D)
    int split = 1;             // 0: one wave per group; 1: shared walks (coop); 2: split walks up to split_max_n
    bool tests_kept = false;   // the last force evaluation counted each group's tested cells
    bool pb_counted = false;   // per-body list lengths of the current walk are known
    int64_t pb_total = 0;
    // the fast multipole plan (tc_fmm_plan) in the caller's buffer
    bool fmm_planned = false;
    uint8_t* fmm_buf = nullptr;
    int64_t fmm_ncells = 0, fmm_m2l = 0, fmm_p2p = 0, fmm_capf = 0, fmm_capm = 0, fmm_capp = 0, fmm_ntasks = 0;
    uint32_t fmm_lvl_off[64] = {};
    hipStream_t gstream = nullptr;
    hipEvent_t g_in = nullptr, g_out = nullptr;
    hipGraphExec_t g_exec = nullptr;
    struct GraphKey {
        const void *pos, *vel, *mass;
        const uint8_t* ws;
        int64_t n;
        int dim, dtype, leaf_cap;
        double dt, theta;
        bool closure;
        double theta_l, theta_p;
        bool operator==(const GraphKey& o) const {
            return pos == o.pos && vel == o.vel && mass == o.mass && ws == o.ws && n == o.n && dim == o.dim &&
                   dtype == o.dtype && leaf_cap == o.leaf_cap && dt == o.dt && theta == o.theta &&
                   closure == o.closure && theta_l == o.theta_l && theta_p == o.theta_p;
        }
    } g_key{};

    template <typename T>
    T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
    DevParams* prm() const { return at<DevParams>(lay.off_params); }
};

namespace {

int hip_fail(tc_ctx* ctx, hipError_t e) {
    if (ctx) ctx->last_hip = e;
    snprintf(g_errbuf, sizeof(g_errbuf), "HIP failure: %s", hipGetErrorString(e));
    return TC_EHIP;
}

// An internal invariant that failed (never expected): reported as TC_EHIP
// with its description for tc_strerror.
int internal_fail(const char* what) {
    snprintf(g_errbuf, sizeof(g_errbuf), "internal error: %s", what);
    return TC_EHIP;
}

#define TC_HIP(ctx, expr)                                  \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return hip_fail((ctx), e_);  \
    } while (0)

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

static_assert(TC_MAX_LEAF_CAP == kMaxLeafCap, "the topology pass sizes its LDS window by kMaxLeafCap");

bool valid_sizes(int64_t n, int dim, int leaf_cap) {
    if (n < 1 || n > TC_MAX_N) return false;
    if (dim != 2 && dim != 3) return false;
    if (leaf_cap < 1 || leaf_cap > TC_MAX_LEAF_CAP) return false;
    const int64_t cmax = (int64_t)levels_for(dim) * (n / (leaf_cap + 1)) + n + 1;
    return cmax < ((int64_t)1 << 28);   // level-order indices are packed into 28 bits
}

hipEvent_t pooled_event(tc_ctx* ctx) {
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Events around one stage's launches on stream s when stage timing is on
// (not inside a graph capture); summed by tc_get_stage_timing.
struct StageScope {
    tc_ctx* ctx;
    int stage;
    hipStream_t s;
    hipEvent_t a = nullptr;
    StageScope(tc_ctx* c, int st, hipStream_t s_) : ctx(c), stage(st), s(s_) {
        if (!ctx->stage_timing || ctx->capturing) return;
        a = pooled_event(ctx);
        if (a && hipEventRecord(a, s) != hipSuccess) {
            ctx->ev_pool.push_back(a);
            a = nullptr;
        }
    }
    ~StageScope() {
        if (!a) return;
        hipEvent_t b = pooled_event(ctx);
        if (b && hipEventRecord(b, s) == hipSuccess) {
            ctx->st_pending.push_back({stage, a, b});
            return;
        }
        ctx->ev_pool.push_back(a);
        if (b) ctx->ev_pool.push_back(b);
    }
};

// Everything tc_build enqueues, after its checks.
// Take the level offsets of the last build whose copy has arrived on the
// host (never waits).
void harvest_depth(tc_ctx* ctx) {
    if (!ctx->lvl_pending || hipEventQuery(ctx->lvl_ev) != hipSuccess) return;
    const int L = levels_for(ctx->dim);
    for (int l = 0; l <= L + 1; ++l) ctx->lvl_hint[l] = ctx->lvl_host[l];
    ctx->have_hint = true;
    ctx->lvl_pending = false;
}

int do_build(tc_ctx* ctx, const void* pos, const void* mass, int64_t n, int leaf_cap, int dtype, hipStream_t s) {
    const int dim = ctx->dim;
    ctx->lay = make_layout(n, dim, leaf_cap);
    const Layout& l = ctx->lay;
    const int f64 = dtype == TC_F64;
    DevParams* prm = ctx->prm();
    {
        StageScope st_(ctx, TC_STAGE_BBOX, s);
        // the packed records live in the moments pass's level-order buffer
        // (at least 112 B per body, unused until the moments pass)
        TC_HIP(ctx, launch_bbox(pos, mass, n, dim, f64, ctx->at<double>(l.off_bbox_part),
                                ctx->at<char>(l.off_mom_lvl), prm, s));
    }
    {
        StageScope st_(ctx, TC_STAGE_KEYS, s);
        TC_HIP(ctx, launch_keys(pos, n, dim, f64, prm, ctx->at<uint64_t>(l.off_keys_a),
                                ctx->at<uint32_t>(l.off_idx_a), s));
    }
    {
        StageScope st_(ctx, TC_STAGE_SORT, s);
        TC_HIP(ctx, launch_sort(ctx->at<uint64_t>(l.off_keys_a), ctx->at<uint32_t>(l.off_idx_a),
                                ctx->at<uint64_t>(l.off_keys_b), ctx->at<uint32_t>(l.off_idx_b), n,
                                dim * levels_for(dim), ctx->at<uint32_t>(l.off_hist),
                                ctx->at<uint32_t>(l.off_digit_tot), s));
    }
    {
        StageScope st_(ctx, TC_STAGE_GATHER, s);
        TC_HIP(ctx, launch_gather(ctx->at<char>(l.off_mom_lvl), ctx->at<uint32_t>(l.off_idx_a), n, f64,
                                  ctx->at<Body>(l.off_bodies), ctx->at<float4>(l.off_bodies32), s));
    }
    {
        StageScope st_(ctx, TC_STAGE_TOPOLOGY, s);
        TC_HIP(ctx, launch_topology(ctx->at<uint64_t>(l.off_keys_a), n, dim, leaf_cap,
                                    ctx->at<uint32_t>(l.off_range), ctx->at<uint32_t>(l.off_nper),
                                    ctx->at<uint32_t>(l.off_cstart), ctx->at<uint32_t>(l.off_scan_part),
                                    l.scan_tiles, ctx->at<Cell>(l.off_cells),
                                    l.cmax, prm, s));
    }
    {
        StageScope st_(ctx, TC_STAGE_LEVELS, s);
        // tiles sized for the cells a tree usually holds (about 4 per leaf_cap
        // bodies), not for the slots
        const int64_t cells_est = std::min<int64_t>(l.cmax, 4 * n / leaf_cap + 1);
        TC_HIP(ctx, launch_level_order(ctx->at<Cell>(l.off_cells), l.cmax, cells_est, dim, prm,
                                       ctx->at<uint32_t>(l.off_lvl_idx_b), ctx->at<uint32_t>(l.off_lvl_hist),
                                       ctx->at<uint32_t>(l.off_digit_tot), ctx->at<uint32_t>(l.off_pre2bfs),
                                       ctx->at<uint32_t>(l.off_lvl_off), s));
    }
    // the depth of this tree, for later moments passes (not inside a capture,
    // and not where nothing may be allocated: the copy needs pinned memory)
    if (!ctx->capturing && !ctx->no_alloc) {
        harvest_depth(ctx);
        if (!ctx->lvl_host) TC_HIP(ctx, hipHostMalloc((void**)&ctx->lvl_host, 4 * 64, hipHostMallocDefault));
        if (!ctx->lvl_ev) TC_HIP(ctx, hipEventCreateWithFlags(&ctx->lvl_ev, hipEventDisableTiming));
        TC_HIP(ctx, hipMemcpyAsync(ctx->lvl_host, ctx->at<uint32_t>(l.off_lvl_off),
                                   4 * (size_t)(levels_for(dim) + 2), hipMemcpyDeviceToHost, s));
        TC_HIP(ctx, hipEventRecord(ctx->lvl_ev, s));
        ctx->lvl_pending = true;
    }
    {
        StageScope st_(ctx, TC_STAGE_GROUPS, s);
        TC_HIP(ctx, launch_groups(ctx->at<Cell>(l.off_cells), l.cmax, ctx->at<uint32_t>(l.off_gper),
                                  ctx->at<uint32_t>(l.off_goff), ctx->at<uint32_t>(l.off_gscan_part),
                                  l.cscan_tiles, ctx->at<int32_t>(l.off_gbeg), ctx->at<int32_t>(l.off_gcnt),
                                  l.gmax, prm, s));
    }
    ctx->mass = mass;
    ctx->n = n;
    ctx->leaf_cap = leaf_cap;
    ctx->dtype = dtype;
    ctx->state = kBuilt;
    ctx->fmm_planned = false;
    return TC_OK;
}

int do_moments(tc_ctx* ctx, hipStream_t s) {
    const Layout& l = ctx->lay;
    StageScope st_(ctx, TC_STAGE_MOMENTS, s);
    TC_HIP(ctx, launch_moments(ctx->at<Cell>(l.off_cells), ctx->at<Body>(l.off_bodies), ctx->dim, l.cmax,
                               ctx->at<uint32_t>(l.off_lvl_idx_b), ctx->at<uint32_t>(l.off_pre2bfs),
                               ctx->at<uint32_t>(l.off_lvl_off), ctx->prm(), ctx->at<Moments>(l.off_mom),
                               ctx->at<Moments>(l.off_mom_lvl), ctx->at<uint2>(l.off_kids),
                               ctx->at<WalkCell>(l.off_walk), ctx->have_hint ? ctx->lvl_hint : nullptr, s));
    ctx->state = kMoments;
    return TC_OK;
}

int do_walk(tc_ctx* ctx, double theta, hipStream_t s) {
    const Layout& l = ctx->lay;
    StageScope st_(ctx, TC_STAGE_RADII, s);
    TC_HIP(ctx, launch_mac(ctx->at<Cell>(l.off_cells), ctx->at<Moments>(l.off_mom), ctx->dim, theta, l.cmax,
                           ctx->at<uint32_t>(l.off_pre2bfs), ctx->at<WalkCell>(l.off_walk), nullptr, ctx->prm(),
                           s));
    ctx->theta = theta;
    ctx->theta_set = true;
    ctx->radii_plain = true;
    ctx->state = kWalked;
    ctx->pb_counted = false;
    return TC_OK;
}

// Opening radii of the learned walk: theta_l into the walk records,
// theta_p into the second radius array.  The plain walk's theta is kept.
int do_learned_radii(tc_ctx* ctx, double theta_l, double theta_p, hipStream_t s) {
    const Layout& l = ctx->lay;
    StageScope st_(ctx, TC_STAGE_RADII, s);
    TC_HIP(ctx, launch_mac(ctx->at<Cell>(l.off_cells), ctx->at<Moments>(l.off_mom), ctx->dim, theta_l, l.cmax,
                           ctx->at<uint32_t>(l.off_pre2bfs), ctx->at<WalkCell>(l.off_walk), nullptr, ctx->prm(),
                           s));
    TC_HIP(ctx, launch_mac(ctx->at<Cell>(l.off_cells), ctx->at<Moments>(l.off_mom), ctx->dim, theta_p, l.cmax,
                           ctx->at<uint32_t>(l.off_pre2bfs), ctx->at<WalkCell>(l.off_walk),
                           ctx->at<double>(l.off_rcp2), ctx->prm(), s));
    ctx->radii_plain = false;
    ctx->pb_counted = false;
    return TC_OK;
}

// The learned walk and forces (after do_learned_radii with the same thetas).
int do_forces_learned(tc_ctx* ctx, double G, double eps, double tau) {
    const Layout& l = ctx->lay;
    hipStream_t s = ctx->stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->timing) {
        e0 = pooled_event(ctx);
        e1 = pooled_event(ctx);
        if (!e0 || !e1) return hip_fail(ctx, hipErrorOutOfMemory);
        TC_HIP(ctx, hipEventRecord(e0, s));
    }
    const float tauf = isinf(tau) ? INFINITY : (float)tau;
    StageScope st_(ctx, TC_STAGE_FORCES, s);
    TC_HIP(ctx, launch_walk_force_learned(
                    ctx->at<WalkCell>(l.off_walk), ctx->at<double>(l.off_rcp2), ctx->at<Body>(l.off_bodies),
                    ctx->dtype == TC_F32 ? ctx->at<float4>(l.off_bodies32) : nullptr, ctx->at<Cell>(l.off_cells),
                    ctx->at<Moments>(l.off_mom), ctx->at<uint32_t>(l.off_lvl_idx_b), ctx->at<uint32_t>(l.off_idx_a),
                    ctx->at<int32_t>(l.off_gbeg), ctx->at<int32_t>(l.off_gcnt), l.gmax,
                    ctx->at<uint32_t>(l.off_queue), ctx->at<MlpState>(l.off_mlp), ctx->leaf_cap, (float)G,
                    (float)(eps * eps), tauf, ctx->n, ctx->prm(), ctx->at<float>(l.off_acc),
                    ctx->at<float>(l.off_pot), ctx->at<int64_t>(l.off_m2p), ctx->at<int64_t>(l.off_p2p),
                    ctx->at<int64_t>(l.off_nlearn), ctx->at<int64_t>(l.off_nfall), s));
    if (ctx->timing) {
        TC_HIP(ctx, hipEventRecord(e1, s));
        ctx->ev_pending.push_back(e0);
        ctx->ev_pending.push_back(e1);
    }
    ctx->G = G;
    ctx->eps = eps;
    ctx->state = kForced;
    ctx->tests_kept = false;
    return TC_OK;
}

int do_forces(tc_ctx* ctx, double G, double eps) {
    const Layout& l = ctx->lay;
    if (!ctx->radii_plain) {   // a learned walk left its own radii in the walk records
        int rc = do_walk(ctx, ctx->theta, ctx->stream);
        if (rc != TC_OK) return rc;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->timing) {
        e0 = pooled_event(ctx);
        e1 = pooled_event(ctx);
        if (!e0 || !e1) return hip_fail(ctx, hipErrorOutOfMemory);
        TC_HIP(ctx, hipEventRecord(e0, ctx->stream));
    }
    StageScope st_(ctx, TC_STAGE_FORCES, ctx->stream);
    float4* walkq = nullptr;
    if (ctx->mp_order == 2 && ctx->dim == 3) {
        walkq = ctx->at<float4>(l.off_walkq);
        TC_HIP(ctx, launch_quad_pack(ctx->at<Moments>(l.off_mom), ctx->at<uint32_t>(l.off_pre2bfs), ctx->prm(), l.cmax,
                                     walkq, ctx->stream));
    }
    if (ctx->split == 2 && ctx->n <= split_max_n(ctx->dim)) {
        TC_HIP(ctx, launch_walk_force_split(ctx->at<WalkCell>(l.off_walk), walkq, ctx->at<Body>(l.off_bodies),
                                            ctx->dtype == TC_F32 ? ctx->at<float4>(l.off_bodies32) : nullptr,
                                            ctx->at<uint32_t>(l.off_idx_a), ctx->at<int32_t>(l.off_gbeg),
                                            ctx->at<int32_t>(l.off_gcnt), l.gmax, ctx->n, ctx->dim, ctx->leaf_cap,
                                            (float)G, (float)(eps * eps), ctx->prm(), ctx->at<float4>(l.off_split),
                                            ctx->at<float>(l.off_acc), ctx->at<float>(l.off_pot),
                                            ctx->at<int64_t>(l.off_m2p), ctx->at<int64_t>(l.off_p2p),
                                            ctx->at<int64_t>(l.off_tests), ctx->plain_acc, ctx->stream));
    } else {
        TC_HIP(ctx, launch_walk_force(ctx->at<WalkCell>(l.off_walk), walkq, ctx->at<Body>(l.off_bodies),
                                      ctx->dtype == TC_F32 ? ctx->at<float4>(l.off_bodies32) : nullptr,
                                      ctx->at<uint32_t>(l.off_idx_a), ctx->at<int32_t>(l.off_gbeg),
                                      ctx->at<int32_t>(l.off_gcnt), l.gmax, ctx->at<uint32_t>(l.off_gorder),
                                      ctx->at<uint32_t>(l.off_queue), ctx->at<uint32_t>(l.off_bcost), ctx->n,
                                      ctx->dim, ctx->leaf_cap,
                                      (float)G, (float)(eps * eps), ctx->prm(), ctx->at<float>(l.off_acc),
                                      ctx->at<float>(l.off_pot), ctx->at<int64_t>(l.off_m2p),
                                      ctx->at<int64_t>(l.off_p2p), ctx->at<int64_t>(l.off_tests), ctx->plain_acc,
                                      ctx->split != 0,
                                      ctx->at<uint32_t>(l.off_lvl_off), ctx->stream));
    }
    if (ctx->timing) {
        TC_HIP(ctx, hipEventRecord(e1, ctx->stream));
        ctx->ev_pending.push_back(e0);
        ctx->ev_pending.push_back(e1);
    }
    ctx->G = G;
    ctx->eps = eps;
    ctx->state = kForced;
    ctx->tests_kept = !(ctx->split == 2 && ctx->n <= split_max_n(ctx->dim));
    return TC_OK;
}

// The part of a step before the force kernel (kick + drift, tree build,
// moments, opening radii: about 70 short kernels) on stream s.
int enqueue_pre_force(tc_ctx* ctx, double dt, void* pos, void* vel, hipStream_t s) {
    const int f64 = ctx->dtype == TC_F64;
    {
        StageScope st_(ctx, TC_STAGE_KICK_DRIFT, s);
        TC_HIP(ctx, launch_kick_drift(pos, vel, ctx->at<float>(ctx->lay.off_acc), ctx->n, ctx->dim, f64, dt, s));
    }
    int rc = do_build(ctx, pos, ctx->mass, ctx->n, ctx->leaf_cap, ctx->dtype, s);
    if (rc == TC_OK) rc = do_moments(ctx, s);
    if (rc == TC_OK)
        rc = ctx->closure ? do_learned_radii(ctx, ctx->cl_theta_l, ctx->cl_theta_p, s) : do_walk(ctx, ctx->theta, s);
    return rc;
}

void drop_graph(tc_ctx* ctx) {
    if (ctx->g_exec) (void)hipGraphExecDestroy(ctx->g_exec);
    ctx->g_exec = nullptr;
}

// Replays the pre-force part as one graph launch: on the context's stream
// when that is a created stream, else (the null stream cannot be captured)
// on a private stream ordered after and before it by events.  The graph is
// (re)captured whenever anything it bakes in (buffers, sizes, dt, theta)
// changes.  Returns TC_OK, or an error with nothing enqueued.
int pre_force_graph(tc_ctx* ctx, double dt, void* pos, void* vel) {
    tc_ctx::GraphKey key{pos,          vel,           ctx->mass,          ctx->ws,
                         ctx->n,       ctx->dim,      ctx->dtype,         ctx->leaf_cap,
                         dt,           ctx->theta,    ctx->closure,       ctx->closure ? ctx->cl_theta_l : 0.0,
                         ctx->closure ? ctx->cl_theta_p : 0.0};
    const bool own = ctx->stream != nullptr;
    if (!own && !ctx->gstream) {
        TC_HIP(ctx, hipStreamCreateWithFlags(&ctx->gstream, hipStreamNonBlocking));
        TC_HIP(ctx, hipEventCreateWithFlags(&ctx->g_in, hipEventDisableTiming));
        TC_HIP(ctx, hipEventCreateWithFlags(&ctx->g_out, hipEventDisableTiming));
    }
    hipStream_t cs = own ? ctx->stream : ctx->gstream;
    if (!ctx->g_exec || !(key == ctx->g_key)) {
        drop_graph(ctx);
        TC_HIP(ctx, hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
        ctx->capturing = true;
        const int rc = enqueue_pre_force(ctx, dt, pos, vel, cs);
        ctx->capturing = false;
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(cs, &g);
        if (rc != TC_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return rc != TC_OK ? rc : hip_fail(ctx, e);
        }
        const hipError_t ei = hipGraphInstantiate(&ctx->g_exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            ctx->g_exec = nullptr;
            return hip_fail(ctx, ei);
        }
        ctx->g_key = key;
    }
    if (own) {
        TC_HIP(ctx, hipGraphLaunch(ctx->g_exec, ctx->stream));
        return TC_OK;
    }
    TC_HIP(ctx, hipEventRecord(ctx->g_in, ctx->stream));
    TC_HIP(ctx, hipStreamWaitEvent(ctx->gstream, ctx->g_in, 0));
    TC_HIP(ctx, hipGraphLaunch(ctx->g_exec, ctx->gstream));
    TC_HIP(ctx, hipEventRecord(ctx->g_out, ctx->gstream));
    TC_HIP(ctx, hipStreamWaitEvent(ctx->stream, ctx->g_out, 0));
    return TC_OK;
}

// Carve-up of the caller's FMM buffer for C cells and the pair capacities.
struct FmmLayout {
    int64_t C, capf, capm, capp, capk, tiles;
    size_t off_geo, off_dc, off_lam, off_moff, off_poff, off_ctr, off_fa, off_fb, off_m2l,
        off_p2p, off_keys_b, off_bt, off_base, off_hist, off_digit, off_ntask, off_nslot, off_toff, off_soff, off_tpart,
        total;
    int64_t ctiles;
};

bool fmm_layout(int64_t C, int64_t capf, int64_t capm, int64_t capp, FmmLayout* f) {
    if (C < 1 || capf < 1 || capm < 1 || capp < 1) return false;
    const int64_t lim = (int64_t)1 << 32;   // offsets are 32-bit
    if (capf >= lim || capm >= lim || capp >= lim) return false;
    memset(f, 0, sizeof(*f));
    f->C = C;
    f->capf = capf;
    f->capm = capm;
    f->capp = capp;
    f->capk = capm > capp ? capm : capp;
    f->tiles = sort_tiles_max(f->capk);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    f->off_geo = take(sizeof(FmmGeo) * (size_t)C);
    f->off_dc = take(sizeof(DttCell) * (size_t)C);
    f->off_lam = take(8 * 20 * (size_t)C);
    f->off_moff = take(4 * (size_t)(C + 1));
    f->off_poff = take(4 * (size_t)(C + 1));
    f->off_ctr = take(8 * 4);
    f->off_fa = take(8 * (size_t)capf);
    f->off_fb = take(8 * (size_t)capf);
    f->off_m2l = take(8 * (size_t)capm);
    f->off_p2p = take(8 * (size_t)capp);
    f->off_keys_b = take(8 * (size_t)f->capk);
    f->off_bt = take(4 * 3 * (size_t)kFmmMaxBlocks);
    f->off_base = take(8 * 3 * (size_t)kFmmMaxBlocks);
    f->off_hist = take(4 * 256 * (size_t)f->tiles);
    f->off_digit = take(4 * 256);
    f->ctiles = (C + kScanTile - 1) / kScanTile;
    f->off_ntask = take(4 * (size_t)C);
    f->off_nslot = take(4 * (size_t)C);
    f->off_toff = take(4 * (size_t)(C + 1));
    f->off_soff = take(4 * (size_t)(C + 1));
    f->off_tpart = take(4 * (size_t)f->ctiles);
    f->total = off;
    return true;
}

// Sort n pair keys ((source << 32) | target) in place by target, stably:
// the low 16 * ceil(bits / 16) bits, an even number of 8-bit passes, so the
// result lands back in keys.
hipError_t fmm_sort(uint64_t* keys, int64_t n, int bits, uint8_t* buf, const FmmLayout& f, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    return launch_sort(keys, nullptr, reinterpret_cast<uint64_t*>(buf + f.off_keys_b), nullptr, n,
                       16 * ((bits + 15) / 16), reinterpret_cast<uint32_t*>(buf + f.off_hist),
                       reinterpret_cast<uint32_t*>(buf + f.off_digit), s);
}

}  // namespace

extern "C" {

size_t tc_fmm_buffer_bytes(int64_t ncells, int64_t frontier_cap, int64_t m2l_cap, int64_t p2p_cap) {
    FmmLayout f;
    if (!fmm_layout(ncells, frontier_cap, m2l_cap, p2p_cap, &f)) return 0;
    return f.total;
}

int tc_fmm_plan(tc_ctx* ctx, double theta, void* buf, size_t bytes, int64_t frontier_cap, int64_t m2l_cap,
                int64_t p2p_cap, int64_t sizes[3]) {
    if (!ctx || !buf || !sizes || !aligned(buf, 256)) return TC_EINVAL;
    if (!(theta >= 0.0) || !isfinite(theta)) return TC_EINVAL;
    if (ctx->dim != 3) return TC_EINVAL;
    if (ctx->state < kMoments) return TC_ESTATE;
    ctx->fmm_planned = false;
    const Layout& l = ctx->lay;
    hipStream_t s = ctx->stream;
    DevParams p;
    TC_HIP(ctx, hipMemcpyAsync(&p, ctx->prm(), sizeof(p), hipMemcpyDeviceToHost, s));
    TC_HIP(ctx, hipStreamSynchronize(s));
    const int64_t C = (int64_t)p.ncells < l.cmax ? (int64_t)p.ncells : l.cmax;
    FmmLayout f;
    if (!fmm_layout(C, frontier_cap, m2l_cap, p2p_cap, &f)) return TC_EINVAL;
    if (bytes < f.total) return TC_EWORKSPACE;
    uint8_t* B = (uint8_t*)buf;
    int bits = 1;
    while (((int64_t)1 << bits) < C) ++bits;
    const Cell* cells = ctx->at<Cell>(l.off_cells);
    const Moments* mom = ctx->at<Moments>(l.off_mom);
    FmmGeo* geo = reinterpret_cast<FmmGeo*>(B + f.off_geo);
    unsigned long long* ctr = reinterpret_cast<unsigned long long*>(B + f.off_ctr);
    uint64_t* fa = reinterpret_cast<uint64_t*>(B + f.off_fa);
    uint64_t* fb = reinterpret_cast<uint64_t*>(B + f.off_fb);
    uint64_t* m2l = reinterpret_cast<uint64_t*>(B + f.off_m2l);
    uint64_t* p2p = reinterpret_cast<uint64_t*>(B + f.off_p2p);
    DttCell* dc = reinterpret_cast<DttCell*>(B + f.off_dc);
    TC_HIP(ctx, launch_fmm_geo(cells, mom, ctx->at<WalkCell>(l.off_walk), ctx->at<uint32_t>(l.off_pre2bfs),
                               ctx->prm(), C, geo, dc, s));
    TC_HIP(ctx, hipMemcpyAsync(ctx->fmm_lvl_off, ctx->at<uint32_t>(l.off_lvl_off), sizeof(ctx->fmm_lvl_off),
                               hipMemcpyDeviceToHost, s));
    TC_HIP(ctx, hipStreamSynchronize(s));
    for (int lv = levels_for(3); lv >= 0; --lv) {   // level offsets cover levels 0..L and the end
        const int64_t cnt = (int64_t)ctx->fmm_lvl_off[lv + 1] - (int64_t)ctx->fmm_lvl_off[lv];
        TC_HIP(ctx, launch_fmm_radii(cells, mom, ctx->at<Body>(l.off_bodies), ctx->at<WalkCell>(l.off_walk),
                                     ctx->at<uint32_t>(l.off_lvl_idx_b), ctx->at<uint32_t>(l.off_lvl_off), lv, cnt,
                                     geo, dc, s));
    }
    TC_HIP(ctx, launch_fill_u32(reinterpret_cast<uint32_t*>(ctr), 8, s));
    TC_HIP(ctx, launch_fill_u32(reinterpret_cast<uint32_t*>(fa), 2, s));   // the pair (root, root)
    // one launch per level of pairs; the traversal is at most twice the
    // tree's depth plus one levels deep
    int64_t nin = 1, fmax = 1;
    unsigned long long hc[3] = {0, 0, 0};
    bool overflow = false;
    for (int it = 0; nin > 0; ++it) {
        if (it > 2 * (levels_for(3) + 1) + 1) return internal_fail("FMM traversal deeper than the tree allows");
        TC_HIP(ctx, launch_fill_u32(reinterpret_cast<uint32_t*>(ctr), 2, s));
        TC_HIP(ctx, launch_fmm_dtt(dc, theta, fa, nin, fb, f.capf, m2l, f.capm, p2p, f.capp, ctr,
                                   reinterpret_cast<uint32_t*>(B + f.off_bt),
                                   reinterpret_cast<unsigned long long*>(B + f.off_base), s));
        TC_HIP(ctx, hipMemcpyAsync(hc, ctr, sizeof(hc), hipMemcpyDeviceToHost, s));
        TC_HIP(ctx, hipStreamSynchronize(s));
        nin = (int64_t)hc[0];
        if (nin > fmax) fmax = nin;
        if (nin > f.capf) {
            overflow = true;
            break;
        }
        uint64_t* t = fa;
        fa = fb;
        fb = t;
    }
    sizes[0] = fmax;
    sizes[1] = (int64_t)hc[1];
    sizes[2] = (int64_t)hc[2];
    if (overflow || sizes[1] > f.capm || sizes[2] > f.capp) return TC_EWORKSPACE;
    TC_HIP(ctx, fmm_sort(m2l, sizes[1], bits, B, f, s));
    TC_HIP(ctx, fmm_sort(p2p, sizes[2], bits, B, f, s));
    TC_HIP(ctx, launch_fmm_offsets(m2l, sizes[1], C, reinterpret_cast<uint32_t*>(B + f.off_moff), s));
    TC_HIP(ctx, launch_fmm_offsets(p2p, sizes[2], C, reinterpret_cast<uint32_t*>(B + f.off_poff), s));
    // the leaf kernel's tasks: long partner lists cut into chunks whose
    // partial sums (4 doubles per body and chunk) use the frontier buffers
    uint32_t* toff = reinterpret_cast<uint32_t*>(B + f.off_toff);
    uint32_t* soff = reinterpret_cast<uint32_t*>(B + f.off_soff);
    TC_HIP(ctx, launch_fmm_tasks(cells, reinterpret_cast<const uint32_t*>(B + f.off_poff), ctx->prm(), C,
                                 reinterpret_cast<uint32_t*>(B + f.off_ntask),
                                 reinterpret_cast<uint32_t*>(B + f.off_nslot), s));
    TC_HIP(ctx, launch_scan_u32(reinterpret_cast<const uint32_t*>(B + f.off_ntask), C, toff,
                                reinterpret_cast<uint32_t*>(B + f.off_tpart), f.ctiles, s));
    TC_HIP(ctx, launch_scan_u32(reinterpret_cast<const uint32_t*>(B + f.off_nslot), C, soff,
                                reinterpret_cast<uint32_t*>(B + f.off_tpart), f.ctiles, s));
    uint32_t tot[2] = {0, 0};
    TC_HIP(ctx, hipMemcpyAsync(&tot[0], toff + C, 4, hipMemcpyDeviceToHost, s));
    TC_HIP(ctx, hipMemcpyAsync(&tot[1], soff + C, 4, hipMemcpyDeviceToHost, s));
    TC_HIP(ctx, hipStreamSynchronize(s));
    const int64_t part_slots = (int64_t)(f.off_fb + 8 * (size_t)f.capf - f.off_fa) / 32;
    if ((int64_t)tot[1] > part_slots) {
        sizes[0] = 2 * (int64_t)tot[1] + 1;          // frontier capacity that holds the partial sums
        return TC_EWORKSPACE;
    }
    if ((int64_t)tot[0] > 2 * f.capk)                      // tasks <= leaves + P2P pairs <= 2 capk
        return internal_fail("FMM leaf tasks exceed their buffer");
    TC_HIP(ctx, launch_fmm_tasks_fill(toff, ctx->prm(), C, reinterpret_cast<uint32_t*>(B + f.off_keys_b), s));
    ctx->fmm_ntasks = (int64_t)tot[0];
    TC_HIP(ctx, hipStreamSynchronize(s));
    ctx->fmm_buf = B;
    ctx->fmm_ncells = C;
    ctx->fmm_m2l = sizes[1];
    ctx->fmm_p2p = sizes[2];
    ctx->fmm_capf = f.capf;
    ctx->fmm_capm = f.capm;
    ctx->fmm_capp = f.capp;
    ctx->theta = theta;
    ctx->fmm_planned = true;
    return TC_OK;
}

int tc_fmm_forces(tc_ctx* ctx, double G, double eps, void* acc, void* pot) {
    if (!ctx) return TC_EINVAL;
    if (!(eps > 0.0) || !isfinite(eps) || !isfinite(G)) return TC_EINVAL;
    if ((acc && !aligned(acc, 4)) || (pot && !aligned(pot, 4))) return TC_EINVAL;
    if (!ctx->fmm_planned) return TC_ESTATE;
    const Layout& l = ctx->lay;
    hipStream_t s = ctx->stream;
    FmmLayout f;
    if (!fmm_layout(ctx->fmm_ncells, ctx->fmm_capf, ctx->fmm_capm, ctx->fmm_capp, &f)) return TC_EINVAL;
    uint8_t* B = ctx->fmm_buf;
    const FmmGeo* geo = reinterpret_cast<const FmmGeo*>(B + f.off_geo);
    double* lam = reinterpret_cast<double*>(B + f.off_lam);
    const Cell* cells = ctx->at<Cell>(l.off_cells);
    TC_HIP(ctx, launch_fmm_m2l(ctx->at<Moments>(l.off_mom), geo, ctx->prm(), f.C,
                               reinterpret_cast<const uint64_t*>(B + f.off_m2l),
                               reinterpret_cast<const uint32_t*>(B + f.off_moff), eps * eps, lam, s));
    for (int lv = 1; lv <= levels_for(3); ++lv) {   // level offsets cover levels 0..L and the end
        const int64_t cnt = (int64_t)ctx->fmm_lvl_off[lv + 1] - (int64_t)ctx->fmm_lvl_off[lv];
        TC_HIP(ctx, launch_fmm_l2l(cells, geo, ctx->at<uint32_t>(l.off_lvl_idx_b), ctx->at<uint32_t>(l.off_lvl_off),
                                   lv, cnt, lam, s));
    }
    TC_HIP(ctx, launch_fmm_leaf(cells, ctx->at<Body>(l.off_bodies),
                                ctx->dtype == TC_F32 ? ctx->at<float4>(l.off_bodies32) : nullptr,
                                ctx->at<uint32_t>(l.off_idx_a), geo, lam,
                                reinterpret_cast<const uint64_t*>(B + f.off_p2p),
                                reinterpret_cast<const uint32_t*>(B + f.off_poff),
                                reinterpret_cast<const uint32_t*>(B + f.off_keys_b),
                                reinterpret_cast<const uint32_t*>(B + f.off_toff),
                                reinterpret_cast<const uint32_t*>(B + f.off_soff), ctx->fmm_ntasks,
                                reinterpret_cast<double*>(B + f.off_fa), ctx->prm(), f.C,
                                (float)G, (float)(eps * eps), ctx->at<float>(l.off_acc), ctx->at<float>(l.off_pot), s));
    ctx->G = G;
    ctx->eps = eps;
    ctx->state = kForced;
    ctx->tests_kept = false;
    if (acc)
        TC_HIP(ctx, hipMemcpyAsync(acc, ctx->at<float>(l.off_acc), 4 * (size_t)ctx->n * 3, hipMemcpyDeviceToDevice, s));
    if (pot)
        TC_HIP(ctx, hipMemcpyAsync(pot, ctx->at<float>(l.off_pot), 4 * (size_t)ctx->n, hipMemcpyDeviceToDevice, s));
    return TC_OK;
}

int tc_fmm_get_pairs(tc_ctx* ctx, int32_t* m2l, int32_t* p2p) {
    if (!ctx) return TC_EINVAL;
    if ((m2l && !aligned(m2l, 4)) || (p2p && !aligned(p2p, 4))) return TC_EINVAL;
    if (!ctx->fmm_planned) return TC_ESTATE;
    FmmLayout f;
    if (!fmm_layout(ctx->fmm_ncells, ctx->fmm_capf, ctx->fmm_capm, ctx->fmm_capp, &f)) return TC_EINVAL;
    if (m2l)
        TC_HIP(ctx, launch_fmm_unpack(reinterpret_cast<const uint64_t*>(ctx->fmm_buf + f.off_m2l), ctx->fmm_m2l, m2l,
                                      ctx->stream));
    if (p2p)
        TC_HIP(ctx, launch_fmm_unpack(reinterpret_cast<const uint64_t*>(ctx->fmm_buf + f.off_p2p), ctx->fmm_p2p, p2p,
                                      ctx->stream));
    return TC_OK;
}

int tc_create(tc_ctx** out, int dim, void* hip_stream) {
    if (!out || (dim != 2 && dim != 3)) return TC_EINVAL;
    tc_ctx* c = new (std::nothrow) tc_ctx();
    if (!c) return TC_EINVAL;
    c->dim = dim;
    c->stream = (hipStream_t)hip_stream;
    *out = c;
    return TC_OK;
}

void tc_destroy(tc_ctx* ctx) {
    if (!ctx) return;
    if (ctx->lvl_ev) (void)hipEventSynchronize(ctx->lvl_ev);
    if (ctx->lvl_ev) (void)hipEventDestroy(ctx->lvl_ev);
    if (ctx->lvl_host) (void)hipHostFree(ctx->lvl_host);
    for (hipEvent_t e : ctx->ev_pending) (void)hipEventDestroy(e);
    for (const auto& e : ctx->st_pending) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    drop_graph(ctx);
    if (ctx->g_in) (void)hipEventDestroy(ctx->g_in);
    if (ctx->g_out) (void)hipEventDestroy(ctx->g_out);
    if (ctx->gstream) (void)hipStreamDestroy(ctx->gstream);
    delete ctx;
}

size_t tc_workspace_bytes(int64_t n, int dim, int leaf_cap) {
    if (!valid_sizes(n, dim, leaf_cap)) return 0;
    return make_layout(n, dim, leaf_cap).total;
}

int tc_set_workspace(tc_ctx* ctx, void* dev, size_t bytes) {
    if (!ctx || !dev || !aligned(dev, 256)) return TC_EINVAL;
    ctx->ws = (uint8_t*)dev;
    ctx->ws_bytes = bytes;
    ctx->state = kNone;
    return TC_OK;
}

int tc_build(tc_ctx* ctx, const void* pos, const void* mass, int64_t n, int dim, int leaf_cap,
             int dtype) {
    if (!ctx || !pos || !mass) return TC_EINVAL;
    if (dim != ctx->dim || !valid_sizes(n, dim, leaf_cap)) return TC_EINVAL;
    if (dtype != TC_F32 && dtype != TC_F64) return TC_EINVAL;
    const size_t es = dtype == TC_F64 ? 8 : 4;
    if (!aligned(pos, es) || !aligned(mass, es)) return TC_EINVAL;
    if (!ctx->ws || ctx->ws_bytes < make_layout(n, dim, leaf_cap).total) return TC_EWORKSPACE;
    return do_build(ctx, pos, mass, n, leaf_cap, dtype, ctx->stream);
}

int tc_moments(tc_ctx* ctx) {
    if (!ctx) return TC_EINVAL;
    if (ctx->state < kBuilt) return TC_ESTATE;
    return do_moments(ctx, ctx->stream);
}

int tc_walk(tc_ctx* ctx, double theta) {
    if (!ctx) return TC_EINVAL;
    if (!(theta >= 0.0 && theta <= 1.0)) return TC_EINVAL;
    if (ctx->state < kMoments) return TC_ESTATE;
    return do_walk(ctx, theta, ctx->stream);
}

int tc_forces(tc_ctx* ctx, double G, double eps, void* acc, void* pot) {
    if (!ctx) return TC_EINVAL;
    if (!(eps > 0.0) || !isfinite(eps) || !isfinite(G)) return TC_EINVAL;
    if ((acc && !aligned(acc, 4)) || (pot && !aligned(pot, 4))) return TC_EINVAL;
    if (ctx->state < kWalked || !ctx->theta_set) return TC_ESTATE;
    int rc = do_forces(ctx, G, eps);
    if (rc != TC_OK) return rc;
    const Layout& l = ctx->lay;
    if (acc)
        TC_HIP(ctx, hipMemcpyAsync(acc, ctx->at<float>(l.off_acc), 4 * (size_t)ctx->n * ctx->dim,
                                   hipMemcpyDeviceToDevice, ctx->stream));
    if (pot)
        TC_HIP(ctx, hipMemcpyAsync(pot, ctx->at<float>(l.off_pot), 4 * (size_t)ctx->n,
                                   hipMemcpyDeviceToDevice, ctx->stream));
    return TC_OK;
}

int tc_leapfrog(tc_ctx* ctx, double dt, void* pos, void* vel) {
    if (!ctx || !pos || !vel || !isfinite(dt)) return TC_EINVAL;
    const size_t es = ctx->dtype == TC_F64 ? 8 : 4;
    if (!aligned(pos, es) || !aligned(vel, es)) return TC_EINVAL;
    if (ctx->state < kForced) return TC_ESTATE;
    if (ctx->closure ? !ctx->mlp_loaded : !ctx->theta_set) return TC_ESTATE;
    int rc = ctx->use_graph ? pre_force_graph(ctx, dt, pos, vel) : enqueue_pre_force(ctx, dt, pos, vel, ctx->stream);
    if (rc != TC_OK) return rc;
    ctx->state = kWalked;
    rc = ctx->closure ? do_forces_learned(ctx, ctx->G, ctx->eps, ctx->cl_tau) : do_forces(ctx, ctx->G, ctx->eps);
    if (rc != TC_OK) return rc;
    StageScope st_(ctx, TC_STAGE_KICK, ctx->stream);
    TC_HIP(ctx, launch_kick(vel, ctx->at<float>(ctx->lay.off_acc), ctx->n, ctx->dim, ctx->dtype == TC_F64, dt,
                            ctx->stream));
    return TC_OK;
}

int tc_lists_count(tc_ctx* ctx, int64_t* total, uint32_t* counts) {
    if (!ctx || !total) return TC_EINVAL;
    if (counts && !aligned(counts, 4)) return TC_EINVAL;
    if (ctx->state < kWalked || !ctx->theta_set) return TC_ESTATE;
    if (!ctx->radii_plain) {   // a learned walk left its own radii in the walk records
        int rc = do_walk(ctx, ctx->theta, ctx->stream);
        if (rc != TC_OK) return rc;
    }
    const Layout& l = ctx->lay;
    hipStream_t s = ctx->stream;
    uint64_t* offs = ctx->at<uint64_t>(l.off_pb_off);
    TC_HIP(ctx, launch_pb_count(ctx->at<WalkCell>(l.off_walk), ctx->at<Body>(l.off_bodies), ctx->n, ctx->dim,
                                ctx->at<uint32_t>(l.off_pb_cnt), offs, ctx->at<uint64_t>(l.off_pb_part), s));
    if (counts)
        TC_HIP(ctx, hipMemcpyAsync(counts, ctx->at<uint32_t>(l.off_pb_cnt), 4 * (size_t)ctx->n,
                                   hipMemcpyDeviceToDevice, s));
    uint64_t tot = 0;
    TC_HIP(ctx, hipMemcpyAsync(&tot, offs + ctx->n, sizeof(tot), hipMemcpyDeviceToHost, s));
    TC_HIP(ctx, hipStreamSynchronize(s));
    ctx->pb_total = (int64_t)tot;
    ctx->pb_counted = true;
    *total = (int64_t)tot;
    return TC_OK;
}

int tc_lists_forces(tc_ctx* ctx, double G, double eps, uint32_t* lists, int64_t cap, void* acc, void* pot) {
    if (!ctx || !lists || !aligned(lists, 4)) return TC_EINVAL;
    if (!(eps > 0.0) || !isfinite(eps) || !isfinite(G)) return TC_EINVAL;
    if ((acc && !aligned(acc, 4)) || (pot && !aligned(pot, 4))) return TC_EINVAL;
    if (ctx->state < kWalked || !ctx->pb_counted) return TC_ESTATE;
    if (cap < ctx->pb_total) return TC_EINVAL;
    const Layout& l = ctx->lay;
    hipStream_t s = ctx->stream;
    TC_HIP(ctx, launch_pb_write_sum(ctx->at<WalkCell>(l.off_walk), ctx->at<Body>(l.off_bodies),
                                    ctx->at<uint32_t>(l.off_idx_a), ctx->n, ctx->dim, ctx->at<uint64_t>(l.off_pb_off),
                                    lists, cap, l.cmax, (float)G, (float)(eps * eps), ctx->at<float>(l.off_acc),
                                    ctx->at<float>(l.off_pot), s));
    ctx->G = G;
    ctx->eps = eps;
    ctx->state = kForced;
    ctx->tests_kept = false;
    if (acc)
        TC_HIP(ctx, hipMemcpyAsync(acc, ctx->at<float>(l.off_acc), 4 * (size_t)ctx->n * ctx->dim,
                                   hipMemcpyDeviceToDevice, s));
    if (pot)
        TC_HIP(ctx, hipMemcpyAsync(pot, ctx->at<float>(l.off_pot), 4 * (size_t)ctx->n, hipMemcpyDeviceToDevice, s));
    return TC_OK;
}

int tc_set_split(tc_ctx* ctx, int mode) {
    if (!ctx || mode < 0 || mode > 2) return TC_EINVAL;
    ctx->split = mode;
    return TC_OK;
}

int tc_set_multipole(tc_ctx* ctx, int order) {
    if (!ctx || (order != 1 && order != 2) || (order == 2 && ctx->dim != 3)) return TC_EINVAL;
    ctx->mp_order = order;
    return TC_OK;
}

int tc_set_accumulation(tc_ctx* ctx, int mode) {
    if (!ctx || (mode != TC_ACC_COMPENSATED && mode != TC_ACC_PLAIN)) return TC_EINVAL;
    ctx->plain_acc = mode == TC_ACC_PLAIN;
    return TC_OK;
}

int tc_set_graph(tc_ctx* ctx, int on) {
    if (!ctx) return TC_EINVAL;
    ctx->use_graph = on != 0;
    if (!ctx->use_graph) drop_graph(ctx);
    return TC_OK;
}

int tc_diag(tc_ctx* ctx, const void* vel, double out[8]) {
    if (!ctx || !vel || !out) return TC_EINVAL;
    if (!aligned(vel, ctx->dtype == TC_F64 ? 8 : 4)) return TC_EINVAL;
    if (ctx->state < kForced) return TC_ESTATE;
    const Layout& l = ctx->lay;
    double* dout = ctx->at<double>(l.off_diag_out);
    StageScope st_(ctx, TC_STAGE_DIAG, ctx->stream);
    TC_HIP(ctx, launch_diag(ctx->mass, vel, ctx->at<float>(l.off_acc), ctx->at<float>(l.off_pot), ctx->n,
                            ctx->dim, ctx->dtype == TC_F64, ctx->at<double>(l.off_diag_part), dout,
                            ctx->stream));
    double host[8];
    TC_HIP(ctx, hipMemcpyAsync(host, dout, sizeof(host), hipMemcpyDeviceToHost, ctx->stream));
    TC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    memcpy(out, host, sizeof(host));
    return TC_OK;
}

int tc_diag_async(tc_ctx* ctx, const void* vel, double* out) {
    if (!ctx || !vel || !out) return TC_EINVAL;
    if (!aligned(vel, ctx->dtype == TC_F64 ? 8 : 4) || !aligned(out, 8)) return TC_EINVAL;
    if (ctx->state < kForced) return TC_ESTATE;
    const Layout& l = ctx->lay;
    StageScope st_(ctx, TC_STAGE_DIAG, ctx->stream);
    TC_HIP(ctx, launch_diag(ctx->mass, vel, ctx->at<float>(l.off_acc), ctx->at<float>(l.off_pot), ctx->n,
                            ctx->dim, ctx->dtype == TC_F64, ctx->at<double>(l.off_diag_part), out, ctx->stream));
    return TC_OK;
}

int tc_status(tc_ctx* ctx) {
    if (!ctx) return TC_EINVAL;
    TC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->last_hip != hipSuccess) return hip_fail(ctx, ctx->last_hip);
    if (!ctx->ws || ctx->state < kBuilt) return TC_OK;
    DevParams p;
    TC_HIP(ctx, hipMemcpy(&p, ctx->prm(), sizeof(p), hipMemcpyDeviceToHost));
    if (p.status & kFlagNonFinite) return TC_ENONFINITE;
    if (p.status & kFlagOverflow) return TC_EWORKSPACE;
    if (p.status & kFlagBadIndex) return TC_EINVAL;
    return TC_OK;
}

const char* tc_strerror(int code) {
    switch (code) {
        case TC_OK: return "ok";
        case TC_EINVAL: return "invalid argument";
        case TC_EWORKSPACE: return "workspace missing or too small";
        case TC_ESTATE: return "call order violated (build -> moments -> walk -> forces -> leapfrog)";
        case TC_EHIP: return g_errbuf[0] ? g_errbuf : "HIP failure";
        case TC_ENONFINITE: return "non-finite position or mass, or non-positive mass";
        default: return "unknown status";
    }
}

/* ---- learned closure ---------------------------------------------------- */

int tc_residuals(tc_ctx* ctx, double theta, double eps, const int32_t* targets, int nt, float* feat,
                 float* y, int32_t* cell, int64_t cap, int64_t* n_out) {
    if (!ctx || !targets || !n_out || nt < 1 || nt > kResidMaxTargets || cap < 0) return TC_EINVAL;
    if (cap > 0 && (!feat || !y || !cell)) return TC_EINVAL;
    if (!(theta > 0.0 && theta <= 1.0) || !(eps > 0.0) || !isfinite(eps)) return TC_EINVAL;
    if (ctx->dim != 3) return TC_EINVAL;
    if (ctx->state < kMoments) return TC_ESTATE;
    int rc = do_walk(ctx, theta, ctx->stream);
    if (rc != TC_OK) return rc;
    const Layout& l = ctx->lay;
    hipStream_t s = ctx->stream;
    uint32_t* inv = ctx->at<uint32_t>(l.off_inv_perm);
    uint32_t* cnt = ctx->at<uint32_t>(l.off_rcount);
    uint32_t* off = ctx->at<uint32_t>(l.off_roffs);
    TC_HIP(ctx, launch_inverse_perm(ctx->at<uint32_t>(l.off_idx_a), ctx->n, inv, s));
    for (int pass = 0; pass < 2; ++pass) {
        TC_HIP(ctx, launch_residuals(pass == 1, ctx->at<WalkCell>(l.off_walk), ctx->at<Body>(l.off_bodies),
                                     ctx->at<Cell>(l.off_cells), ctx->at<Moments>(l.off_mom),
                                     ctx->at<uint32_t>(l.off_lvl_idx_b), inv, ctx->prm(), ctx->n, targets, nt,
                                     eps * eps, cnt, off, cap, feat, y, cell, s));
        if (pass == 0)
            TC_HIP(ctx, launch_scan_u32(cnt, nt, off, ctx->at<uint32_t>(l.off_rscan_part),
                                        (nt + kScanTile - 1) / kScanTile, s));
    }
    uint32_t total = 0;
    TC_HIP(ctx, hipMemcpyAsync(&total, off + nt, sizeof(total), hipMemcpyDeviceToHost, s));
    TC_HIP(ctx, hipStreamSynchronize(s));
    *n_out = total;
    return TC_OK;
}

int tc_direct(tc_ctx* ctx, const int32_t* targets, int nt, double G, double eps, double* acc, double* pot) {
    if (!ctx || !targets || nt < 1 || nt > kResidMaxTargets) return TC_EINVAL;
    if (!(eps >= 0.0) || !isfinite(eps) || !isfinite(G)) return TC_EINVAL;
    if ((acc && !aligned(acc, 8)) || (pot && !aligned(pot, 8))) return TC_EINVAL;
    if (ctx->state < kBuilt) return TC_ESTATE;
    const Layout& l = ctx->lay;
    hipStream_t s = ctx->stream;
    uint32_t* inv = ctx->at<uint32_t>(l.off_inv_perm);
    TC_HIP(ctx, launch_inverse_perm(ctx->at<uint32_t>(l.off_idx_a), ctx->n, inv, s));
    TC_HIP(ctx, launch_direct64(ctx->at<Body>(l.off_bodies), inv, ctx->n, targets, nt, eps * eps, G, ctx->prm(), acc,
                                pot, s));
    return TC_OK;
}

int tc_mlp_load(tc_ctx* ctx, const float* params) {
    if (!ctx || !params || !aligned(params, 4)) return TC_EINVAL;
    if (!ctx->ws || ctx->state < kBuilt) return TC_ESTATE;
    TC_HIP(ctx, launch_mlp_load(ctx->at<MlpState>(ctx->lay.off_mlp), params, ctx->stream));
    ctx->mlp_step = 0;
    ctx->mlp_loaded = true;
    return TC_OK;
}

int tc_mlp_get(tc_ctx* ctx, float* params) {
    if (!ctx || !params || !aligned(params, 4)) return TC_EINVAL;
    if (!ctx->mlp_loaded) return TC_ESTATE;
    TC_HIP(ctx, launch_mlp_get(ctx->at<MlpState>(ctx->lay.off_mlp), params, ctx->stream));
    return TC_OK;
}

int tc_mlp_forward(tc_ctx* ctx, const float* feat, int64_t nrows, const int32_t* idx, int64_t nb, float* yhat) {
    if (!ctx || !feat || !yhat || nb < 1 || nrows < 1 || (!idx && nb > nrows)) return TC_EINVAL;
    if (!ctx->mlp_loaded) return TC_ESTATE;
    TC_HIP(ctx, launch_mlp_forward(ctx->at<MlpState>(ctx->lay.off_mlp), feat, nrows, idx, nb, yhat,
                                   &ctx->prm()->status, ctx->stream));
    return TC_OK;
}

int tc_mlp_step(tc_ctx* ctx, const float* feat, const float* y, int64_t nrows, const int32_t* idx, int64_t nb,
                double lr, float* loss, float* grad) {
    if (!ctx || !feat || !y || nb < 1 || nb > kMlpBatchMax || !(lr >= 0.0) || !isfinite(lr)) return TC_EINVAL;
    if (nrows < 1 || (!idx && nb > nrows)) return TC_EINVAL;
    if (!ctx->mlp_loaded) return TC_ESTATE;
    MlpState* st = ctx->at<MlpState>(ctx->lay.off_mlp);
    ctx->mlp_step += 1;
    TC_HIP(ctx, launch_mlp_step(st, feat, y, nrows, idx, nb, (float)lr, ctx->mlp_step, grad, &ctx->prm()->status,
                                ctx->stream));
    if (loss) {
        TC_HIP(ctx, hipMemcpyAsync(loss, &st->loss, sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
        TC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    return TC_OK;
}

int tc_forces_learned(tc_ctx* ctx, double G, double eps, double theta_l, double theta_p, double tau, void* acc,
                      void* pot) {
    if (!ctx) return TC_EINVAL;
    if (!(eps > 0.0) || !isfinite(eps) || !isfinite(G)) return TC_EINVAL;
    if (!(theta_l > 0.0 && theta_l <= 1.0) || !(theta_p >= 0.0 && theta_p < theta_l) || !(tau >= 0.0))
        return TC_EINVAL;
    if ((acc && !aligned(acc, 4)) || (pot && !aligned(pot, 4))) return TC_EINVAL;
    if (ctx->dim != 3) return TC_EINVAL;
    if (ctx->state < kMoments || !ctx->mlp_loaded) return TC_ESTATE;
    int rc = do_learned_radii(ctx, theta_l, theta_p, ctx->stream);
    if (rc == TC_OK) rc = do_forces_learned(ctx, G, eps, tau);
    if (rc != TC_OK) return rc;
    const Layout& l = ctx->lay;
    hipStream_t s = ctx->stream;
    if (acc)
        TC_HIP(ctx, hipMemcpyAsync(acc, ctx->at<float>(l.off_acc), 4 * (size_t)ctx->n * 3,
                                   hipMemcpyDeviceToDevice, s));
    if (pot)
        TC_HIP(ctx, hipMemcpyAsync(pot, ctx->at<float>(l.off_pot), 4 * (size_t)ctx->n,
                                   hipMemcpyDeviceToDevice, s));
    return TC_OK;
}

// The device address of this device's scratch, looked up on the first call
// on each device (with that device current) and kept.
int scratch_address(tc_ctx* ctx, uint8_t** out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static uint8_t* addr[kMaxDevices] = {};
    int dev = 0;
    TC_HIP(ctx, hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return internal_fail("device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        TC_HIP(ctx, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return internal_fail("no device address for the scratch array");
        addr[dev] = static_cast<uint8_t*>(p);
    }
    *out = addr[dev];
    return TC_OK;
}

int tc_forces_noalloc(tc_ctx* ctx, const void* pos, const void* mass, int64_t n, int leaf_cap, int dtype,
                      double theta, double G, double eps, void* acc, void* pot) {
    if (!ctx || !pos || !mass) return TC_EINVAL;
    const int dim = ctx->dim;
    if (!valid_sizes(n, dim, leaf_cap)) return TC_EINVAL;
    if (dtype != TC_F32 && dtype != TC_F64) return TC_EINVAL;
    const size_t es = dtype == TC_F64 ? 8 : 4;
    if (!aligned(pos, es) || !aligned(mass, es)) return TC_EINVAL;
    if (!(theta >= 0.0 && theta <= 1.0)) return TC_EINVAL;
    if (!(eps > 0.0) || !isfinite(eps) || !isfinite(G)) return TC_EINVAL;
    if ((acc && !aligned(acc, 4)) || (pot && !aligned(pot, 4))) return TC_EINVAL;
    if (make_layout(n, dim, leaf_cap).total > (size_t)TC_NOALLOC_SCRATCH_BYTES) return TC_EWORKSPACE;
    uint8_t* ws = nullptr;
    int rc = scratch_address(ctx, &ws);
    if (rc != TC_OK) return rc;
    ctx->ws = ws;
    ctx->ws_bytes = (size_t)TC_NOALLOC_SCRATCH_BYTES;
    ctx->state = kNone;
    // no events either: timing stays off for this call
    const bool timing = ctx->timing, stage_timing = ctx->stage_timing;
    ctx->timing = ctx->stage_timing = false;
    ctx->no_alloc = true;
    hipStream_t s = ctx->stream;
    rc = do_build(ctx, pos, mass, n, leaf_cap, dtype, s);
    if (rc == TC_OK) rc = do_moments(ctx, s);
    if (rc == TC_OK) rc = do_walk(ctx, theta, s);
    if (rc == TC_OK) rc = do_forces(ctx, G, eps);
    ctx->no_alloc = false;
    ctx->timing = timing;
    ctx->stage_timing = stage_timing;
    if (rc != TC_OK) return rc;
    const Layout& l = ctx->lay;
    if (acc)
        TC_HIP(ctx, hipMemcpyAsync(acc, ctx->at<float>(l.off_acc), 4 * (size_t)n * dim, hipMemcpyDeviceToDevice, s));
    if (pot) TC_HIP(ctx, hipMemcpyAsync(pot, ctx->at<float>(l.off_pot), 4 * (size_t)n, hipMemcpyDeviceToDevice, s));
    return TC_OK;
}

int tc_set_closure(tc_ctx* ctx, double theta_l, double theta_p, double tau) {
    if (!ctx) return TC_EINVAL;
    if (theta_l == 0.0) {
        ctx->closure = false;
        return TC_OK;
    }
    if (ctx->dim != 3) return TC_EINVAL;
    if (!(theta_l > 0.0 && theta_l <= 1.0) || !(theta_p >= 0.0 && theta_p < theta_l) || !(tau >= 0.0))
        return TC_EINVAL;
    ctx->closure = true;
    ctx->cl_theta_l = theta_l;
    ctx->cl_theta_p = theta_p;
    ctx->cl_tau = tau;
    return TC_OK;
}

int tc_get_learned_counts(tc_ctx* ctx, int64_t* learned, int64_t* fallback) {
    if (!ctx) return TC_EINVAL;
    if (ctx->state < kForced) return TC_ESTATE;
    int64_t ng = 0;
    int rc = tc_num_groups(ctx, &ng);
    if (rc != TC_OK) return rc;
    const Layout& l = ctx->lay;
    if (learned)
        TC_HIP(ctx, hipMemcpyAsync(learned, ctx->at<int64_t>(l.off_nlearn), 8 * (size_t)ng,
                                   hipMemcpyDeviceToDevice, ctx->stream));
    if (fallback)
        TC_HIP(ctx, hipMemcpyAsync(fallback, ctx->at<int64_t>(l.off_nfall), 8 * (size_t)ng,
                                   hipMemcpyDeviceToDevice, ctx->stream));
    return TC_OK;
}

int tc_num_cells(tc_ctx* ctx, int64_t* ncells) {
    if (!ctx || !ncells) return TC_EINVAL;
    if (ctx->state < kBuilt) return TC_ESTATE;
    DevParams p;
    TC_HIP(ctx, hipMemcpyAsync(&p, ctx->prm(), sizeof(p), hipMemcpyDeviceToHost, ctx->stream));
    TC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *ncells = p.ncells < ctx->lay.cmax ? p.ncells : ctx->lay.cmax;
    return TC_OK;
}

int tc_get_root(tc_ctx* ctx, double* lo, double* size) {
    if (!ctx || !lo || !size) return TC_EINVAL;
    if (ctx->state < kBuilt) return TC_ESTATE;
    DevParams p;
    TC_HIP(ctx, hipMemcpyAsync(&p, ctx->prm(), sizeof(p), hipMemcpyDeviceToHost, ctx->stream));
    TC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int a = 0; a < ctx->dim; ++a) lo[a] = p.lo[a];
    *size = p.size;
    return TC_OK;
}

int tc_get_keys(tc_ctx* ctx, uint64_t* key_sorted, uint32_t* perm) {
    if (!ctx) return TC_EINVAL;
    if (ctx->state < kBuilt) return TC_ESTATE;
    const Layout& l = ctx->lay;
    if (key_sorted)
        TC_HIP(ctx, hipMemcpyAsync(key_sorted, ctx->at<uint64_t>(l.off_keys_a), 8 * (size_t)ctx->n,
                                   hipMemcpyDeviceToDevice, ctx->stream));
    if (perm)
        TC_HIP(ctx, hipMemcpyAsync(perm, ctx->at<uint32_t>(l.off_idx_a), 4 * (size_t)ctx->n,
                                   hipMemcpyDeviceToDevice, ctx->stream));
    return TC_OK;
}

int tc_get_cells(tc_ctx* ctx, int32_t* level, uint64_t* prefix, int32_t* begin, int32_t* count,
                 int32_t* parent, int32_t* skip, int32_t* nch, int32_t* leaf, double* M, double* com,
                 double* Q) {
    if (!ctx) return TC_EINVAL;
    if (ctx->state < kBuilt) return TC_ESTATE;
    if ((M || com || Q) && ctx->state < kMoments) return TC_ESTATE;
    const Layout& l = ctx->lay;
    TC_HIP(ctx, launch_export(ctx->at<Cell>(l.off_cells), ctx->at<Moments>(l.off_mom), ctx->dim, l.cmax,
                              ctx->prm(), level, prefix, begin, count, parent, skip, nch, leaf, M, com, Q,
                              ctx->stream));
    return TC_OK;
}

int tc_num_groups(tc_ctx* ctx, int64_t* ngroups) {
    if (!ctx || !ngroups) return TC_EINVAL;
    if (ctx->state < kBuilt) return TC_ESTATE;
    DevParams p;
    TC_HIP(ctx, hipMemcpyAsync(&p, ctx->prm(), sizeof(p), hipMemcpyDeviceToHost, ctx->stream));
    TC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *ngroups = p.ngroups < ctx->lay.gmax ? p.ngroups : ctx->lay.gmax;
    return TC_OK;
}

int tc_get_groups(tc_ctx* ctx, int32_t* begin, int32_t* count) {
    if (!ctx) return TC_EINVAL;
    if (ctx->state < kBuilt) return TC_ESTATE;
    int64_t ng = 0;
    int rc = tc_num_groups(ctx, &ng);
    if (rc != TC_OK) return rc;
    const Layout& l = ctx->lay;
    if (begin)
        TC_HIP(ctx, hipMemcpyAsync(begin, ctx->at<int32_t>(l.off_gbeg), 4 * (size_t)ng,
                                   hipMemcpyDeviceToDevice, ctx->stream));
    if (count)
        TC_HIP(ctx, hipMemcpyAsync(count, ctx->at<int32_t>(l.off_gcnt), 4 * (size_t)ng,
                                   hipMemcpyDeviceToDevice, ctx->stream));
    return TC_OK;
}

int tc_get_counts(tc_ctx* ctx, int64_t* m2p, int64_t* p2p) {
    if (!ctx) return TC_EINVAL;
    if (ctx->state < kForced) return TC_ESTATE;
    int64_t ng = 0;
    int rc = tc_num_groups(ctx, &ng);
    if (rc != TC_OK) return rc;
    const Layout& l = ctx->lay;
    if (m2p)
        TC_HIP(ctx, hipMemcpyAsync(m2p, ctx->at<int64_t>(l.off_m2p), 8 * (size_t)ng,
                                   hipMemcpyDeviceToDevice, ctx->stream));
    if (p2p)
        TC_HIP(ctx, hipMemcpyAsync(p2p, ctx->at<int64_t>(l.off_p2p), 8 * (size_t)ng,
                                   hipMemcpyDeviceToDevice, ctx->stream));
    return TC_OK;
}

int tc_get_tests(tc_ctx* ctx, int64_t* tests) {
    if (!ctx || !tests) return TC_EINVAL;
    if (ctx->state < kForced || !ctx->tests_kept) return TC_ESTATE;
    int64_t ng = 0;
    int rc = tc_num_groups(ctx, &ng);
    if (rc != TC_OK) return rc;
    TC_HIP(ctx, hipMemcpyAsync(tests, ctx->at<int64_t>(ctx->lay.off_tests), 8 * (size_t)ng,
                               hipMemcpyDeviceToDevice, ctx->stream));
    return TC_OK;
}

int tc_set_timing(tc_ctx* ctx, int on) {
    if (!ctx) return TC_EINVAL;
    ctx->timing = on != 0;
    ctx->t_total_ms = 0.0;
    ctx->t_launches = 0;
    return TC_OK;
}

int tc_set_stage_timing(tc_ctx* ctx, int on) {
    if (!ctx) return TC_EINVAL;
    for (const auto& e : ctx->st_pending) {
        (void)hipEventSynchronize(e.b);
        ctx->ev_pool.push_back(e.a);
        ctx->ev_pool.push_back(e.b);
    }
    ctx->st_pending.clear();
    ctx->stage_timing = on != 0;
    for (int k = 0; k < TC_NSTAGES; ++k) {
        ctx->st_ms[k] = 0.0;
        ctx->st_count[k] = 0;
    }
    return TC_OK;
}

int tc_get_stage_timing(tc_ctx* ctx, double ms[TC_NSTAGES], int64_t count[TC_NSTAGES]) {
    if (!ctx || !ms || !count) return TC_EINVAL;
    for (const auto& e : ctx->st_pending) {
        TC_HIP(ctx, hipEventSynchronize(e.b));
        float t = 0.f;
        TC_HIP(ctx, hipEventElapsedTime(&t, e.a, e.b));
        ctx->st_ms[e.stage] += t;
        ctx->st_count[e.stage] += 1;
        ctx->ev_pool.push_back(e.a);
        ctx->ev_pool.push_back(e.b);
    }
    ctx->st_pending.clear();
    for (int k = 0; k < TC_NSTAGES; ++k) {
        ms[k] = ctx->st_ms[k];
        count[k] = ctx->st_count[k];
    }
    return TC_OK;
}

int tc_get_timing(tc_ctx* ctx, double* total_ms, int64_t* launches) {
    if (!ctx || !total_ms || !launches) return TC_EINVAL;
    for (size_t k = 0; k + 1 < ctx->ev_pending.size(); k += 2) {
        TC_HIP(ctx, hipEventSynchronize(ctx->ev_pending[k + 1]));
        float ms = 0.f;
        TC_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev_pending[k], ctx->ev_pending[k + 1]));
        ctx->t_total_ms += ms;
        ctx->t_launches += 1;
        ctx->ev_pool.push_back(ctx->ev_pending[k]);
        ctx->ev_pool.push_back(ctx->ev_pending[k + 1]);
    }
    ctx->ev_pending.clear();
    *total_ms = ctx->t_total_ms;
    *launches = ctx->t_launches;
    return TC_OK;
}

}  // extern "C"
