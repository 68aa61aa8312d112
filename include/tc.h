/*
 * tc.h - C ABI of the MI355X treecode hot path.
 *
 * The library computes softened gravitational accelerations with the
 * treecode of Duy, Yamazaki & Oyanagi, "Performance Evaluation of Treecode
 * Algorithm for N-Body Simulation Using GridRPC System", §3.1: bodies are
 * placed in a quad-tree (2D) or oct-tree (3D) obtained by recursive 4-/8-way
 * subdivision of space until a subspace holds at most leaf_cap bodies; each
 * cell stands for its bodies as one body of their total mass at their
 * centre of mass; a walk from the root puts a cell on the interaction list
 * when it is distant enough and otherwise descends into its children; the
 * force on a body (F = G m_a m_b / r^2) is the sum over its list; finally
 * each body updates its position and velocity.  The step order of the
 * paper's client program (§3.2: construct the tree, build the lists,
 * compute the forces, move the bodies) is the call order below.
 *
 * Conventions
 *   - All pointers named dev/pos/mass/vel/acc/pot are DEVICE pointers (HIP
 *     device memory of the current device) owned by the caller; the library
 *     never allocates or frees device memory.  Its only device storage is
 *     the caller's workspace (tc_set_workspace).
 *   - Positions are [n][dim] row-major, masses [n], velocities [n][dim],
 *     all of the dtype given to tc_build (TC_F32 or TC_F64), naturally
 *     aligned.  Accelerations are FP32 [n][dim], potentials FP32 [n], in the
 *     caller's body order.
 *   - Every call enqueues work on the stream given to tc_create and returns
 *     without waiting, except where "synchronises" is stated.  A context is
 *     not thread-safe and serves one stream.
 *   - Return values: TC_OK or a negative tc_status_code.  Argument and state
 *     errors are detected on the host before anything is launched.
 */
#ifndef TC_H
#define TC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tc_ctx tc_ctx;

enum tc_status_code {
    TC_OK = 0,
    TC_EINVAL = -1,      /* bad argument: n, dim, leaf_cap, theta, eps, dt, null/misaligned pointer */
    TC_EWORKSPACE = -2,  /* no workspace, or smaller than tc_workspace_bytes() */
    TC_ESTATE = -3,      /* call order violated (see each call) */
    TC_EHIP = -4,        /* a HIP runtime call or launch failed, or an internal check
                            that is never expected to fail did (tc_strerror names it) */
    TC_ENONFINITE = -5   /* sticky: a position or mass was NaN/Inf, or a mass was <= 0 */
};

enum tc_dtype { TC_F32 = 0, TC_F64 = 1 };

/* Largest supported leaf_cap and body count. */
#define TC_MAX_LEAF_CAP 256
#define TC_MAX_N 2000000000LL

/* Create a context for dim = 2 or 3 that enqueues on hip_stream (a
 * hipStream_t; NULL = the null stream).  *out receives the context. */
int tc_create(tc_ctx **out, int dim, void *hip_stream);

/* Destroy a context (NULL is a no-op).  Does not touch the workspace.
 * Besides host memory, a context holds one event and 256 bytes of pinned
 * host memory, into which each tc_build copies its tree's level offsets
 * (the moments pass of later builds sizes its launches by that depth). */
void tc_destroy(tc_ctx *ctx);

/* Bytes of device workspace needed for n bodies in dim dimensions with the
 * given leaf_cap (0 for invalid arguments).  The bound covers the largest
 * possible tree: at most L * floor(n / (leaf_cap + 1)) internal cells
 * (L = 21 levels in 3D, 31 in 2D) plus n leaves. */
size_t tc_workspace_bytes(int64_t n, int dim, int leaf_cap);

/* Hand the context a device workspace of `bytes` bytes, 256-byte aligned,
 * which it uses until the next tc_set_workspace or tc_destroy.  The caller
 * keeps ownership. */
int tc_set_workspace(tc_ctx *ctx, void *dev, size_t bytes);

/* Tree construction (§3.1): root cube, Morton keys, stable radix sort,
 * gather of bodies into key order, and the cell topology in depth-first
 * pre-order.  pos/mass are device arrays of `dtype`; the mass pointer is
 * kept for tc_leapfrog and tc_diag and must stay valid.  1 <= n <= TC_MAX_N,
 * dim equal to the context's, 1 <= leaf_cap <= TC_MAX_LEAF_CAP.  Non-finite
 * inputs or non-positive masses raise the sticky TC_ENONFINITE (see
 * tc_status); the kernels still run to completion on such data. */
int tc_build(tc_ctx *ctx, const void *pos, const void *mass, int64_t n, int dim,
             int leaf_cap, int dtype);

/* Cell moments (§3.1: total mass at the centre of mass), bottom-up in FP64,
 * plus the traceless quadrupole in 3D.  Requires tc_build (TC_ESTATE). */
int tc_moments(tc_ctx *ctx);

/* Fix the opening parameter theta (0 <= theta <= 1) and prepare each cell's
 * opening radius r = s/theta + |com - centre| (s the cell side).  A cell is
 * accepted for a walk group (see tc_num_groups) iff the squared distance
 * from its centre of mass to the group's bounding box exceeds r^2;
 * theta = 0 accepts nothing (the direct sum).  Requires tc_moments. */
int tc_walk(tc_ctx *ctx, double theta);

/* Walk and force summation (§3.1, §3.2): for every body, the softened
 * acceleration G sum m (x_j - x_i) / (|x_j - x_i|^2 + eps^2)^{3/2} and
 * potential -G sum m / (|x_j - x_i|^2 + eps^2)^{1/2} over its group's
 * interaction list (accepted cells as pseudo-bodies, bodies of opened
 * leaves directly, self excluded), FP32 with compensated accumulation.
 * eps > 0 and finite, G finite.  acc ([n][dim] FP32) and pot ([n] FP32)
 * may each be NULL; the results are also kept for tc_leapfrog/tc_diag.
 * Requires tc_walk. */
int tc_forces(tc_ctx *ctx, double G, double eps, void *acc, void *pot);

/* One kick-drift-kick leapfrog step of size dt (finite) on pos and vel (in
 * place, dtype of tc_build, caller order): v += dt/2 a(x); x += dt v;
 * rebuild, moments, walk and forces at the new x with the last theta, G and
 * eps (or the learned walk set by tc_set_closure, with the network of the
 * last tc_mlp_load); v += dt/2 a(x').  Requires a previous tc_forces or
 * tc_forces_learned (it supplies a(x), G and eps); the plain walk also
 * requires a tc_walk (its theta), the learned walk a tc_mlp_load, else
 * TC_ESTATE.
 * With tc_set_graph(ctx, 1) everything before the force kernel (about 70
 * short kernels) is recorded once as a HIP graph and replayed: on the
 * context's stream if it is a created stream, else (the null stream cannot
 * be recorded) on a stream private to the context, ordered after and before
 * the context's stream by events.  It is recorded again when pos, vel, the
 * workspace, n, dt or theta change.  Results are the same as without it. */
int tc_leapfrog(tc_ctx *ctx, double dt, void *pos, void *vel);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): one whole
 * force evaluation, tc_build + tc_moments + tc_walk(theta) + tc_forces(G,
 * eps) with the same arguments, checks and results, whose workspace is a
 * device array inside the library (TC_NOALLOC_SCRATCH_BYTES per GPU, held
 * until the process ends) instead of the caller's.  Nothing is allocated:
 * no device or pinned memory, no events (force and stage timing skip this
 * call).  TC_EWORKSPACE when tc_workspace_bytes(n, dim, leaf_cap) exceeds
 * the scratch (47,786 bodies in 3D with leaf_cap 16).  Afterwards the
 * context works on that scratch as if tc_set_workspace had been called with
 * it (tc_leapfrog, tc_diag, the accessors), until the next
 * tc_set_workspace.  Every context on one GPU shares its scratch, which
 * keeps the last call's contents: calls that overlap on one GPU (other
 * streams, other contexts, other threads) race and must be ordered by the
 * caller. */
#define TC_NOALLOC_SCRATCH_BYTES (64u << 20)
int tc_forces_noalloc(tc_ctx *ctx, const void *pos, const void *mass, int64_t n, int leaf_cap, int dtype,
                      double theta, double G, double eps, void *acc, void *pot);

/* ---- per-body lists (the treecode as §3.1 states it) ----------------------
 * Every body walks the tree alone (its box is the point itself) at the
 * opening radii of the last tc_walk, and its list of accepted cells and
 * nearby bodies is written to memory before being summed.  The grouped walk
 * of tc_forces is the fast path; this one measures what per-body lists cost
 * and how accurate they are. */

/* Count every body's list (one walk per body) and return the total number
 * of entries in *total (host); counts (device u32 [n], bodies in key order,
 * see tc_get_keys) may be NULL.  Synchronises.  Requires tc_walk. */
int tc_lists_count(tc_ctx *ctx, int64_t *total, uint32_t *counts);

/* Write the lists into `lists` (device u32, cap >= the total of the last
 * tc_lists_count, else TC_EINVAL; body k's list follows body k-1's, bodies in
 * key order; an entry is a cell's level-order index, or 0x80000000 | the
 * key-order index of a body) and sum them: acc/pot as tc_forces (device,
 * FP32, caller order, either may be NULL).  Entries are offsets from the body
 * formed in FP64 and rounded to FP32; chunk sums are compensated and the
 * wave's lanes reduced in FP64.  Requires tc_lists_count after the last
 * tc_walk. */
int tc_lists_forces(tc_ctx *ctx, double G, double eps, uint32_t *lists, int64_t cap, void *acc, void *pot);

/* ---- Fast multipole method (3D) ------------------------------------------
 * The method §5 of the paper names as the way past the treecode's cost:
 * cells act on cells through Cartesian expansions.  Each cell's multipole is
 * its mass and traceless quadrupole about its centre of mass (the dipole
 * vanishes there); its local expansion about its geometric centre z has 20
 * FP64 coefficients, phi(z + d) = -G sum_{n<=3} (1/n!) Lam_n[d^n].  A dual tree
 * traversal from (root, root) sorts cell pairs: a cell with itself becomes
 * all pairs of its children (a leaf sums directly); target A and source B
 * interact through an expansion (M2L, at total order 3, with the softened
 * kernel (r^2 + eps^2)^(-1/2)) when |z_A - com_B| > (rho_A + rho_B) / theta,
 * rho_A and rho_B bounding their bodies about z_A and com_B (a leaf: its
 * farthest body; a cell: the largest centre distance plus radius over its
 * children; capped by the geometric bounds (sqrt 3/2) s and (sqrt 3/2) s +
 * |com - z|); two leaves that are not sum directly (P2P, FP32 with
 * compensated chunks); otherwise the larger cell (smaller level, A on a tie,
 * never a leaf) is split.  Parents pass their expansions down (L2L); each
 * body gets its leaf's expansion (L2P) plus its leaf's direct sums.
 * theta = 0 makes every pair direct: the result is the direct sum. */

/* Bytes of the caller's FMM buffer for ncells cells (tc_num_cells) and the
 * capacities of the traversal's widest level of pairs and of its M2L and
 * P2P pair lists (each 1 <= cap < 2^32).  0 for invalid sizes. */
size_t tc_fmm_buffer_bytes(int64_t ncells, int64_t frontier_cap, int64_t m2l_cap, int64_t p2p_cap);

/* Traverse at theta >= 0 (after tc_moments; 3D contexts only) into the
 * device buffer buf (256-byte aligned, bytes >= tc_fmm_buffer_bytes of the
 * same capacities; owned by the caller, kept until the next tc_build or
 * plan).  Synchronises the stream.  sizes[0..2] receive the widest level,
 * the M2L pair count and the P2P pair count; if any exceeds its capacity
 * the call returns TC_EWORKSPACE (sizes then hold lower bounds: retry with
 * larger capacities).  Pairs are kept grouped by target, in a fixed order
 * within each target, so results are reproducible bit for bit. */
int tc_fmm_plan(tc_ctx *ctx, double theta, void *buf, size_t bytes, int64_t frontier_cap, int64_t m2l_cap,
                int64_t p2p_cap, int64_t sizes[3]);

/* Forces of the current plan: acc [n][3] and pot [n] (FP32, device, caller
 * order; either may be NULL).  eps > 0.  TC_ESTATE without a plan. */
int tc_fmm_forces(tc_ctx *ctx, double G, double eps, void *acc, void *pot);

/* The plan's pairs as (target, source) pre-order cell indices, grouped by
 * target:
 * m2l [sizes[1]][2] and p2p [sizes[2]][2] int32 device arrays (either may be
 * NULL).  For tests. */
int tc_fmm_get_pairs(tc_ctx *ctx, int32_t *m2l, int32_t *p2p);

/* How a group's walk is spread over waves, for sizes with fewer walk groups
 * than the GPU keeps waves resident, where one wave per group leaves a lone,
 * latency-bound walk per SIMD.  mode 1 (the default): for n <= 163840 a
 * block of 4 waves shares each group's walk (the cells of one level, 5 to 7
 * by n and dim, dealt out among them) and adds their FP32 partial sums in
 * FP64 in wave order.  mode 2: for n <= 12288 in 3D and n <= 24576 in 2D
 * each group's walk is cut into one task per (level-1 cell, child) (64 in
 * 3D, 16 in 2D) whose FP32 partial sums are added in FP64 in a fixed order,
 * and above that as mode 1.  mode 0: one wave per group at any n.  The
 * interactions and counts are those of the one-wave walk in every mode;
 * only the summation order differs.  TC_EINVAL for another mode. */
int tc_set_split(tc_ctx *ctx, int mode);

/* Expansion order of accepted cells in tc_forces and tc_leapfrog: 1 (the
 * default) is the monopole of §3.1; 2 (3D only, else TC_EINVAL) adds each
 * accepted cell's quadrupole term: with d the cell's centre of mass minus
 * the body, s = (|d|^2 + eps^2)^{-1/2} and Q its traceless quadrupole
 * (sum m (3 dd - |d|^2 I)), a += G [-Q d s^5 + (5/2) (d.Q d) d s^7] and
 * phi -= (G/2) (d.Q d) s^5.  The walk and its counts are unchanged. */
int tc_set_multipole(tc_ctx *ctx, int order);

/* Per-body accumulation in the force kernel of tc_forces and tc_leapfrog:
 * TC_ACC_COMPENSATED (default) sums each chunk of 64 list entries in FP32
 * and folds the chunk sums into Neumaier-compensated totals;
 * TC_ACC_PLAIN keeps one running FP32 sum per component over the whole
 * list (the uncompensated reference for precision studies).  The learned
 * walk always compensates. */
#define TC_ACC_COMPENSATED 0
#define TC_ACC_PLAIN 1
int tc_set_accumulation(tc_ctx *ctx, int mode);

/* Switch the graph replay of tc_leapfrog on or off (default: every kernel
 * launched on the context's stream).  Off also frees the recorded graph. */
int tc_set_graph(tc_ctx *ctx, int on);

/* FP64 diagnostics of the last forces, with deterministic reductions:
 * out[0] = 1/2 sum m v^2, out[1] = 1/2 sum m phi, out[2..4] = sum m v,
 * out[5..7] = sum m a (z entries 0 in 2D).  vel is a device array of the
 * build dtype; out is HOST memory.  Synchronises.  Requires tc_forces. */
int tc_diag(tc_ctx *ctx, const void *vel, double out[8]);

/* The same diagnostics (same kernels, same values), enqueued on the
 * context's stream without a copy to the host or a wait: out is a DEVICE
 * array of 8 doubles owned by the caller (8-byte aligned), written when the
 * stream reaches the call.  For loops that keep a record per step and read
 * it later.  TC_EINVAL for a NULL or misaligned pointer; requires
 * tc_forces. */
int tc_diag_async(tc_ctx *ctx, const void *vel, double *out);

/* Synchronise the stream and return TC_OK, the sticky TC_ENONFINITE raised
 * by a build, or TC_EHIP if an earlier call recorded a HIP failure. */
int tc_status(tc_ctx *ctx);

/* Static message for a status code (TC_EHIP includes the last HIP error). */
const char *tc_strerror(int code);

/* ---- reference sums ------------------------------------------------------ */

/* FP64 direct sum for nt sample bodies (device int32 original indices,
 * 1 <= nt <= TC_RESID_MAX_TARGETS): acc[t][3] = G sum_{j != i} m_j d /
 * (|d|^2 + eps^2)^(3/2), d = x_j - x_i, and pot[t] = -G sum_{j != i} m_j /
 * (|d|^2 + eps^2)^(1/2) over all n bodies (the force law of §3.1 summed
 * exactly; positions and masses as held after tc_build, i.e. the input
 * values widened to FP64).  acc, pot: device FP64, either may be NULL.
 * eps >= 0 (eps = 0 needs distinct positions).  Summation order is fixed,
 * so results are reproducible.  A target outside [0, n) yields NaN and makes
 * tc_status report TC_EINVAL.  Requires tc_build. */
int tc_direct(tc_ctx *ctx, const int32_t *targets, int nt, double G, double eps, double *acc, double *pot);

/* ---- learned closure ---------------------------------------------------
 * An extension of the paper's monopole cells (§3.1): for a body x and an
 * accepted cell (centre of mass C, mass M, side s, traceless quadrupole Q)
 * a network predicts the residual in units of the quadrupole scale
 *     y = (a_exact - a_mono) |x - C|^4 / (M s^2)      (G = 1)
 * between the exact sum over the cell's bodies and its monopole, from the
 * features f = [(x - C)/s (3), Q/(M s^2) (6: xx yy zz xy xz yz),
 * ln(M / mbar) (1)], mbar = total mass / n.  The network is 10-64-64-3
 * with GELU (erf form), BF16 matrix-core products with FP32 accumulation and
 * FP32 master weights.  Parameters (canonical order, 5059 FP32): W1 [10][64],
 * b1 [64], W2 [64][64], b2 [64], W3 [64][3], b3 [3]; y = gelu(gelu(f W1 +
 * b1) W2 + b2) W3 + b3.  3D only. */

#define TC_MLP_NPARAM 5059
#define TC_MLP_BATCH_MAX 65536
#define TC_RESID_MAX_TARGETS 65536

/* Training pairs for nt target bodies (device int32 original indices,
 * 1 <= nt <= TC_RESID_MAX_TARGETS): each target walks alone (its box is the
 * body itself) at theta (0 < theta <= 1), and every accepted cell gives one
 * pair: feat [.][10] FP32, y [.][3] FP32 (exact sum in FP64), cell [.] the
 * cell's pre-order index.  Pairs are in target order.  At most cap pairs are
 * written (device buffers); *n_out (host) receives the total.  Prepares the
 * opening radii for theta as tc_walk does.  Synchronises.  Requires
 * tc_moments.  A target outside [0, n) gets no pairs and makes tc_status
 * report TC_EINVAL. */
int tc_residuals(tc_ctx *ctx, double theta, double eps, const int32_t *targets, int nt, float *feat,
                 float *y, int32_t *cell, int64_t cap, int64_t *n_out);

/* Load network parameters (device, TC_MLP_NPARAM FP32, canonical order) and
 * reset the Adam state.  Requires a workspace and tc_build. */
int tc_mlp_load(tc_ctx *ctx, const float *params);

/* Copy the FP32 master parameters out (device buffer).  Requires tc_mlp_load. */
int tc_mlp_get(tc_ctx *ctx, float *params);

/* Network outputs yhat [nb][3] (device) for feature rows feat[idx[k]] of
 * feat [nrows][10] (idx: device int32 [nb], or NULL for rows 0..nb-1, then
 * nb <= nrows).  A device index outside [0, nrows) leaves that output
 * unwritten and makes tc_status report TC_EINVAL. */
int tc_mlp_forward(tc_ctx *ctx, const float *feat, int64_t nrows, const int32_t *idx, int64_t nb, float *yhat);

/* One training step on the batch feat[idx[k]], y[idx[k]] (k < nb <=
 * TC_MLP_BATCH_MAX; feat [nrows][10], y [nrows][3]; idx may be NULL, then
 * nb <= nrows; a device index outside [0, nrows) drops that sample and
 * makes tc_status report TC_EINVAL): forward, mean squared error over the
 * nb x 3 outputs, backward, gradients summed in a fixed order, one Adam
 * step (beta 0.9/0.999, epsilon 1e-8) with learning rate lr >= 0.  *loss
 * (host, may be NULL: then nothing synchronises) gets the batch loss before
 * the update, grad (device, may be NULL) the gradient in canonical order. */
int tc_mlp_step(tc_ctx *ctx, const float *feat, const float *y, int64_t nrows, const int32_t *idx, int64_t nb,
                double lr, float *loss, float *grad);

/* Forces with the learned closure (3D only).  The walk of tc_forces with
 * two opening parameters theta_p < theta_l <= 1 (the opening test of §3.1
 * evaluated with each): a cell accepted at theta_l and at theta_p is a
 * monopole entry; a cell accepted at theta_l but opened at theta_p is a
 * learned cell.  For a learned cell the network loaded by tc_mlp_load
 * predicts, for each body of the walk group, the normalised residual yhat
 * (features as tc_residuals); if the largest predicted residual relative to
 * the monopole, |yhat| s^2 / |x - C|^2, over the group exceeds tau the
 * cell falls back to the plain walk of its subtree at theta_p, otherwise it
 * is a monopole entry plus G M s^2 yhat / |x - C|^4 per body (no softening).
 * tau = 0 gives exactly the plain walk at theta_p; tau = +inf gives the
 * plain walk at theta_l plus every correction.  The potential keeps the
 * monopoles.  acc/pot as tc_forces (device, FP32, either may be NULL).
 * Requires tc_moments and tc_mlp_load; TC_EINVAL for parameters outside
 * the ranges above or dim != 3.  The theta of the last tc_walk stays the
 * plain walk's: a later tc_forces, tc_lists_count or plain tc_leapfrog
 * walks at that theta again (its opening radii are recomputed first). */
int tc_forces_learned(tc_ctx *ctx, double G, double eps, double theta_l, double theta_p, double tau,
                      void *acc, void *pot);

/* Make tc_leapfrog evaluate its forces with the learned walk of
 * tc_forces_learned at (theta_l, theta_p, tau), same ranges, 3D only; every
 * step then rebuilds the tree, computes both opening radii and runs the
 * learned walk with the network last loaded by tc_mlp_load (that network's
 * parameters are read when the step runs).  theta_l = 0 switches back to
 * the plain walk at the theta of the last tc_walk.  Off by default. */
int tc_set_closure(tc_ctx *ctx, double theta_l, double theta_p, double tau);

/* Per walk group, the learned cells of the last tc_forces_learned that
 * were kept (learned) and that fell back (fallback): device int64 buffers
 * of tc_num_groups() entries, either may be NULL.  Requires
 * tc_forces_learned (after a plain tc_forces the contents are stale). */
int tc_get_learned_counts(tc_ctx *ctx, int64_t *learned, int64_t *fallback);

/* ---- inspection (tests and benchmarks) -------------------------------- */

/* Number of cells of the current tree.  Synchronises.  Requires tc_build. */
int tc_num_cells(tc_ctx *ctx, int64_t *ncells);

/* Root cube: lo[dim] corner and side.  Synchronises.  Requires tc_build. */
int tc_get_root(tc_ctx *ctx, double *lo, double *size);

/* Copy the sorted keys (u64 [n]) and the permutation (u32 [n], sorted
 * position -> original index) into device buffers (either may be NULL). */
int tc_get_keys(tc_ctx *ctx, uint64_t *key_sorted, uint32_t *perm);

/* Copy the per-cell arrays, in pre-order, into device buffers of at least
 * tc_num_cells() elements (com: [C][dim], Q: [C][6]); any may be NULL.
 * M/com/Q require tc_moments.  begin/count index the sorted bodies; skip is
 * the pre-order index just past the cell's subtree; parent is -1 for the
 * root; leaf is 1 for leaves. */
int tc_get_cells(tc_ctx *ctx, int32_t *level, uint64_t *prefix, int32_t *begin,
                 int32_t *count, int32_t *parent, int32_t *skip, int32_t *nch,
                 int32_t *leaf, double *M, double *com, double *Q);

/* Number of walk groups of the current tree.  A walk group is a run of at
 * most 64 consecutive bodies in key order lying inside one cluster cell (a
 * maximal cell of at most 1024 bodies, or a deeper leaf); each cluster cell
 * is cut into such runs in order.  Synchronises.  Requires tc_build. */
int tc_num_groups(tc_ctx *ctx, int64_t *ngroups);

/* Copy the groups' first sorted body and size (int32 [ngroups] device
 * buffers; either may be NULL).  Requires tc_build. */
int tc_get_groups(tc_ctx *ctx, int32_t *begin, int32_t *count);

/* Per-group interaction counts of the last tc_forces (device int64 arrays
 * of tc_num_groups() entries): accepted cells and bodies of opened leaves
 * (the group's own bodies included).  Synchronises.  Requires tc_forces. */
int tc_get_counts(tc_ctx *ctx, int64_t *m2p, int64_t *p2p);

/* Per-group number of cells whose opening test ran in the last tc_forces
 * walk (device int64 [tc_num_groups()]): the root and every child of an
 * opened cell, a measure of the walk's work (§3.1's traversal; not part of
 * the method's results).  TC_EINVAL for a NULL buffer; TC_ESTATE unless
 * the last force evaluation was a tc_forces (or tc_leapfrog) walk by one
 * wave or by waves sharing a group (not split walks, tc_set_split(ctx, 2),
 * whose tasks repeat the top of the walk, nor the learned, per-body-list or
 * FMM evaluations).  Synchronises like tc_get_counts. */
int tc_get_tests(tc_ctx *ctx, int64_t *tests);

/* Time the force kernel with HIP events on the context's stream: when on,
 * every tc_forces accumulates the kernel's duration. */
int tc_set_timing(tc_ctx *ctx, int on);

/* Total milliseconds and launch count of the timed force kernels since
 * timing was switched on.  Synchronises. */
int tc_get_timing(tc_ctx *ctx, double *total_ms, int64_t *launches);

/* Stages of a force evaluation and of a leapfrog step, for per-stage
 * timing: the kick + drift, the build (root cube, Morton keys, radix sort,
 * gather, topology, level order, walk groups), the moments, the opening
 * radii, the walk + force kernels (plain or learned, with their schedule
 * kernels), the closing kick, and the diagnostics. */
enum tc_stage {
    TC_STAGE_KICK_DRIFT = 0, TC_STAGE_BBOX, TC_STAGE_KEYS, TC_STAGE_SORT, TC_STAGE_GATHER,
    TC_STAGE_TOPOLOGY, TC_STAGE_LEVELS, TC_STAGE_GROUPS, TC_STAGE_MOMENTS, TC_STAGE_RADII,
    TC_STAGE_FORCES, TC_STAGE_KICK, TC_STAGE_DIAG, TC_NSTAGES
};

/* Switch per-stage timing on or off (and reset its totals): when on, every
 * call records a pair of HIP events on the context's stream around each
 * stage it enqueues (not inside the graph replay of tc_set_graph, whose
 * stages are not timed). */
int tc_set_stage_timing(tc_ctx *ctx, int on);

/* Milliseconds and occurrences per stage (host arrays of TC_NSTAGES, indexed
 * by tc_stage) since stage timing was switched on.  Synchronises. */
int tc_get_stage_timing(tc_ctx *ctx, double ms[TC_NSTAGES], int64_t count[TC_NSTAGES]);

#ifdef __cplusplus
}
#endif

#endif /* TC_H */
