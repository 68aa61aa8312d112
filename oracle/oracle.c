/*
 * FP64 CPU oracle for the treecode hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or helper with the
 * GPU library; the two meet only through the seeded input generators.
 *
 * What it computes (Duy, Yamazaki & Oyanagi, "Performance Evaluation of
 * Treecode Algorithm for N-Body Simulation Using GridRPC System"):
 *
 *   - the exact result: the direct pairwise sum of the force law of §3.1
 *     (F = G m_a m_b / r^2, with Plummer softening eps), in FP64;
 *   - the treecode of §3.1 step by step: the space is divided recursively
 *     into 4 (2D) or 8 (3D) subspaces until a subspace holds at most leaf_cap
 *     bodies; each cell carries the total mass of its bodies placed at their
 *     centre of mass; the walk starts at the root and puts a cell on the
 *     interaction list when it is distant enough, otherwise descends into its
 *     children; the force on a body is the sum over its list.
 *
 * Readings of what the paper leaves open (shared with the GPU path by
 * specification, not by code):
 *   - root cube: per-axis minimum corner, side = smallest power of two >= the
 *     largest per-axis extent (1 if the extent is 0);
 *   - subdivision follows Morton digits of FP64-quantised coordinates
 *     (L = 21 levels in 3D, 31 in 2D), digit = 4bx+2by+bz (3D), 2bx+by (2D);
 *     a cell is a leaf iff it holds <= leaf_cap bodies or sits at level L;
 *     empty subspaces are never materialised; children are kept in digit
 *     order and the cell array is the depth-first pre-order;
 *   - "distant enough" is a group opening criterion: cell c is accepted for a
 *     group of bodies iff the squared distance from c's centre of mass to the
 *     group's bounding box exceeds (s_c/theta + |com_c - centre_c|)^2, strict;
 *     theta = 0 accepts nothing;
 *   - groups are runs of gs consecutive bodies in Morton order (gs = 1 is
 *     the paper's literal per-body list);
 *   - self-interaction is excluded.
 *
 * Every floating-point expression whose result decides an integer (keys,
 * tree, opening decisions) is written out in a fixed order and this file
 * must be compiled with -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXD 3

/* ------------------------------------------------------------------------ */
/* Direct sum: the plain definition of the exact softened result (§3.1).    */
/* ------------------------------------------------------------------------ */

/* For each target t (an original body index): acc[t] = G sum_{j != t}
 * m_j (x_j - x_t) / (|x_j - x_t|^2 + eps^2)^{3/2} and
 * pot[t] = -G sum_{j != t} m_j / (|x_j - x_t|^2 + eps^2)^{1/2}.
 * pos is [n][dim] row-major.  Outputs are [nt][dim] and [nt]. */
void orc_direct(int64_t n, int dim, const double *pos, const double *mass,
                double G, double eps, int64_t nt, const int64_t *targets,
                double *acc, double *pot)
{
    const double e2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t i = targets ? targets[t] : t;
        double a[ORC_MAXD] = {0, 0, 0}, p = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[ORC_MAXD], r2 = e2;
            for (int k = 0; k < dim; ++k) {
                d[k] = pos[j * dim + k] - pos[i * dim + k];
                r2 += d[k] * d[k];
            }
            const double inv = 1.0 / sqrt(r2);
            const double w = mass[j] * inv;
            p -= w;
            const double w3 = w * inv * inv;
            for (int k = 0; k < dim; ++k) a[k] += w3 * d[k];
        }
        for (int k = 0; k < dim; ++k) acc[t * dim + k] = G * a[k];
        if (pot) pot[t] = G * p;
    }
}

/* ------------------------------------------------------------------------ */
/* Tree (§3.1): root cube, Morton digits, recursive subdivision, moments.   */
/* ------------------------------------------------------------------------ */

typedef struct orc_tree {
    int dim, L, leaf_cap;
    int64_t n;
    double lo[ORC_MAXD], size;
    uint64_t *key_orig;  /* key of each body, original order     */
    uint64_t *key;       /* keys in sorted order                  */
    uint32_t *perm;      /* sorted position -> original index     */
    double *x;           /* sorted positions [n][dim]             */
    double *m;           /* sorted masses [n]                     */
    int64_t ncells, cap;
    int32_t *level, *parent, *skip, *nch, *leaf;
    uint64_t *prefix;
    int64_t *begin, *count;
    double *M, *S, *com, *Q; /* per cell: M, S[dim], com[dim], Q[6] */
} orc_tree;

static int levels_for(int dim) { return dim == 3 ? 21 : 31; }

/* Root cube of the subdivided space. */
static void root_cube(int64_t n, int dim, const double *pos, double *lo, double *size)
{
    double hi[ORC_MAXD];
    for (int k = 0; k < dim; ++k) { lo[k] = pos[k]; hi[k] = pos[k]; }
    for (int64_t i = 1; i < n; ++i)
        for (int k = 0; k < dim; ++k) {
            const double v = pos[i * dim + k];
            if (v < lo[k]) lo[k] = v;
            if (v > hi[k]) hi[k] = v;
        }
    double ext = 0.0;
    for (int k = 0; k < dim; ++k) {
        const double e = hi[k] - lo[k];
        if (e > ext) ext = e;
    }
    if (ext == 0.0) { *size = 1.0; return; }
    int e2;
    const double f = frexp(ext, &e2);        /* ext = f * 2^e2, f in [0.5,1) */
    *size = (f == 0.5) ? ext : ldexp(1.0, e2);
}

/* Quantised coordinate along one axis: floor((x - lo) * 2^L / size),
 * clamped to 2^L - 1.  size is a power of two so the scale is exact. */
static uint64_t quantise(double x, double lo, double scale, int L)
{
    const double t = (x - lo) * scale;
    double f = floor(t);
    const double top = ldexp(1.0, L) - 1.0;
    if (f > top) f = top;
    if (f < 0.0) f = 0.0;
    return (uint64_t)f;
}

/* Morton key: level-major digits, level 1 most significant. */
static uint64_t morton(const uint64_t *q, int dim, int L)
{
    uint64_t key = 0;
    for (int l = 1; l <= L; ++l) {
        uint64_t digit = 0;
        for (int k = 0; k < dim; ++k)
            digit = (digit << 1) | ((q[k] >> (L - l)) & 1u);
        key = (key << dim) | digit;
    }
    return key;
}

typedef struct { uint64_t key; uint32_t idx; } kv_t;

static int kv_cmp(const void *a, const void *b)
{
    const kv_t *x = (const kv_t *)a, *y = (const kv_t *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

static void grow(orc_tree *t)
{
    int64_t c = t->cap ? t->cap * 2 : 1024;
    t->level = realloc(t->level, c * sizeof(int32_t));
    t->parent = realloc(t->parent, c * sizeof(int32_t));
    t->skip = realloc(t->skip, c * sizeof(int32_t));
    t->nch = realloc(t->nch, c * sizeof(int32_t));
    t->leaf = realloc(t->leaf, c * sizeof(int32_t));
    t->prefix = realloc(t->prefix, c * sizeof(uint64_t));
    t->begin = realloc(t->begin, c * sizeof(int64_t));
    t->count = realloc(t->count, c * sizeof(int64_t));
    t->cap = c;
}

/* The digit of a key at level l (1..L). */
static unsigned digit_at(uint64_t key, int dim, int L, int l)
{
    return (unsigned)((key >> (dim * (L - l))) & ((1u << dim) - 1u));
}

/* Recursive subdivision of a cell holding sorted bodies [b, e): the cell is
 * emitted in pre-order, then, if it holds more than leaf_cap bodies and is
 * above level L, split into its non-empty subspaces in digit order. */
static void subdivide(orc_tree *t, int level, uint64_t prefix, int64_t b, int64_t e, int32_t parent)
{
    if (t->ncells == t->cap) grow(t);
    const int64_t c = t->ncells++;
    t->level[c] = level;
    t->prefix[c] = prefix;
    t->begin[c] = b;
    t->count[c] = e - b;
    t->parent[c] = parent;
    t->nch[c] = 0;
    const int split = (e - b) > t->leaf_cap && level < t->L;
    t->leaf[c] = !split;
    if (split) {
        int64_t s = b;
        while (s < e) {
            const unsigned d = digit_at(t->key[s], t->dim, t->L, level + 1);
            int64_t f = s;
            while (f < e && digit_at(t->key[f], t->dim, t->L, level + 1) == d) ++f;
            t->nch[c] += 1;
            subdivide(t, level + 1, (prefix << t->dim) | d, s, f, (int32_t)c);
            s = f;
        }
    }
    t->skip[c] = (int32_t)t->ncells;
}

/* Cell monopole (§3.1: total mass at the centre of mass) and the traceless
 * quadrupole, bottom-up.  Leaves sum their bodies in sorted order; internal
 * cells sum their children in digit order.  Q is (xx, yy, zz, xy, xz, yz),
 * Q_ab = sum m (3 d_a d_b - |d|^2 delta_ab) about the cell's centre of mass,
 * moved from children by the parallel-axis shift.  3D only (zero in 2D). */
static void moments(orc_tree *t, int64_t c)
{
    const int D = t->dim;
    double M = 0.0, S[ORC_MAXD] = {0, 0, 0}, Q[6] = {0, 0, 0, 0, 0, 0};
    if (t->leaf[c]) {
        for (int64_t j = t->begin[c]; j < t->begin[c] + t->count[c]; ++j) {
            M = M + t->m[j];
            for (int k = 0; k < D; ++k) S[k] = S[k] + t->m[j] * t->x[j * D + k];
        }
        double com[ORC_MAXD];
        for (int k = 0; k < D; ++k) com[k] = S[k] / M;
        if (D == 3) {
            for (int64_t j = t->begin[c]; j < t->begin[c] + t->count[c]; ++j) {
                double d[3];
                for (int k = 0; k < 3; ++k) d[k] = t->x[j * 3 + k] - com[k];
                const double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
                const double mj = t->m[j];
                Q[0] = Q[0] + mj * ((3.0 * d[0]) * d[0] - r2);
                Q[1] = Q[1] + mj * ((3.0 * d[1]) * d[1] - r2);
                Q[2] = Q[2] + mj * ((3.0 * d[2]) * d[2] - r2);
                Q[3] = Q[3] + mj * ((3.0 * d[0]) * d[1]);
                Q[4] = Q[4] + mj * ((3.0 * d[0]) * d[2]);
                Q[5] = Q[5] + mj * ((3.0 * d[1]) * d[2]);
            }
        }
        t->M[c] = M;
        for (int k = 0; k < D; ++k) { t->S[c * D + k] = S[k]; t->com[c * D + k] = com[k]; }
        for (int k = 0; k < 6; ++k) t->Q[c * 6 + k] = Q[k];
        return;
    }
    for (int64_t ch = c + 1; ch < t->skip[c]; ch = t->skip[ch]) moments(t, ch);
    for (int64_t ch = c + 1; ch < t->skip[c]; ch = t->skip[ch]) {
        M = M + t->M[ch];
        for (int k = 0; k < D; ++k) S[k] = S[k] + t->S[ch * D + k];
    }
    double com[ORC_MAXD];
    for (int k = 0; k < D; ++k) com[k] = S[k] / M;
    if (D == 3) {
        for (int64_t ch = c + 1; ch < t->skip[c]; ch = t->skip[ch]) {
            double s[3];
            for (int k = 0; k < 3; ++k) s[k] = t->com[ch * 3 + k] - com[k];
            const double r2 = (s[0] * s[0] + s[1] * s[1]) + s[2] * s[2];
            const double Mc = t->M[ch];
            const double *q = t->Q + ch * 6;
            Q[0] = Q[0] + (q[0] + Mc * ((3.0 * s[0]) * s[0] - r2));
            Q[1] = Q[1] + (q[1] + Mc * ((3.0 * s[1]) * s[1] - r2));
            Q[2] = Q[2] + (q[2] + Mc * ((3.0 * s[2]) * s[2] - r2));
            Q[3] = Q[3] + (q[3] + Mc * ((3.0 * s[0]) * s[1]));
            Q[4] = Q[4] + (q[4] + Mc * ((3.0 * s[0]) * s[2]));
            Q[5] = Q[5] + (q[5] + Mc * ((3.0 * s[1]) * s[2]));
        }
    }
    t->M[c] = M;
    for (int k = 0; k < D; ++k) { t->S[c * D + k] = S[k]; t->com[c * D + k] = com[k]; }
    for (int k = 0; k < 6; ++k) t->Q[c * 6 + k] = Q[k];
}

/* Build the tree of n bodies.  pos is [n][dim] (FP64, original order).
 * Returns NULL on bad arguments. */
orc_tree *orc_tree_build(int64_t n, int dim, const double *pos, const double *mass, int leaf_cap)
{
    if (n < 1 || (dim != 2 && dim != 3) || leaf_cap < 1) return NULL;
    orc_tree *t = calloc(1, sizeof(orc_tree));
    t->dim = dim;
    t->L = levels_for(dim);
    t->leaf_cap = leaf_cap;
    t->n = n;
    root_cube(n, dim, pos, t->lo, &t->size);
    int e2;
    frexp(t->size, &e2);                        /* size = 2^(e2-1) */
    const double scale = ldexp(1.0, t->L - (e2 - 1));
    t->key_orig = malloc(n * sizeof(uint64_t));
    kv_t *kv = malloc(n * sizeof(kv_t));
    for (int64_t i = 0; i < n; ++i) {
        uint64_t q[ORC_MAXD];
        for (int k = 0; k < dim; ++k) q[k] = quantise(pos[i * dim + k], t->lo[k], scale, t->L);
        t->key_orig[i] = morton(q, dim, t->L);
        kv[i].key = t->key_orig[i];
        kv[i].idx = (uint32_t)i;
    }
    qsort(kv, n, sizeof(kv_t), kv_cmp);      /* stable by (key, original index) */
    t->key = malloc(n * sizeof(uint64_t));
    t->perm = malloc(n * sizeof(uint32_t));
    t->x = malloc(n * dim * sizeof(double));
    t->m = malloc(n * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        t->key[i] = kv[i].key;
        t->perm[i] = kv[i].idx;
        for (int k = 0; k < dim; ++k) t->x[i * dim + k] = pos[(int64_t)kv[i].idx * dim + k];
        t->m[i] = mass[kv[i].idx];
    }
    free(kv);
    subdivide(t, 0, 0, 0, n, -1);
    t->M = malloc(t->ncells * sizeof(double));
    t->S = malloc(t->ncells * dim * sizeof(double));
    t->com = malloc(t->ncells * dim * sizeof(double));
    t->Q = malloc(t->ncells * 6 * sizeof(double));
    moments(t, 0);
    return t;
}

void orc_tree_free(orc_tree *t)
{
    if (!t) return;
    free(t->key_orig); free(t->key); free(t->perm); free(t->x); free(t->m);
    free(t->level); free(t->parent); free(t->skip); free(t->nch); free(t->leaf);
    free(t->prefix); free(t->begin); free(t->count);
    free(t->M); free(t->S); free(t->com); free(t->Q);
    free(t);
}

int64_t orc_tree_ncells(const orc_tree *t) { return t->ncells; }

void orc_tree_root(const orc_tree *t, double *lo, double *size)
{
    for (int k = 0; k < t->dim; ++k) lo[k] = t->lo[k];
    *size = t->size;
}

/* Copy out the body-order arrays (any pointer may be NULL). */
void orc_tree_bodies(const orc_tree *t, uint64_t *key_orig, uint64_t *key, uint32_t *perm)
{
    if (key_orig) memcpy(key_orig, t->key_orig, t->n * sizeof(uint64_t));
    if (key) memcpy(key, t->key, t->n * sizeof(uint64_t));
    if (perm) memcpy(perm, t->perm, t->n * sizeof(uint32_t));
}

/* Copy out the per-cell arrays in pre-order (any pointer may be NULL). */
void orc_tree_cells(const orc_tree *t, int32_t *level, uint64_t *prefix, int64_t *begin,
                    int64_t *count, int32_t *parent, int32_t *skip, int32_t *nch, int32_t *leaf,
                    double *M, double *com, double *Q)
{
    const int64_t C = t->ncells;
    if (level) memcpy(level, t->level, C * sizeof(int32_t));
    if (prefix) memcpy(prefix, t->prefix, C * sizeof(uint64_t));
    if (begin) memcpy(begin, t->begin, C * sizeof(int64_t));
    if (count) memcpy(count, t->count, C * sizeof(int64_t));
    if (parent) memcpy(parent, t->parent, C * sizeof(int32_t));
    if (skip) memcpy(skip, t->skip, C * sizeof(int32_t));
    if (nch) memcpy(nch, t->nch, C * sizeof(int32_t));
    if (leaf) memcpy(leaf, t->leaf, C * sizeof(int32_t));
    if (M) memcpy(M, t->M, C * sizeof(double));
    if (com) memcpy(com, t->com, C * t->dim * sizeof(double));
    if (Q) memcpy(Q, t->Q, C * 6 * sizeof(double));
}

/* ------------------------------------------------------------------------ */
/* Opening criterion and walk (§3.1).                                       */
/* ------------------------------------------------------------------------ */

/* Squared opening radius of every cell for a given theta:
 * r = s_c / theta + |com_c - centre_c|, s_c = size / 2^level the cell side,
 * centre_c the geometric centre of the cell's subspace.  theta = 0 gives
 * +infinity (nothing is accepted). */
void orc_mac_radii(const orc_tree *t, double theta, double *rcrit2)
{
    const int D = t->dim;
    for (int64_t c = 0; c < t->ncells; ++c) {
        if (theta == 0.0) { rcrit2[c] = INFINITY; continue; }
        const int l = t->level[c];
        const double s = ldexp(t->size, -l);
        /* the cell's integer origin along each axis, from its key prefix */
        uint64_t org[ORC_MAXD] = {0, 0, 0};
        for (int j = 1; j <= l; ++j) {
            const unsigned d = (unsigned)((t->prefix[c] >> (D * (l - j))) & ((1u << D) - 1u));
            for (int k = 0; k < D; ++k)
                org[k] = (org[k] << 1) | ((d >> (D - 1 - k)) & 1u);
        }
        double dd[ORC_MAXD] = {0, 0, 0};
        for (int k = 0; k < D; ++k) {
            const double centre = t->lo[k] + ((double)org[k] + 0.5) * s;
            dd[k] = t->com[c * D + k] - centre;
        }
        double d2 = dd[0] * dd[0] + dd[1] * dd[1];
        if (D == 3) d2 = d2 + dd[2] * dd[2];
        const double r = s / theta + sqrt(d2);
        rcrit2[c] = r * r;
    }
}

/* Group bounding box of sorted bodies [b, e). */
static void group_box(const orc_tree *t, int64_t b, int64_t e, double *lo, double *hi)
{
    const int D = t->dim;
    for (int k = 0; k < D; ++k) { lo[k] = t->x[b * D + k]; hi[k] = lo[k]; }
    for (int64_t j = b + 1; j < e; ++j)
        for (int k = 0; k < D; ++k) {
            const double v = t->x[j * D + k];
            if (v < lo[k]) lo[k] = v;
            if (v > hi[k]) hi[k] = v;
        }
}

/* The opening decision: accept iff dist^2(com, box) > rcrit2, strict. */
static int accepts(const orc_tree *t, int64_t c, const double *rcrit2, const double *lo, const double *hi)
{
    const int D = t->dim;
    double d[ORC_MAXD] = {0, 0, 0};
    for (int k = 0; k < D; ++k) {
        const double x = t->com[c * D + k];
        const double below = lo[k] - x, above = x - hi[k];
        double v = 0.0;
        if (below > v) v = below;
        if (above > v) v = above;
        d[k] = v;
    }
    double d2 = d[0] * d[0] + d[1] * d[1];
    if (D == 3) d2 = d2 + d[2] * d[2];
    return d2 > rcrit2[c];
}

typedef struct {
    int32_t *items;       /* terminal cells in walk order; -1-c marks a P2P leaf c */
    int64_t nitems, cap;
    int64_t m2p, p2p;     /* accepted cells, bodies from opened leaves */
    int64_t tests;        /* cells whose opening test ran */
} walk_out;

static void push_item(walk_out *w, int32_t v)
{
    if (w->items) {
        if (w->nitems == w->cap) {
            w->cap = w->cap ? 2 * w->cap : 256;
            w->items = realloc(w->items, w->cap * sizeof(int32_t));
        }
        w->items[w->nitems] = v;
    }
    w->nitems++;
}

/* Walk from cell c (recursive descent, §3.1). */
static void walk_rec(const orc_tree *t, int64_t c, const double *rcrit2, const double *lo,
                     const double *hi, walk_out *w)
{
    w->tests += 1;
    if (accepts(t, c, rcrit2, lo, hi)) {
        w->m2p += 1;
        push_item(w, (int32_t)c);
        return;
    }
    if (t->leaf[c]) {
        w->p2p += t->count[c];
        push_item(w, (int32_t)(-1 - c));
        return;
    }
    for (int64_t ch = c + 1; ch < t->skip[c]; ch = t->skip[ch]) walk_rec(t, ch, rcrit2, lo, hi, w);
}

static void walk_range(const orc_tree *t, const double *rcrit2, int64_t b, int64_t e, walk_out *w)
{
    double lo[ORC_MAXD], hi[ORC_MAXD];
    group_box(t, b, e, lo, hi);
    walk_rec(t, 0, rcrit2, lo, hi, w);
}

static void walk_group(const orc_tree *t, const double *rcrit2, int gs, int64_t g, walk_out *w)
{
    const int64_t b = g * gs, e = (b + gs < t->n) ? b + gs : t->n;
    walk_range(t, rcrit2, b, e, w);
}

/* Groups of at most gs consecutive sorted bodies that never straddle a
 * cluster cell, a maximal cell holding at most kc bodies: the bodies of each
 * cluster cell, in order, are cut into runs of gs (the last run shorter).
 * Writes the groups' first body and size (when the arrays are not NULL) and
 * returns their number. */
int64_t orc_groups(const orc_tree *t, int gs, int64_t kc, int64_t *gbeg, int64_t *gcnt)
{
    int64_t ng = 0;
    for (int64_t c = 0; c < t->ncells;) {
        if (t->count[c] <= kc || t->leaf[c]) {
            for (int64_t o = 0; o < t->count[c]; o += gs) {
                if (gbeg) gbeg[ng] = t->begin[c] + o;
                if (gcnt) gcnt[ng] = (t->count[c] - o < gs) ? t->count[c] - o : gs;
                ++ng;
            }
            c = t->skip[c];
        } else {
            c = c + 1;
        }
    }
    return ng;
}

/* Number of accepted cells (m2p) and of bodies from opened leaves (p2p,
 * the group's own bodies included) for every group of gs sorted bodies. */
void orc_walk_counts(const orc_tree *t, double theta, int gs, int64_t *m2p, int64_t *p2p)
{
    double *rc = malloc(t->ncells * sizeof(double));
    orc_mac_radii(t, theta, rc);
    const int64_t G = (t->n + gs - 1) / gs;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t g = 0; g < G; ++g) {
        walk_out w = {0};
        walk_group(t, rc, gs, g, &w);
        m2p[g] = w.m2p;
        p2p[g] = w.p2p;
    }
    free(rc);
}

/* The same for explicit groups: group k holds sorted bodies
 * [gbeg[k], gbeg[k] + gcnt[k]). */
void orc_walk_counts_ranges(const orc_tree *t, double theta, int64_t ng, const int64_t *gbeg,
                            const int64_t *gcnt, int64_t *m2p, int64_t *p2p)
{
    double *rc = malloc(t->ncells * sizeof(double));
    orc_mac_radii(t, theta, rc);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t g = 0; g < ng; ++g) {
        walk_out w = {0};
        walk_range(t, rc, gbeg[g], gbeg[g] + gcnt[g], &w);
        m2p[g] = w.m2p;
        p2p[g] = w.p2p;
    }
    free(rc);
}

/* Cells whose opening test ran in the walk of each explicit group (a
 * measurement of the walk's work, not part of the method): the root and
 * every child of an opened cell. */
void orc_walk_tests_ranges(const orc_tree *t, double theta, int64_t ng, const int64_t *gbeg,
                           const int64_t *gcnt, int64_t *tests)
{
    double *rc = malloc(t->ncells * sizeof(double));
    orc_mac_radii(t, theta, rc);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t g = 0; g < ng; ++g) {
        walk_out w = {0};
        walk_range(t, rc, gbeg[g], gbeg[g] + gcnt[g], &w);
        tests[g] = w.tests;
    }
    free(rc);
}

/* The terminal items of one group's walk, in walk order: c >= 0 is an
 * accepted cell, -1-c an opened leaf whose bodies interact directly.
 * Returns the item count; writes at most cap items. */
int64_t orc_walk_items(const orc_tree *t, double theta, int gs, int64_t g, int32_t *out, int64_t cap)
{
    double *rc = malloc(t->ncells * sizeof(double));
    orc_mac_radii(t, theta, rc);
    walk_out w = {0};
    w.items = malloc(256 * sizeof(int32_t));
    w.cap = 256;
    walk_group(t, rc, gs, g, &w);
    for (int64_t k = 0; k < w.nitems && k < cap; ++k) out[k] = w.items[k];
    free(w.items);
    free(rc);
    return w.nitems;
}

/* Forces on the bodies of one group (sorted [b, e)): the sum over the
 * group's list of the softened point-mass interaction, cells as
 * pseudo-bodies of mass M at their centre of mass (§3.1). */
/* Forces on the sorted bodies [b, e) from their group's walk.  With
 * order 2 (3D) an accepted cell also contributes its quadrupole term: for
 * d = C - x (cell centre of mass minus body), softened 1/r = s =
 * (|d|^2 + eps^2)^{-1/2} and the traceless Q = sum m (3 dd - |d|^2 I),
 *   a_Q = G [ -Q d s^5 + (5/2) (d.Q d) d s^7 ],  phi_Q = -(G/2) (d.Q d) s^5,
 * the second term of the expansion of -G sum m / |x - x_j| about C with 1/r
 * replaced by its softened value. */
static void group_forces(const orc_tree *t, const double *rc, int64_t b, int64_t e, double G,
                         double e2, int order, double *acc, double *pot)
{
    const int D = t->dim;
    walk_out w = {0};
    w.items = malloc(256 * sizeof(int32_t));
    w.cap = 256;
    walk_range(t, rc, b, e, &w);
    for (int64_t i = b; i < e; ++i) {
        double a[ORC_MAXD] = {0, 0, 0}, p = 0.0;
        const double *xi = t->x + i * D;
        for (int64_t k = 0; k < w.nitems; ++k) {
            const int32_t it = w.items[k];
            int64_t jb, je;
            const double *src, *ms;
            if (it >= 0) { jb = it; je = it + 1; src = t->com; ms = t->M; }
            else { const int64_t c = -1 - it; jb = t->begin[c]; je = jb + t->count[c]; src = t->x; ms = t->m; }
            for (int64_t j = jb; j < je; ++j) {
                if (it < 0 && j == i) continue;
                double d[ORC_MAXD], r2 = e2;
                for (int q = 0; q < D; ++q) { d[q] = src[j * D + q] - xi[q]; r2 += d[q] * d[q]; }
                const double inv = 1.0 / sqrt(r2);
                const double wv = ms[j] * inv;
                p -= wv;
                const double w3 = wv * inv * inv;
                for (int q = 0; q < D; ++q) a[q] += w3 * d[q];
                if (order == 2 && D == 3 && it >= 0) {
                    const double *Q = t->Q + (int64_t)j * 6;     /* xx yy zz xy xz yz */
                    const double qd[3] = {Q[0] * d[0] + Q[3] * d[1] + Q[4] * d[2],
                                          Q[3] * d[0] + Q[1] * d[1] + Q[5] * d[2],
                                          Q[4] * d[0] + Q[5] * d[1] + Q[2] * d[2]};
                    const double dqd = d[0] * qd[0] + d[1] * qd[1] + d[2] * qd[2];
                    const double s2 = inv * inv, s5 = s2 * s2 * inv, s7 = s5 * s2;
                    for (int q = 0; q < 3; ++q) a[q] += -qd[q] * s5 + 2.5 * dqd * d[q] * s7;
                    p -= 0.5 * dqd * s5;
                }
            }
        }
        const int64_t o = t->perm[i];
        for (int q = 0; q < D; ++q) acc[o * D + q] = G * a[q];
        if (pot) pot[o] = G * p;
    }
    free(w.items);
}

/* The terminal items of the walk of sorted bodies [b, e), in walk order
 * (c >= 0 accepted cell, -1-c opened leaf c).  Returns the item count;
 * writes at most cap items. */
int64_t orc_walk_items_range(const orc_tree *t, double theta, int64_t b, int64_t e, int32_t *out, int64_t cap)
{
    double *rc = malloc(t->ncells * sizeof(double));
    orc_mac_radii(t, theta, rc);
    walk_out w = {0};
    w.items = malloc(256 * sizeof(int32_t));
    w.cap = 256;
    walk_range(t, rc, b, e, &w);
    for (int64_t k = 0; k < w.nitems && k < cap; ++k) out[k] = w.items[k];
    free(w.items);
    free(rc);
    return w.nitems;
}

/* Treecode forces for the bodies of the selected groups of gs consecutive
 * sorted bodies (all groups when groups == NULL).  acc [n][dim] and pot [n]
 * are in original body order; only the selected groups' bodies are
 * written. */
void orc_tree_forces(const orc_tree *t, double theta, int gs, double G, double eps,
                     int64_t ngsel, const int64_t *groups, double *acc, double *pot)
{
    double *rc = malloc(t->ncells * sizeof(double));
    orc_mac_radii(t, theta, rc);
    const int64_t NG = groups ? ngsel : (t->n + gs - 1) / gs;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t s = 0; s < NG; ++s) {
        const int64_t g = groups ? groups[s] : s;
        const int64_t b = g * gs, e = (b + gs < t->n) ? b + gs : t->n;
        group_forces(t, rc, b, e, G, eps * eps, 1, acc, pot);
    }
    free(rc);
}

/* The same for explicit groups [gbeg[k], gbeg[k] + gcnt[k]), k < ng. */
void orc_tree_forces_ranges(const orc_tree *t, double theta, double G, double eps, int64_t ng,
                            const int64_t *gbeg, const int64_t *gcnt, int order, double *acc, double *pot)
{
    double *rc = malloc(t->ncells * sizeof(double));
    orc_mac_radii(t, theta, rc);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < ng; ++k)
        group_forces(t, rc, gbeg[k], gbeg[k] + gcnt[k], G, eps * eps, order, acc, pot);
    free(rc);
}

/* ------------------------------------------------------------------------ */
/* Learned closure: training pairs (features and normalised residuals).      */
/* ------------------------------------------------------------------------ */

/* For each target (a sorted body position p) the walk of the one-body group
 * [p, p+1) at theta gives the accepted cells.  For each accepted cell c with
 * centre of mass C, mass M, side s, traceless quadrupole Q:
 *   features  (x - C)/s (3), Q/(M s^2) (6: xx yy zz xy xz yz), ln(M / mbar)
 *             with mbar = (total mass)/n,
 *   residual  y = (a_exact - a_mono) |x - C|^4 / (M s^2), where a_exact is
 *             the softened sum over the cell's bodies and a_mono = M (C - x) /
 *             (|C - x|^2 + eps^2)^{3/2} (G = 1): the residual in units of the
 *             quadrupole scale M s^2 / |x - C|^4, so targets are of order
 *             |Q| / (M s^2) at every distance.
 * Pairs are in target order, then in walk order.  Writes at most cap pairs
 * (feat [cap][10] FP32, y [cap][3] FP64, target index and cell), count[t]
 * per target; returns the total number of pairs.  3D only. */
int64_t orc_residuals(const orc_tree *t, double theta, double eps, int64_t nt, const int64_t *tpos,
                      int64_t cap, float *feat, double *y, int64_t *tgt, int32_t *cell, int64_t *count)
{
    if (t->dim != 3) return -1;
    const double e2 = eps * eps;
    const double mbar = t->M[0] / (double)t->n;
    double *rc = malloc(t->ncells * sizeof(double));
    orc_mac_radii(t, theta, rc);
    int64_t *off = malloc((nt + 1) * sizeof(int64_t));
    walk_out *ws = calloc(nt, sizeof(walk_out));
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < nt; ++k) {
        ws[k].items = malloc(256 * sizeof(int32_t));
        ws[k].cap = 256;
        walk_range(t, rc, tpos[k], tpos[k] + 1, &ws[k]);
    }
    off[0] = 0;
    for (int64_t k = 0; k < nt; ++k) {
        count[k] = ws[k].m2p;
        off[k + 1] = off[k] + ws[k].m2p;
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < nt; ++k) {
        const int64_t p = tpos[k];
        const double *x = t->x + p * 3;
        int64_t o = off[k];
        for (int64_t it = 0; it < ws[k].nitems; ++it) {
            const int32_t c = ws[k].items[it];
            if (c < 0) continue;
            if (o < cap) {
                const double *C = t->com + (int64_t)c * 3;
                const double M = t->M[c];
                const double s = ldexp(t->size, -t->level[c]);
                double ex[3] = {0, 0, 0};
                for (int64_t j = t->begin[c]; j < t->begin[c] + t->count[c]; ++j) {
                    double d[3], r2 = e2;
                    for (int q = 0; q < 3; ++q) { d[q] = t->x[j * 3 + q] - x[q]; r2 += d[q] * d[q]; }
                    const double inv = 1.0 / sqrt(r2);
                    const double w3 = t->m[j] * inv * inv * inv;
                    for (int q = 0; q < 3; ++q) ex[q] += w3 * d[q];
                }
                double dc[3], d2 = 0.0;
                for (int q = 0; q < 3; ++q) { dc[q] = C[q] - x[q]; d2 += dc[q] * dc[q]; }
                const double inv = 1.0 / sqrt(d2 + e2);
                const double w3 = M * inv * inv * inv;
                for (int q = 0; q < 3; ++q) y[o * 3 + q] = (ex[q] - w3 * dc[q]) * (d2 * d2) / (M * s * s);
                for (int q = 0; q < 3; ++q) feat[o * 10 + q] = (float)((x[q] - C[q]) / s);
                const double qs = M * s * s;
                for (int q = 0; q < 6; ++q) feat[o * 10 + 3 + q] = (float)(t->Q[(int64_t)c * 6 + q] / qs);
                feat[o * 10 + 9] = (float)log(M / mbar);
                tgt[o] = k;
                cell[o] = c;
            }
            ++o;
        }
        free(ws[k].items);
    }
    const int64_t total = off[nt];
    free(ws);
    free(off);
    free(rc);
    return total;
}

/* Sorted position of each of the given original body indices. */
void orc_sorted_positions(const orc_tree *t, int64_t k, const int64_t *orig, int64_t *pos)
{
    int64_t *inv = malloc(t->n * sizeof(int64_t));
    for (int64_t i = 0; i < t->n; ++i) inv[t->perm[i]] = i;
    for (int64_t j = 0; j < k; ++j) pos[j] = inv[orig[j]];
    free(inv);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the number of OpenMP threads used by later calls (benchmarking). */
void orc_set_num_threads(int k)
{
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

/* ------------------------------------------------------------------------ */
/* Fast multipole method (§5 names it as the way beyond the treecode's      */
/* O(N log N)).  The paper gives no algorithm, so this is the textbook      */
/* Cartesian form (Greengard & Rokhlin 1987; Dehnen 2002), 3D only:         */
/*                                                                          */
/*   - every cell carries its multipole about its centre of mass (M, Q: the */
/*     dipole vanishes there; Q is the traceless quadrupole, whose trace    */
/*     part would only act through the softening) and a local expansion     */
/*     about its geometric centre z: the coefficients Lam_n (n = 0..3) of   */
/*       phi(z + dl) = -G sum_n (1/n!) Lam_n[dl^n],                         */
/*       a(z + dl)   =  G sum_{n>=1} (1/(n-1)!) Lam_n[dl^(n-1), .];         */
/*   - g(R) = (|R|^2 + eps^2)^(-1/2) and D_n = its n-th derivative tensor;  */
/*     a source cell B acting on a target cell A with R = z_A - com_B adds  */
/*       Lam_n += M D_n(R) + (1/6) Q : D_(n+2)(R)   (the second term only   */
/*     while n + 2 <= 3), the expansion truncated at total order 3 (M2L);   */
/*   - a child's expansion receives its parent's, moved by t = z_c - z_p:   */
/*       Lam'_n += sum_k (1/k!) Lam_(n+k)[t^k]  (L2L), top-down;            */
/*   - the dual tree traversal from the pair (root, root): a cell with      */
/*     itself splits into all pairs of its children (a leaf: direct sum);  */
/*     a pair is accepted for M2L iff |z_A - com_B| > (rho_A + rho_B)/theta */
/*     (strict), with rho_A bounding A's bodies about z_A and rho_B bounding */
/*     B's bodies about com_B: for a leaf the largest distance of one of    */
/*     its bodies, for an internal cell the largest over its children of    */
/*     (distance between the two centres + the child's radius), each        */
/*     capped by the geometric bound ((sqrt 3 / 2) s about z, plus         */
/*     |com - z| about com); otherwise two leaves sum directly (P2P) and    */
/*     otherwise the                                                        */
/*     larger cell (smaller level; the target on a tie, or whichever is not */
/*     a leaf) is split into its children.  theta = 0 accepts nothing, and  */
/*     the result is the direct sum;                                        */
/*   - a body's force is its leaf's expansion evaluated at the body (L2P)   */
/*     plus the direct sums over its leaf's P2P partners, self excluded.    */
/* ------------------------------------------------------------------------ */

#define ORC_HALF_SQRT3 0.8660254037844386

/* Geometric centre of cell c's subspace. */
static void cell_centre(const orc_tree *t, int64_t c, double *ctr)
{
    const int D = t->dim, l = t->level[c];
    const double s = ldexp(t->size, -l);
    uint64_t org[ORC_MAXD] = {0, 0, 0};
    for (int j = 1; j <= l; ++j) {
        const unsigned d = (unsigned)((t->prefix[c] >> (D * (l - j))) & ((1u << D) - 1u));
        for (int k = 0; k < D; ++k) org[k] = (org[k] << 1) | ((d >> (D - 1 - k)) & 1u);
    }
    for (int k = 0; k < D; ++k) ctr[k] = t->lo[k] + ((double)org[k] + 0.5) * s;
}

typedef struct {
    const orc_tree *t;
    double theta;
    double *ctr, *rhoA, *rhoB;    /* per cell */
    int32_t *m2l, *p2p;           /* (target, source) pairs, pre-order ids */
    int64_t nm2l, np2p, cap_m, cap_p;
} fmm_ctx;

static void fmm_push(int32_t *arr, int64_t *n, int64_t cap, int64_t a, int64_t b)
{
    if (*n < cap) {
        arr[2 * *n] = (int32_t)a;
        arr[2 * *n + 1] = (int32_t)b;
    }
    *n += 1;
}

static int fmm_accept(const fmm_ctx *f, int64_t A, int64_t B)
{
    if (f->theta == 0.0) return 0;
    double d[3];
    for (int k = 0; k < 3; ++k) d[k] = f->ctr[A * 3 + k] - f->t->com[B * 3 + k];
    const double d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    const double r = (f->rhoA[A] + f->rhoB[B]) / f->theta;
    return d2 > r * r;
}

static void fmm_rec(fmm_ctx *f, int64_t A, int64_t B)
{
    const orc_tree *t = f->t;
    if (A == B) {
        if (t->leaf[A]) {
            fmm_push(f->p2p, &f->np2p, f->cap_p, A, A);
            return;
        }
        for (int64_t a = A + 1; a < t->skip[A]; a = t->skip[a])
            for (int64_t b = A + 1; b < t->skip[A]; b = t->skip[b]) fmm_rec(f, a, b);
        return;
    }
    if (fmm_accept(f, A, B)) {
        fmm_push(f->m2l, &f->nm2l, f->cap_m, A, B);
        return;
    }
    if (t->leaf[A] && t->leaf[B]) {
        fmm_push(f->p2p, &f->np2p, f->cap_p, A, B);
        return;
    }
    if (!t->leaf[A] && (t->leaf[B] || t->level[A] <= t->level[B])) {
        for (int64_t a = A + 1; a < t->skip[A]; a = t->skip[a]) fmm_rec(f, a, B);
    } else {
        for (int64_t b = B + 1; b < t->skip[B]; b = t->skip[b]) fmm_rec(f, A, b);
    }
}

static double dist3(const double *a, const double *b)
{
    double d[3];
    for (int k = 0; k < 3; ++k) d[k] = a[k] - b[k];
    return sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
}

static void fmm_setup(fmm_ctx *f, const orc_tree *t, double theta)
{
    memset(f, 0, sizeof(*f));
    f->t = t;
    f->theta = theta;
    f->ctr = malloc(t->ncells * 3 * sizeof(double));
    f->rhoA = malloc(t->ncells * sizeof(double));
    f->rhoB = malloc(t->ncells * sizeof(double));
    for (int64_t c = 0; c < t->ncells; ++c) cell_centre(t, c, f->ctr + c * 3);
    /* children follow their parent in pre-order: go backwards */
    for (int64_t c = t->ncells - 1; c >= 0; --c) {
        const double *z = f->ctr + c * 3, *com = t->com + c * 3;
        double ra = 0.0, rb = 0.0;
        if (t->leaf[c]) {
            for (int64_t j = t->begin[c]; j < t->begin[c] + t->count[c]; ++j) {
                const double da = dist3(t->x + j * 3, z), db = dist3(t->x + j * 3, com);
                if (da > ra) ra = da;
                if (db > rb) rb = db;
            }
        } else {
            for (int64_t ch = c + 1; ch < t->skip[c]; ch = t->skip[ch]) {
                const double da = dist3(f->ctr + ch * 3, z) + f->rhoA[ch];
                const double db = dist3(t->com + ch * 3, com) + f->rhoB[ch];
                if (da > ra) ra = da;
                if (db > rb) rb = db;
            }
        }
        const double s = ldexp(t->size, -t->level[c]);
        const double ga = ORC_HALF_SQRT3 * s, gb = ORC_HALF_SQRT3 * s + dist3(com, z);
        f->rhoA[c] = ra < ga ? ra : ga;
        f->rhoB[c] = rb < gb ? rb : gb;
    }
}

static void fmm_teardown(fmm_ctx *f)
{
    free(f->ctr);
    free(f->rhoA);
    free(f->rhoB);
}

/* The interaction pairs of the dual tree traversal at theta, in traversal
 * order: m2l[2k], m2l[2k+1] = (target, source) pre-order cell ids, at most
 * cap_m pairs written (likewise p2p).  Returns 0 (counts in n_m2l, n_p2p),
 * or -1 for a 2D tree. */
int orc_fmm_pairs(const orc_tree *t, double theta, int32_t *m2l, int64_t cap_m, int32_t *p2p, int64_t cap_p,
                  int64_t *n_m2l, int64_t *n_p2p)
{
    if (t->dim != 3) return -1;
    fmm_ctx f;
    fmm_setup(&f, t, theta);
    f.m2l = m2l;
    f.p2p = p2p;
    f.cap_m = cap_m;
    f.cap_p = cap_p;
    fmm_rec(&f, 0, 0);
    *n_m2l = f.nm2l;
    *n_p2p = f.np2p;
    fmm_teardown(&f);
    return 0;
}

/* Local expansion coefficients, full tensors: lam[0] = Lam_0,
 * lam[1 + a] = Lam_1, lam[4 + 3a + b] = Lam_2, lam[13 + 9a + 3b + c] = Lam_3. */
#define FMM_NL 40
#define L1(a) (1 + (a))
#define L2(a, b) (4 + 3 * (a) + (b))
#define L3(a, b, c) (13 + 9 * (a) + 3 * (b) + (c))

/* M2L: add to lam the expansion about a point R away from a source of mass
 * M and traceless quadrupole Q6 = (xx, yy, zz, xy, xz, yz) at its centre of
 * mass (R = target centre - source centre of mass). */
void orc_fmm_m2l(double M, const double *Q6, const double *R, double eps, double *lam)
{
    const double r2 = ((R[0] * R[0] + R[1] * R[1]) + R[2] * R[2]) + eps * eps;
    const double s = 1.0 / sqrt(r2);
    const double s3 = s * s * s, s5 = s3 * s * s, s7 = s5 * s * s;
    double D1[3], D2[3][3], D3[3][3][3], Q[3][3];
    Q[0][0] = Q6[0]; Q[1][1] = Q6[1]; Q[2][2] = Q6[2];
    Q[0][1] = Q[1][0] = Q6[3];
    Q[0][2] = Q[2][0] = Q6[4];
    Q[1][2] = Q[2][1] = Q6[5];
    for (int a = 0; a < 3; ++a) {
        D1[a] = -R[a] * s3;
        for (int b = 0; b < 3; ++b) {
            D2[a][b] = 3.0 * R[a] * R[b] * s5 - (a == b ? s3 : 0.0);
            for (int c = 0; c < 3; ++c)
                D3[a][b][c] = -15.0 * R[a] * R[b] * R[c] * s7 +
                              3.0 * ((a == b ? R[c] : 0.0) + (a == c ? R[b] : 0.0) + (b == c ? R[a] : 0.0)) * s5;
        }
    }
    double q0 = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) q0 += Q[a][b] * D2[a][b];
    lam[0] += M * s + q0 / 6.0;
    for (int a = 0; a < 3; ++a) {
        double q1 = 0.0;
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) q1 += Q[b][c] * D3[a][b][c];
        lam[L1(a)] += M * D1[a] + q1 / 6.0;
        for (int b = 0; b < 3; ++b) {
            lam[L2(a, b)] += M * D2[a][b];
            for (int c = 0; c < 3; ++c) lam[L3(a, b, c)] += M * D3[a][b][c];
        }
    }
}

/* L2L: add to out the expansion lam moved by t (new centre = old + t). */
void orc_fmm_l2l(const double *lam, const double *t, double *out)
{
    double s0 = lam[0], s1[3], s2[3][3];
    for (int a = 0; a < 3; ++a) {
        s1[a] = lam[L1(a)];
        for (int b = 0; b < 3; ++b) s2[a][b] = lam[L2(a, b)];
    }
    for (int a = 0; a < 3; ++a) {
        s0 += lam[L1(a)] * t[a];
        for (int b = 0; b < 3; ++b) {
            s0 += 0.5 * lam[L2(a, b)] * t[a] * t[b];
            s1[a] += lam[L2(a, b)] * t[b];
            for (int c = 0; c < 3; ++c) {
                s0 += lam[L3(a, b, c)] * t[a] * t[b] * t[c] / 6.0;
                s1[a] += 0.5 * lam[L3(a, b, c)] * t[b] * t[c];
                s2[a][b] += lam[L3(a, b, c)] * t[c];
            }
        }
    }
    out[0] += s0;
    for (int a = 0; a < 3; ++a) {
        out[L1(a)] += s1[a];
        for (int b = 0; b < 3; ++b) {
            out[L2(a, b)] += s2[a][b];
            for (int c = 0; c < 3; ++c) out[L3(a, b, c)] += lam[L3(a, b, c)];
        }
    }
}

/* L2P: acceleration and potential at offset dl from the expansion centre. */
void orc_fmm_l2p(const double *lam, const double *dl, double G, double *acc, double *pot)
{
    double phi = lam[0];
    for (int a = 0; a < 3; ++a) {
        double g = lam[L1(a)];
        phi += lam[L1(a)] * dl[a];
        for (int b = 0; b < 3; ++b) {
            g += lam[L2(a, b)] * dl[b];
            phi += 0.5 * lam[L2(a, b)] * dl[a] * dl[b];
            for (int c = 0; c < 3; ++c) {
                g += 0.5 * lam[L3(a, b, c)] * dl[b] * dl[c];
                phi += lam[L3(a, b, c)] * dl[a] * dl[b] * dl[c] / 6.0;
            }
        }
        acc[a] = G * g;
    }
    *pot = -G * phi;
}

/* The FMM force on every body (original order): acc [n][3], pot [n].
 * Returns 0, or -1 for a 2D tree. */
int orc_fmm_forces(const orc_tree *t, double theta, double G, double eps, double *acc, double *pot)
{
    if (t->dim != 3) return -1;
    fmm_ctx f;
    fmm_setup(&f, t, theta);
    /* traversal: count, then record */
    fmm_rec(&f, 0, 0);
    f.cap_m = f.nm2l;
    f.cap_p = f.np2p;
    f.m2l = malloc((f.cap_m + 1) * 2 * sizeof(int32_t));
    f.p2p = malloc((f.cap_p + 1) * 2 * sizeof(int32_t));
    f.nm2l = f.np2p = 0;
    fmm_rec(&f, 0, 0);

    const int64_t C = t->ncells;
    double *lam = calloc(C * FMM_NL, sizeof(double));
    for (int64_t k = 0; k < f.nm2l; ++k) {
        const int64_t A = f.m2l[2 * k], B = f.m2l[2 * k + 1];
        double R[3];
        for (int a = 0; a < 3; ++a) R[a] = f.ctr[A * 3 + a] - t->com[B * 3 + a];
        orc_fmm_m2l(t->M[B], t->Q + B * 6, R, eps, lam + A * FMM_NL);
    }
    /* top-down: pre-order visits every parent before its children */
    for (int64_t c = 0; c < C; ++c) {
        if (t->leaf[c]) continue;
        for (int64_t ch = c + 1; ch < t->skip[c]; ch = t->skip[ch]) {
            double tt[3];
            for (int a = 0; a < 3; ++a) tt[a] = f.ctr[ch * 3 + a] - f.ctr[c * 3 + a];
            orc_fmm_l2l(lam + c * FMM_NL, tt, lam + ch * FMM_NL);
        }
    }
    /* P2P partners of each target leaf */
    int64_t *pcnt = calloc(C + 1, sizeof(int64_t));
    for (int64_t k = 0; k < f.np2p; ++k) pcnt[f.p2p[2 * k] + 1] += 1;
    for (int64_t c = 0; c < C; ++c) pcnt[c + 1] += pcnt[c];
    int64_t *fill = malloc(C * sizeof(int64_t));
    memcpy(fill, pcnt, C * sizeof(int64_t));
    int32_t *src = malloc((f.np2p + 1) * sizeof(int32_t));
    for (int64_t k = 0; k < f.np2p; ++k) src[fill[f.p2p[2 * k]]++] = f.p2p[2 * k + 1];
    const double e2 = eps * eps;
#pragma omp parallel for schedule(dynamic)
    for (int64_t c = 0; c < C; ++c) {
        if (!t->leaf[c]) continue;
        for (int64_t i = t->begin[c]; i < t->begin[c] + t->count[c]; ++i) {
            double dl[3], a[3], p;
            for (int k = 0; k < 3; ++k) dl[k] = t->x[i * 3 + k] - f.ctr[c * 3 + k];
            orc_fmm_l2p(lam + c * FMM_NL, dl, G, a, &p);
            double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
            for (int64_t q = pcnt[c]; q < pcnt[c + 1]; ++q) {
                const int64_t B = src[q];
                for (int64_t j = t->begin[B]; j < t->begin[B] + t->count[B]; ++j) {
                    if (j == i) continue;
                    const double dx = t->x[j * 3] - t->x[i * 3], dy = t->x[j * 3 + 1] - t->x[i * 3 + 1],
                                 dz = t->x[j * 3 + 2] - t->x[i * 3 + 2];
                    const double r2 = dx * dx + dy * dy + dz * dz + e2;
                    const double s = 1.0 / sqrt(r2);
                    const double ms = t->m[j] * s, ms3 = ms * s * s;
                    ax += ms3 * dx;
                    ay += ms3 * dy;
                    az += ms3 * dz;
                    ph -= ms;
                }
            }
            const int64_t o = t->perm[i];
            acc[o * 3] = a[0] + G * ax;
            acc[o * 3 + 1] = a[1] + G * ay;
            acc[o * 3 + 2] = a[2] + G * az;
            pot[o] = p + G * ph;
        }
    }
    free(pcnt);
    free(fill);
    free(src);
    free(lam);
    free(f.m2l);
    free(f.p2p);
    fmm_teardown(&f);
    return 0;
}
