/*
 * tree.c -- root cube, Morton keys and the level-restricted adaptive 2^d-tree
 * with colleagues, coarse neighbours and the flags of Step 0.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Definitions (Sec. 3.2, "An O(N log N) DMK method"; Sec. 3.5, Step 0):
 *  - points are rescaled and centred into the unit box [-1/2,1/2]^d;
 *  - a box is refined (into all 2^d children) while it holds more than n_s
 *    points and its level is below the depth cap;
 *  - level restriction: two leaves sharing a boundary point (face, edge or
 *    corner) differ by at most one level.  The tree kept is the smallest
 *    refinement of the count-based tree with that property; it is found here
 *    by refining any leaf that violates it until none does;
 *  - colleagues: same-level boxes sharing a boundary point, the box included;
 *  - coarse neighbours of a leaf at level l: leaves at level l-1 sharing a
 *    boundary point with it;
 *  - F_leaf; F_out = non-leaf with more than n_s points; F_in = some colleague
 *    has F_out.  A point's terminal box is its coarsest ancestor-or-self with
 *    F_out = 0; the far field of its charge stops at that level.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t key; int64_t idx; } kv_t;

static int kv_cmp(const void *a, const void *b)
{
    const kv_t *x = (const kv_t *)a, *y = (const kv_t *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
    return 0;
}

static int u64_cmp(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* Bit b of coordinate d goes to key bit dim*b + (dim-1-d): x is the most
 * significant coordinate within each group. */
static uint64_t interleave(int dim, const uint64_t *c, int nbits)
{
    uint64_t key = 0;
    for (int b = 0; b < nbits; ++b)
        for (int d = 0; d < dim; ++d)
            key |= ((c[d] >> b) & 1ull) << (dim * b + (dim - 1 - d));
    return key;
}

static void deinterleave(int dim, uint64_t key, int nbits, uint64_t *c)
{
    for (int d = 0; d < dim; ++d) c[d] = 0;
    for (int b = 0; b < nbits; ++b)
        for (int d = 0; d < dim; ++d)
            c[d] |= ((key >> (dim * b + (dim - 1 - d))) & 1ull) << b;
}

/* first index in sorted a[0..n) with a[i] >= v */
static int64_t lower_bound_u64(const uint64_t *a, int64_t n, uint64_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static int64_t find_u64(const uint64_t *a, int64_t n, uint64_t v)
{
    int64_t i = lower_bound_u64(a, n, v);
    return (i < n && a[i] == v) ? i : -1;
}

/* points with the given level-l prefix occupy [*lo, *hi) of the sorted keys */
static void prefix_range(const orc_tree *t, uint64_t prefix, int l, int64_t *lo, int64_t *hi)
{
    int shift = t->dim * (t->bits - l);
    if (l == 0) { *lo = 0; *hi = t->n; return; }
    uint64_t a = prefix << shift;
    uint64_t b = (prefix + 1) << shift;
    *lo = lower_bound_u64(t->key, t->n, a);
    /* (prefix+1) << shift can wrap to 0 only for the last box of a level
       when dim*bits == 64, which does not occur (63 or 62 bits) */
    *hi = lower_bound_u64(t->key, t->n, b);
}

typedef struct { uint64_t *v; int64_t n, cap; } vec_t;

static void vec_push(vec_t *a, uint64_t x)
{
    if (a->n == a->cap) {
        a->cap = a->cap ? 2 * a->cap : 64;
        a->v = (uint64_t *)realloc(a->v, (size_t)a->cap * sizeof(uint64_t));
    }
    a->v[a->n++] = x;
}

static void vec_sort_unique(vec_t *a)
{
    if (a->n == 0) return;
    qsort(a->v, (size_t)a->n, sizeof(uint64_t), u64_cmp);
    int64_t m = 1;
    for (int64_t i = 1; i < a->n; ++i)
        if (a->v[i] != a->v[m - 1]) a->v[m++] = a->v[i];
    a->n = m;
}

#define MAXLEV 64

/* existing boxes of level l: the root, or all children of refined level-(l-1) boxes */
static void existing_at(int dim, vec_t *ref, int l, vec_t *out)
{
    out->n = 0;
    if (l == 0) { vec_push(out, 0); return; }
    int nc = 1 << dim;
    for (int64_t i = 0; i < ref[l - 1].n; ++i)
        for (int c = 0; c < nc; ++c) vec_push(out, (ref[l - 1].v[i] << dim) | (uint64_t)c);
}

int orc_tree_build(int dim, int64_t n, const double *pts, int ns, int maxdepth, orc_tree *t)
{
    memset(t, 0, sizeof(*t));
    if (dim != 2 && dim != 3) return -1;
    t->dim = dim;
    t->bits = (dim == 3) ? 21 : 31;
    t->ns = ns;
    if (maxdepth <= 0) maxdepth = (dim == 3) ? 20 : 30;
    if (maxdepth > t->bits) maxdepth = t->bits;
    t->maxdepth = maxdepth;
    t->n = n;

    /* root cube: centre of the bounding box, side = largest extent (slightly
       enlarged so that no point lands exactly on the upper face) */
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int d = 0; d < dim; ++d) {
        lo[d] = n ? pts[d] : 0.0;
        hi[d] = lo[d];
    }
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < dim; ++d) {
            double v = pts[i * dim + d];
            if (v < lo[d]) lo[d] = v;
            if (v > hi[d]) hi[d] = v;
        }
    double ext = 0.0;
    for (int d = 0; d < dim; ++d) {
        t->center[d] = 0.5 * (lo[d] + hi[d]);
        if (hi[d] - lo[d] > ext) ext = hi[d] - lo[d];
    }
    t->side = (ext > 0.0) ? ext * (1.0 + ldexp(1.0, -40)) : 1.0;

    /* Morton keys, stable sort by (key, input index) */
    const double scale = ldexp(1.0, t->bits);
    const uint64_t kmax = (1ull << t->bits) - 1ull;
    kv_t *kv = (kv_t *)malloc((size_t)(n ? n : 1) * sizeof(kv_t));
    double *xn = (double *)malloc((size_t)(n ? n : 1) * dim * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        uint64_t c[3];
        for (int d = 0; d < dim; ++d) {
            double x = (pts[i * dim + d] - t->center[d]) / t->side;
            xn[i * dim + d] = x;
            double f = floor((x + 0.5) * scale);
            uint64_t k = (f <= 0.0) ? 0ull : (uint64_t)f;
            if (k > kmax) k = kmax;
            c[d] = k;
        }
        kv[i].key = interleave(dim, c, t->bits);
        kv[i].idx = i;
    }
    qsort(kv, (size_t)n, sizeof(kv_t), kv_cmp);
    t->perm = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
    t->key = (uint64_t *)malloc((size_t)(n ? n : 1) * sizeof(uint64_t));
    t->xs = (double *)malloc((size_t)(n ? n : 1) * dim * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        t->perm[i] = kv[i].idx;
        t->key[i] = kv[i].key;
        for (int d = 0; d < dim; ++d) t->xs[i * dim + d] = xn[kv[i].idx * dim + d];
    }
    free(kv);
    free(xn);

    /* refined[l]: sorted prefixes of refined boxes at level l */
    vec_t ref[MAXLEV];
    memset(ref, 0, sizeof(ref));
    vec_t ex = {0, 0, 0};

    /* count-based refinement */
    for (int l = 0; l < maxdepth; ++l) {
        existing_at(dim, ref, l, &ex);
        for (int64_t i = 0; i < ex.n; ++i) {
            int64_t a, b;
            prefix_range(t, ex.v[i], l, &a, &b);
            if (b - a > ns) vec_push(&ref[l], ex.v[i]);
        }
        if (ref[l].n == 0) break;
    }

    /* level restriction: refine a leaf A at level a whenever a refined box at
       level a+1 shares a boundary point with A; repeat until none is left */
    const int nc = 1 << dim;
    for (;;) {
        int changed = 0;
        for (int a = 0; a + 1 < maxdepth; ++a) {
            if (ref[a + 1].n == 0) continue;
            existing_at(dim, ref, a, &ex);
            vec_t add = {0, 0, 0};
            for (int64_t i = 0; i < ex.n; ++i) {
                uint64_t P = ex.v[i];
                if (find_u64(ref[a].v, ref[a].n, P) >= 0) continue; /* not a leaf */
                uint64_t c[3];
                deinterleave(dim, P, a, c);
                int64_t lim = (int64_t)1 << (a + 1);
                int viol = 0;
                /* ring of level-(a+1) regions around A: offsets -1..2 per axis */
                int nring = 1;
                for (int d = 0; d < dim; ++d) nring *= 4;
                for (int r = 0; r < nring && !viol; ++r) {
                    int rr = r, inside = 1;
                    uint64_t q[3];
                    for (int d = dim - 1; d >= 0; --d) {
                        int o = rr % 4 - 1;
                        rr /= 4;
                        int64_t v = 2 * (int64_t)c[d] + o;
                        if (o == 0 || o == 1) { /* within A along this axis */ }
                        else inside = 0;
                        if (v < 0 || v >= lim) { inside = 2; break; }
                        q[d] = (uint64_t)v;
                    }
                    if (inside != 0) continue; /* own child or outside domain */
                    uint64_t Q = interleave(dim, q, a + 1);
                    if (find_u64(ref[a + 1].v, ref[a + 1].n, Q) >= 0) viol = 1;
                }
                if (viol) vec_push(&add, P);
            }
            for (int64_t i = 0; i < add.n; ++i) vec_push(&ref[a], add.v[i]);
            if (add.n) { vec_sort_unique(&ref[a]); changed = 1; }
            free(add.v);
        }
        if (!changed) break;
    }

    /* materialise boxes, level-major, Morton order within a level */
    int nl = 0;
    int64_t nbox = 0;
    int64_t lstart[MAXLEV + 1];
    vec_t lev[MAXLEV];
    memset(lev, 0, sizeof(lev));
    for (int l = 0; l < MAXLEV; ++l) {
        if (l > 0 && ref[l - 1].n == 0) break;
        existing_at(dim, ref, l, &lev[l]);
        lstart[l] = nbox;
        nbox += lev[l].n;
        nl = l + 1;
    }
    lstart[nl] = nbox;
    t->nlevels = nl;
    t->nbox = nbox;
    t->level_start = (int64_t *)malloc((size_t)(nl + 1) * sizeof(int64_t));
    memcpy(t->level_start, lstart, (size_t)(nl + 1) * sizeof(int64_t));
    t->level = (int32_t *)malloc((size_t)nbox * sizeof(int32_t));
    t->bkey = (uint64_t *)malloc((size_t)nbox * sizeof(uint64_t));
    t->parent = (int64_t *)malloc((size_t)nbox * sizeof(int64_t));
    t->child0 = (int64_t *)malloc((size_t)nbox * sizeof(int64_t));
    t->pstart = (int64_t *)malloc((size_t)nbox * sizeof(int64_t));
    t->pcount = (int64_t *)malloc((size_t)nbox * sizeof(int64_t));
    t->leaf = (uint8_t *)malloc((size_t)nbox);
    t->fout = (uint8_t *)malloc((size_t)nbox);
    t->fin = (uint8_t *)malloc((size_t)nbox);
    t->terminal = (uint8_t *)malloc((size_t)nbox);
    int ncol = (dim == 3) ? 27 : 9;
    int ncmax = nc - 1;
    t->colleague = (int64_t *)malloc((size_t)nbox * ncol * sizeof(int64_t));
    t->ncoarse = (int32_t *)malloc((size_t)nbox * sizeof(int32_t));
    t->coarse = (int64_t *)malloc((size_t)nbox * ncmax * sizeof(int64_t));

    for (int l = 0; l < nl; ++l) {
        for (int64_t i = 0; i < lev[l].n; ++i) {
            int64_t b = lstart[l] + i;
            uint64_t P = lev[l].v[i];
            t->level[b] = l;
            t->bkey[b] = P;
            int64_t a, e;
            prefix_range(t, P, l, &a, &e);
            t->pstart[b] = a;
            t->pcount[b] = e - a;
            int64_t ri = find_u64(ref[l].v, ref[l].n, P);
            t->leaf[b] = (ri < 0);
            t->child0[b] = (ri < 0) ? -1 : lstart[l + 1] + ri * nc;
            if (l == 0) t->parent[b] = -1;
            else t->parent[b] = lstart[l - 1] + find_u64(lev[l - 1].v, lev[l - 1].n, P >> dim);
            t->fout[b] = (!t->leaf[b]) && (t->pcount[b] > ns);
        }
    }
    /* colleagues and coarse neighbours */
    for (int l = 0; l < nl; ++l) {
        int64_t lim = (int64_t)1 << l;
        for (int64_t i = 0; i < lev[l].n; ++i) {
            int64_t b = lstart[l] + i;
            uint64_t c[3];
            deinterleave(dim, lev[l].v[i], l, c);
            for (int k = 0; k < ncol; ++k) {
                int kk = k, ok = 1;
                uint64_t q[3];
                for (int d = dim - 1; d >= 0; --d) {
                    int o = kk % 3 - 1;
                    kk /= 3;
                    int64_t v = (int64_t)c[d] + o;
                    if (v < 0 || v >= lim) ok = 0;
                    q[d] = (uint64_t)v;
                }
                int64_t j = -1;
                if (ok) {
                    int64_t f = find_u64(lev[l].v, lev[l].n, interleave(dim, q, l));
                    if (f >= 0) j = lstart[l] + f;
                }
                t->colleague[b * ncol + k] = j;
            }
            t->ncoarse[b] = 0;
            if (l > 0 && t->leaf[b]) {
                for (int k = 0; k < ncol; ++k) {
                    int kk = k, ok = 1;
                    uint64_t q[3];
                    for (int d = dim - 1; d >= 0; --d) {
                        int o = kk % 3 - 1;
                        kk /= 3;
                        int64_t v = (int64_t)c[d] + o;
                        if (v < 0 || v >= lim) ok = 0;
                        q[d] = (uint64_t)v >> 1;
                    }
                    if (!ok) continue;
                    uint64_t Q = interleave(dim, q, l - 1);
                    if (Q == (lev[l].v[i] >> dim)) continue; /* own parent */
                    int64_t f = find_u64(lev[l - 1].v, lev[l - 1].n, Q);
                    if (f < 0) continue;
                    int64_t j = lstart[l - 1] + f;
                    if (!t->leaf[j]) continue;
                    int dup = 0;
                    for (int m = 0; m < t->ncoarse[b]; ++m)
                        if (t->coarse[b * ncmax + m] == j) dup = 1;
                    if (!dup) t->coarse[b * ncmax + t->ncoarse[b]++] = j;
                }
            }
        }
    }
    for (int64_t b = 0; b < nbox; ++b) {
        int fin = 0;
        for (int k = 0; k < ncol; ++k) {
            int64_t j = t->colleague[b * ncol + k];
            if (j >= 0 && t->fout[j]) fin = 1;
        }
        t->fin[b] = fin;
        t->terminal[b] = (!t->fout[b]) && (t->parent[b] < 0 || t->fout[t->parent[b]]);
    }
    t->tlevel = (int32_t *)malloc((size_t)(n ? n : 1) * sizeof(int32_t));
    for (int64_t b = 0; b < nbox; ++b)
        if (t->terminal[b])
            for (int64_t i = t->pstart[b]; i < t->pstart[b] + t->pcount[b]; ++i)
                t->tlevel[i] = t->level[b];

    for (int l = 0; l < MAXLEV; ++l) { free(ref[l].v); free(lev[l].v); }
    free(ex.v);
    return 0;
}

void orc_tree_free(orc_tree *t)
{
    free(t->perm); free(t->key); free(t->xs); free(t->level_start);
    free(t->level); free(t->bkey); free(t->parent); free(t->child0);
    free(t->pstart); free(t->pcount); free(t->leaf); free(t->fout);
    free(t->fin); free(t->terminal); free(t->colleague); free(t->ncoarse);
    free(t->coarse); free(t->tlevel);
    memset(t, 0, sizeof(*t));
}
