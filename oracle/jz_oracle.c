/*
 * CPU oracle for exact k-nearest-neighbour search and friends-of-friends (FoF).
 *
 * TEST INFRASTRUCTURE ONLY. This file builds a separate shared library that
 * only the tests, the smoke check and the benchmark's CPU-baseline leg load.
 * It shares no code, header, table or helper with the GPU library, and the GPU
 * library never loads it.
 *
 * What is computed (the paper's problem statements):
 *   - kNN (nearest-neighbour section; self-queries as in the benchmarks of the
 *     kNN-across-domains section): for every point i, the k points j (j = i
 *     included) that are closest to i.
 *   - FoF (friends-of-friends section, Eq. 18): connected components of the
 *     graph that links every pair of points no farther apart than the linking
 *     length b.
 *
 * Fixed arithmetic (the paper fixes only "float32"; this is the reading both
 * sides use): for points p, q in float32,
 *     dx = fl(p.x - q.x), dy = ..., dz = ...
 *     dist2 = fl( fl( fl(dx*dx) + fl(dy*dy) ) + fl(dz*dz) )
 * with IEEE-754 binary32 round-to-nearest-even, no fused multiply-add (the
 * build passes -ffp-contract=off) and subnormals kept.
 * kNN order: ascending (dist2, j) pairs (index breaks distance ties).
 * FoF edge: dist2 <= fl(b*b) (inclusive). Label: the smallest member index.
 *
 * Brute-force entry points (*_bf) are the definitions written out. The kd-tree
 * entry points (*_kd) give the same answers faster for large inputs; they only
 * skip work that a rigorous bound proves irrelevant, and the tests check them
 * against *_bf bit for bit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define JZO_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------------- */
/* distance                                                                   */

static inline float d2f(const float *p, const float *q) {
    float dx = p[0] - q[0];
    float dy = p[1] - q[1];
    float dz = p[2] - q[2];
    float xx = dx * dx;
    float yy = dy * dy;
    float zz = dz * dz;
    float s = xx + yy;
    return s + zz;
}

/* Rigorous bounds between a point q and an axis-aligned box [lo, hi] that
 * contains points p. Every step is a correctly rounded, monotone operation on
 * non-negative values, so for each p in the box the computed d2f(q, p) lies in
 * [box_low(q), box_up(q)] exactly (no safety margin needed). */
static inline float box_low(const float *q, const float *lo, const float *hi) {
    float g[3];
    for (int a = 0; a < 3; ++a) {
        float l = lo[a] - q[a];
        float h = q[a] - hi[a];
        float m = l > h ? l : h;
        g[a] = m > 0.0f ? m : 0.0f;
    }
    float xx = g[0] * g[0], yy = g[1] * g[1], zz = g[2] * g[2];
    float s = xx + yy;
    return s + zz;
}

static inline float box_up(const float *q, const float *lo, const float *hi) {
    float g[3];
    for (int a = 0; a < 3; ++a) {
        float l = q[a] - lo[a];
        float h = hi[a] - q[a];
        g[a] = l > h ? l : h;
    }
    float xx = g[0] * g[0], yy = g[1] * g[1], zz = g[2] * g[2];
    float s = xx + yy;
    return s + zz;
}

static int clamp_threads(int nthreads) {
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    return nthreads < 1 ? 1 : nthreads;
}

/* ------------------------------------------------------------------------- */
/* kNN, brute force                                                           */

/* For each requested row i (rows == NULL: all rows 0..n-1), scan j = 0..n-1 in
 * increasing order and keep the k smallest distances. A new candidate replaces
 * the current k-th only if strictly closer, and equal distances are inserted
 * after the ones already held; because j only increases this realizes the
 * (dist2, j) order without ever comparing indices. Rows shorter than k (k > n)
 * are padded with idx = -1, dist2 = +inf. */
JZO_API int jzo_knn_bf(const float *pts, int64_t n, int k, const int64_t *rows,
                       int64_t nrows, int32_t *idx, float *d2, int nthreads) {
    if (k < 1 || n < 0) return -1;
    int64_t R = rows ? nrows : n;
    int fail = 0;
#pragma omp parallel num_threads(clamp_threads(nthreads))
    {
        float *bd = (float *)malloc(sizeof(float) * (size_t)k);
        int32_t *bj = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
        if (!bd || !bj) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 8)
        for (int64_t r = 0; r < R; ++r) {
            if (!bd || !bj) continue;
            int64_t i = rows ? rows[r] : r;
            const float *p = pts + 3 * i;
            int cnt = 0;
            for (int64_t j = 0; j < n; ++j) {
                float d = d2f(p, pts + 3 * j);
                if (cnt == k && !(d < bd[k - 1])) continue;
                int pos = cnt < k ? cnt : k - 1;
                while (pos > 0 && bd[pos - 1] > d) {
                    bd[pos] = bd[pos - 1];
                    bj[pos] = bj[pos - 1];
                    --pos;
                }
                bd[pos] = d;
                bj[pos] = (int32_t)j;
                if (cnt < k) ++cnt;
            }
            for (int t = 0; t < k; ++t) {
                idx[r * k + t] = t < cnt ? bj[t] : -1;
                d2[r * k + t] = t < cnt ? bd[t] : INFINITY;
            }
        }
        free(bd);
        free(bj);
    }
    return fail ? -2 : 0;
}

/* kNN of separate query points among source points (the paper's "multiple
 * point types"), brute force: for each query q, the k source points j closest
 * to q, ascending by (dist2, j), scanning j in increasing order with the same
 * strict-< insertion as jzo_knn_bf. A query equal to a source point finds it
 * at distance 0; fewer than k sources pad with idx = -1, dist2 = +inf. */
JZO_API int jzo_knn_cross_bf(const float *src, int64_t ns, const float *qry, int64_t nq, int k,
                             int32_t *idx, float *d2, int nthreads) {
    if (k < 1 || ns < 0 || nq < 0) return -1;
    int fail = 0;
#pragma omp parallel num_threads(clamp_threads(nthreads))
    {
        float *bd = (float *)malloc(sizeof(float) * (size_t)k);
        int32_t *bj = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
        if (!bd || !bj) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 8)
        for (int64_t r = 0; r < nq; ++r) {
            if (!bd || !bj) continue;
            const float *p = qry + 3 * r;
            int cnt = 0;
            for (int64_t j = 0; j < ns; ++j) {
                float d = d2f(p, src + 3 * j);
                if (cnt == k && !(d < bd[k - 1])) continue;
                int pos = cnt < k ? cnt : k - 1;
                while (pos > 0 && bd[pos - 1] > d) {
                    bd[pos] = bd[pos - 1];
                    bj[pos] = bj[pos - 1];
                    --pos;
                }
                bd[pos] = d;
                bj[pos] = (int32_t)j;
                if (cnt < k) ++cnt;
            }
            for (int t = 0; t < k; ++t) {
                idx[r * k + t] = t < cnt ? bj[t] : -1;
                d2[r * k + t] = t < cnt ? bd[t] : INFINITY;
            }
        }
        free(bd);
        free(bj);
    }
    return fail ? -2 : 0;
}

/* ------------------------------------------------------------------------- */
/* periodic box (the paper's periodic cosmological case)                      */

/* Minimum-image distance in the periodic cube [0, L)^3 (points inside it):
 * dx = fl(x_i - x_j) is moved by one period when it lies beyond half of it,
 *     dx > h: dx = fl(dx - L);  dx < -h: dx = fl(dx + L);  h = fl(L / 2),
 * and dist2 is the fixed expression of the wrapped differences. Since
 * fl(a - b) = -fl(b - a) and the wrap is symmetric, dist2 stays symmetric. */
static inline float wrapf(float d, float L, float h) {
    if (d > h) return d - L;
    if (d < -h) return d + L;
    return d;
}

static inline float d2f_per(const float *p, const float *q, float L, float h) {
    float dx = wrapf(p[0] - q[0], L, h);
    float dy = wrapf(p[1] - q[1], L, h);
    float dz = wrapf(p[2] - q[2], L, h);
    float xx = dx * dx;
    float yy = dy * dy;
    float zz = dz * dz;
    float s = xx + yy;
    return s + zz;
}

/* jzo_knn_bf with the periodic distance (same selection rule). */
JZO_API int jzo_knn_bf_per(const float *pts, int64_t n, float L, int k, const int64_t *rows,
                           int64_t nrows, int32_t *idx, float *d2, int nthreads) {
    if (k < 1 || n < 0 || !(L > 0.0f)) return -1;
    const float h = 0.5f * L;
    int64_t R = rows ? nrows : n;
    int fail = 0;
#pragma omp parallel num_threads(clamp_threads(nthreads))
    {
        float *bd = (float *)malloc(sizeof(float) * (size_t)k);
        int32_t *bj = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
        if (!bd || !bj) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 8)
        for (int64_t r = 0; r < R; ++r) {
            if (!bd || !bj) continue;
            int64_t i = rows ? rows[r] : r;
            const float *p = pts + 3 * i;
            int cnt = 0;
            for (int64_t j = 0; j < n; ++j) {
                float d = d2f_per(p, pts + 3 * j, L, h);
                if (cnt == k && !(d < bd[k - 1])) continue;
                int pos = cnt < k ? cnt : k - 1;
                while (pos > 0 && bd[pos - 1] > d) {
                    bd[pos] = bd[pos - 1];
                    bj[pos] = bj[pos - 1];
                    --pos;
                }
                bd[pos] = d;
                bj[pos] = (int32_t)j;
                if (cnt < k) ++cnt;
            }
            for (int t = 0; t < k; ++t) {
                idx[r * k + t] = t < cnt ? bj[t] : -1;
                d2[r * k + t] = t < cnt ? bd[t] : INFINITY;
            }
        }
        free(bd);
        free(bj);
    }
    return fail ? -2 : 0;
}

/* ------------------------------------------------------------------------- */
/* union-find (sequential; roots are always the smallest index of a component) */

static int32_t uf_find(int32_t *par, int32_t x) {
    while (par[x] != x) {
        par[x] = par[par[x]];
        x = par[x];
    }
    return x;
}

static void uf_unite(int32_t *par, int32_t a, int32_t b) {
    a = uf_find(par, a);
    b = uf_find(par, b);
    if (a == b) return;
    if (a < b) par[b] = a; else par[a] = b;
}

/* Components of an explicit edge list by union-find; label = min index. */
JZO_API int jzo_components_uf(int64_t n, const int32_t *edges, int64_t m, int32_t *label) {
    for (int64_t i = 0; i < n; ++i) label[i] = (int32_t)i;
    for (int64_t e = 0; e < m; ++e) uf_unite(label, edges[2 * e], edges[2 * e + 1]);
    for (int64_t i = 0; i < n; ++i) label[i] = uf_find(label, (int32_t)i);
    return 0;
}

/* Components of an explicit edge list by breadth-first search over an
 * adjacency (CSR) built here; each component is labelled by the first vertex
 * reached when scanning vertices in increasing order, i.e. its min index. */
JZO_API int jzo_components_bfs(int64_t n, const int32_t *edges, int64_t m, int32_t *label) {
    int64_t *deg = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *adj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    if (!deg || !adj || !queue) { free(deg); free(adj); free(queue); return -2; }
    for (int64_t e = 0; e < m; ++e) { deg[edges[2 * e] + 1]++; deg[edges[2 * e + 1] + 1]++; }
    for (int64_t i = 0; i < n; ++i) deg[i + 1] += deg[i];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!fill) { free(deg); free(adj); free(queue); return -2; }
    memcpy(fill, deg, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t e = 0; e < m; ++e) {
        int32_t a = edges[2 * e], b = edges[2 * e + 1];
        adj[fill[a]++] = b;
        adj[fill[b]++] = a;
    }
    for (int64_t i = 0; i < n; ++i) label[i] = -1;
    for (int64_t s = 0; s < n; ++s) {
        if (label[s] >= 0) continue;
        int64_t head = 0, tail = 0;
        queue[tail++] = (int32_t)s;
        label[s] = (int32_t)s;
        while (head < tail) {
            int32_t v = queue[head++];
            for (int64_t t = deg[v]; t < deg[v + 1]; ++t) {
                int32_t w = adj[t];
                if (label[w] < 0) { label[w] = (int32_t)s; queue[tail++] = w; }
            }
        }
    }
    free(deg); free(adj); free(queue); free(fill);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* FoF, brute force                                                           */

/* All pairs i < j with d2f <= fl(b*b) are united. Rows are split over threads;
 * each thread unites its edges in a private union-find, and the private forests
 * are merged at the end (uniting i with its private root keeps exactly the same
 * connectivity). Label = min index of the component. */
JZO_API int jzo_fof_bf(const float *pts, int64_t n, float b, int32_t *label, int nthreads) {
    if (!(b >= 0.0f)) return -1;
    float b2 = b * b;
    int T = clamp_threads(nthreads);
    int32_t *loc = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * (size_t)T);
    if (!loc && n > 0) return -2;
#pragma omp parallel num_threads(T)
    {
        int t = omp_get_thread_num();
        int32_t *par = loc + (size_t)t * (size_t)n;
        for (int64_t i = 0; i < n; ++i) par[i] = (int32_t)i;
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i) {
            const float *p = pts + 3 * i;
            for (int64_t j = i + 1; j < n; ++j)
                if (d2f(p, pts + 3 * j) <= b2) uf_unite(par, (int32_t)i, (int32_t)j);
        }
    }
    for (int64_t i = 0; i < n; ++i) label[i] = (int32_t)i;
    for (int t = 0; t < T; ++t) {
        int32_t *par = loc + (size_t)t * (size_t)n;
        for (int64_t i = 0; i < n; ++i) uf_unite(label, (int32_t)i, uf_find(par, (int32_t)i));
    }
    for (int64_t i = 0; i < n; ++i) label[i] = uf_find(label, (int32_t)i);
    free(loc);
    return 0;
}

/* jzo_fof_bf with the periodic distance. */
JZO_API int jzo_fof_bf_per(const float *pts, int64_t n, float L, float b, int32_t *label,
                           int nthreads) {
    if (!(b >= 0.0f) || !(L > 0.0f)) return -1;
    const float b2 = b * b, h = 0.5f * L;
    int T = clamp_threads(nthreads);
    int32_t *loc = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * (size_t)T);
    if (!loc && n > 0) return -2;
#pragma omp parallel num_threads(T)
    {
        int t = omp_get_thread_num();
        int32_t *par = loc + (size_t)t * (size_t)n;
        for (int64_t i = 0; i < n; ++i) par[i] = (int32_t)i;
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i) {
            const float *p = pts + 3 * i;
            for (int64_t j = i + 1; j < n; ++j)
                if (d2f_per(p, pts + 3 * j, L, h) <= b2) uf_unite(par, (int32_t)i, (int32_t)j);
        }
    }
    for (int64_t i = 0; i < n; ++i) label[i] = (int32_t)i;
    for (int t = 0; t < T; ++t) {
        int32_t *par = loc + (size_t)t * (size_t)n;
        for (int64_t i = 0; i < n; ++i) uf_unite(label, (int32_t)i, uf_find(par, (int32_t)i));
    }
    for (int64_t i = 0; i < n; ++i) label[i] = uf_find(label, (int32_t)i);
    free(loc);
    return 0;
}

/* Neighbours within b of sampled rows (dist2 <= fl(b*b)), brute force.
 * cnt[r] receives the number of neighbours of rows[r] (self included); their
 * indices, ascending, go to nbr starting at offset r*cap (at most cap kept). */
JZO_API int jzo_range_rows_bf(const float *pts, int64_t n, float b, const int64_t *rows,
                              int64_t nrows, int64_t cap, int64_t *cnt, int32_t *nbr,
                              int nthreads) {
    if (!(b >= 0.0f)) return -1;
    float b2 = b * b;
#pragma omp parallel for schedule(dynamic, 1) num_threads(clamp_threads(nthreads))
    for (int64_t r = 0; r < nrows; ++r) {
        const float *p = pts + 3 * rows[r];
        int64_t c = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (d2f(p, pts + 3 * j) <= b2) {
                if (c < cap) nbr[r * cap + c] = (int32_t)j;
                ++c;
            }
        }
        cnt[r] = c;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* kd-tree (median splits, tight boxes) used by the *_kd entry points         */

typedef struct {
    float lo[3], hi[3];
    int64_t a, b;   /* range in the permutation */
    int64_t left;   /* index of the left child (right = left + 1); -1 for a leaf */
} kdnode;

typedef struct {
    const float *p;
    int32_t *perm;
    kdnode *node;
    int64_t nnode;
} kdtree;

#define KD_LEAF 16

static inline int kd_less(const float *P, int axis, int32_t i, int32_t j) {
    float a = P[3 * (int64_t)i + axis], b = P[3 * (int64_t)j + axis];
    return a < b || (a == b && i < j);
}

/* Rearranges v[lo..hi) so that v[k] holds the element of rank k - lo under
 * kd_less, with smaller elements before it and larger after (quickselect). */
static void kd_select(int32_t *v, int64_t lo, int64_t hi, int64_t k, const float *P, int axis) {
    while (hi - lo > 1) {
        int64_t mid = lo + (hi - lo) / 2;
        /* median of three into v[mid] */
        if (kd_less(P, axis, v[mid], v[lo])) { int32_t t = v[mid]; v[mid] = v[lo]; v[lo] = t; }
        if (kd_less(P, axis, v[hi - 1], v[lo])) { int32_t t = v[hi - 1]; v[hi - 1] = v[lo]; v[lo] = t; }
        if (kd_less(P, axis, v[hi - 1], v[mid])) { int32_t t = v[hi - 1]; v[hi - 1] = v[mid]; v[mid] = t; }
        int32_t pivot = v[mid];
        v[mid] = v[hi - 1];
        v[hi - 1] = pivot;
        int64_t store = lo;
        for (int64_t t = lo; t < hi - 1; ++t) {
            if (kd_less(P, axis, v[t], pivot)) {
                int32_t x = v[t]; v[t] = v[store]; v[store] = x;
                ++store;
            }
        }
        v[hi - 1] = v[store];
        v[store] = pivot;
        if (store == k) return;
        if (k < store) hi = store; else lo = store + 1;
    }
}

static void kd_box(kdtree *T, kdnode *nd) {
    for (int a = 0; a < 3; ++a) { nd->lo[a] = INFINITY; nd->hi[a] = -INFINITY; }
    for (int64_t t = nd->a; t < nd->b; ++t) {
        const float *q = T->p + 3 * (int64_t)T->perm[t];
        for (int a = 0; a < 3; ++a) {
            if (q[a] < nd->lo[a]) nd->lo[a] = q[a];
            if (q[a] > nd->hi[a]) nd->hi[a] = q[a];
        }
    }
}

static void kd_split(kdtree *T, int64_t id) {
    kdnode *nd = &T->node[id];
    kd_box(T, nd);
    nd->left = -1;
    if (nd->b - nd->a <= KD_LEAF) return;
    int axis = 0;
    float ext = nd->hi[0] - nd->lo[0];
    for (int a = 1; a < 3; ++a) {
        float e = nd->hi[a] - nd->lo[a];
        if (e > ext) { ext = e; axis = a; }
    }
    if (!(ext > 0.0f)) return; /* all points identical: keep as one leaf */
    int64_t mid = nd->a + (nd->b - nd->a) / 2;
    kd_select(T->perm, nd->a, nd->b, mid, T->p, axis);
    int64_t l;
#pragma omp atomic capture
    { l = T->nnode; T->nnode += 2; }
    T->node[l].a = nd->a; T->node[l].b = mid;
    T->node[l + 1].a = mid; T->node[l + 1].b = nd->b;
    nd->left = l;
    int64_t size = nd->b - nd->a;
    if (size > 65536) {
#pragma omp task
        kd_split(T, l);
#pragma omp task
        kd_split(T, l + 1);
#pragma omp taskwait
    } else {
        kd_split(T, l);
        kd_split(T, l + 1);
    }
}

static int kd_build(kdtree *T, const float *pts, int64_t n, int nthreads) {
    T->p = pts;
    T->perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t cap = 2 * (n / (KD_LEAF / 2) + 2);
    T->node = (kdnode *)malloc(sizeof(kdnode) * (size_t)cap);
    if (!T->perm || !T->node) { free(T->perm); free(T->node); return -2; }
    for (int64_t i = 0; i < n; ++i) T->perm[i] = (int32_t)i;
    T->nnode = 1;
    T->node[0].a = 0;
    T->node[0].b = n;
#pragma omp parallel num_threads(clamp_threads(nthreads))
#pragma omp single
    kd_split(T, 0);
    return 0;
}

static void kd_free(kdtree *T) { free(T->perm); free(T->node); }

static inline int pair_less(float da, int32_t ja, float db, int32_t jb) {
    return da < db || (da == db && ja < jb);
}

/* Exact kNN with a kd-tree: a subtree is skipped only if its box lower bound
 * is strictly greater than the current k-th distance, so every candidate that
 * could enter the (dist2, j) top-k is evaluated. Answers rows[0..nrows) or,
 * with rows == NULL, the consecutive rows first .. first + nrows - 1. */
static void kd_knn_rows(const kdtree *T, int64_t n, int k, const int64_t *rows, int64_t first,
                        int64_t nrows, int32_t *idx, float *d2, int nthreads,
                        const float *qpts) {
    const float *pts = T->p;
#pragma omp parallel num_threads(clamp_threads(nthreads))
    {
        float *bd = (float *)malloc(sizeof(float) * (size_t)k);
        int32_t *bj = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
        int64_t stack[256];
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < nrows; ++r) {
            int64_t i = rows ? rows[r] : first + r;
            const float *q = qpts ? qpts + 3 * i : pts + 3 * i;
            int cnt = 0;
            int sp = 0;
            if (n > 0) stack[sp++] = 0;
            while (sp > 0) {
                const kdnode *nd = &T->node[stack[--sp]];
                if (cnt == k && box_low(q, nd->lo, nd->hi) > bd[k - 1]) continue;
                if (nd->left < 0) {
                    for (int64_t t = nd->a; t < nd->b; ++t) {
                        int32_t j = T->perm[t];
                        float d = d2f(q, pts + 3 * (int64_t)j);
                        if (cnt == k && !pair_less(d, j, bd[k - 1], bj[k - 1])) continue;
                        int pos = cnt < k ? cnt : k - 1;
                        while (pos > 0 && pair_less(d, j, bd[pos - 1], bj[pos - 1])) {
                            bd[pos] = bd[pos - 1];
                            bj[pos] = bj[pos - 1];
                            --pos;
                        }
                        bd[pos] = d;
                        bj[pos] = j;
                        if (cnt < k) ++cnt;
                    }
                } else {
                    const kdnode *L = &T->node[nd->left], *Rn = &T->node[nd->left + 1];
                    float dl = box_low(q, L->lo, L->hi), dr = box_low(q, Rn->lo, Rn->hi);
                    /* push the farther child first so the nearer one is visited first */
                    if (dl <= dr) { stack[sp++] = nd->left + 1; stack[sp++] = nd->left; }
                    else { stack[sp++] = nd->left; stack[sp++] = nd->left + 1; }
                }
            }
            for (int t = 0; t < k; ++t) {
                idx[r * k + t] = t < cnt ? bj[t] : -1;
                d2[r * k + t] = t < cnt ? bd[t] : INFINITY;
            }
        }
        free(bd);
        free(bj);
    }
}

JZO_API int jzo_knn_kd(const float *pts, int64_t n, int k, const int64_t *rows, int64_t nrows,
                       int32_t *idx, float *d2, int nthreads) {
    if (k < 1 || n < 0) return -1;
    kdtree T;
    if (kd_build(&T, pts, n, nthreads)) return -2;
    kd_knn_rows(&T, n, k, rows, 0, rows ? nrows : n, idx, d2, nthreads, NULL);
    kd_free(&T);
    return 0;
}

/* jzo_knn_cross_bf with a kd-tree over the sources (same output). */
JZO_API int jzo_knn_cross_kd(const float *src, int64_t ns, const float *qry, int64_t nq, int k,
                             int32_t *idx, float *d2, int nthreads) {
    if (k < 1 || ns < 0 || nq < 0) return -1;
    kdtree T;
    if (kd_build(&T, src, ns, nthreads)) return -2;
    kd_knn_rows(&T, ns, k, NULL, 0, nq, idx, d2, nthreads, qry);
    kd_free(&T);
    return 0;
}

/* A kd-tree kept between calls, so that a large input can be answered in row
 * ranges (the caller then never holds the whole n x k result). The points must
 * stay valid and unchanged until jzo_kd_free. */
typedef struct {
    kdtree T;
    int64_t n;
} kdhandle;

JZO_API void *jzo_kd_new(const float *pts, int64_t n, int nthreads) {
    if (n < 0) return NULL;
    kdhandle *h = (kdhandle *)malloc(sizeof(kdhandle));
    if (!h) return NULL;
    if (kd_build(&h->T, pts, n, nthreads)) { free(h); return NULL; }
    h->n = n;
    return h;
}

/* kNN rows of a kept tree: rows[0..nrows), or first .. first + nrows - 1 when
 * rows is NULL. Same output as jzo_knn_kd / jzo_knn_bf for those rows. */
JZO_API int jzo_kd_knn(void *handle, int k, const int64_t *rows, int64_t first, int64_t nrows,
                       int32_t *idx, float *d2, int nthreads) {
    kdhandle *h = (kdhandle *)handle;
    if (!h || k < 1 || nrows < 0) return -1;
    if (!rows && (first < 0 || first + nrows > h->n)) return -1;
    kd_knn_rows(&h->T, h->n, k, rows, first, nrows, idx, d2, nthreads, NULL);
    return 0;
}

JZO_API void jzo_kd_free(void *handle) {
    kdhandle *h = (kdhandle *)handle;
    if (!h) return;
    kd_free(&h->T);
    free(h);
}

/* Exact FoF with a kd-tree. For each point i a range search visits the tree:
 *   - a box whose lower bound exceeds b2 holds no neighbour of i;
 *   - a box whose upper bound is <= b2 holds only neighbours of i: i is united
 *     with the box's first point and the box is flagged, meaning all of its
 *     points are connected through i (they are all linked to i);
 *   - a box whose own upper bound (its diagonal) is <= b2 is flagged up front
 *     (all of its points are pairwise linked);
 *   - otherwise leaves are checked point by point.
 * Flagged boxes are expanded at the end by uniting all their points. Each
 * thread unites into a private union-find; the forests are merged after. */
JZO_API int jzo_fof_kd(const float *pts, int64_t n, float b, int32_t *label, int nthreads) {
    if (!(b >= 0.0f)) return -1;
    float b2 = b * b;
    kdtree T;
    if (kd_build(&T, pts, n, nthreads)) return -2;
    int TH = clamp_threads(nthreads);
    uint8_t *whole = (uint8_t *)calloc((size_t)T.nnode + 1, 1);
    int32_t *loc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1) * (size_t)TH);
    if (!whole || !loc) { free(whole); free(loc); kd_free(&T); return -2; }
    for (int64_t id = 0; id < T.nnode; ++id) {
        kdnode *nd = &T.node[id];
        const float *c = nd->lo;
        /* upper bound of the distance between two points of the box: from the
         * corner lo to the box gives the per-axis extent hi - lo */
        if (nd->b > nd->a && box_up(c, nd->lo, nd->hi) <= b2) whole[id] = 1;
    }
#pragma omp parallel num_threads(TH)
    {
        int t = omp_get_thread_num();
        int32_t *par = loc + (size_t)t * (size_t)n;
        for (int64_t i = 0; i < n; ++i) par[i] = (int32_t)i;
        int64_t stack[256];
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            const float *q = pts + 3 * i;
            int sp = 0;
            if (n > 0) stack[sp++] = 0;
            while (sp > 0) {
                int64_t id = stack[--sp];
                kdnode *nd = &T.node[id];
                if (box_low(q, nd->lo, nd->hi) > b2) continue;
                if (box_up(q, nd->lo, nd->hi) <= b2) {
                    uf_unite(par, (int32_t)i, T.perm[nd->a]);
#pragma omp atomic write
                    whole[id] = 1;
                    continue;
                }
                if (nd->left < 0) {
                    for (int64_t s = nd->a; s < nd->b; ++s) {
                        int32_t j = T.perm[s];
                        if (j != i && d2f(q, pts + 3 * (int64_t)j) <= b2) uf_unite(par, (int32_t)i, j);
                    }
                } else {
                    stack[sp++] = nd->left;
                    stack[sp++] = nd->left + 1;
                }
            }
        }
    }
    for (int64_t i = 0; i < n; ++i) label[i] = (int32_t)i;
    for (int t = 0; t < TH; ++t) {
        int32_t *par = loc + (size_t)t * (size_t)n;
        for (int64_t i = 0; i < n; ++i) uf_unite(label, (int32_t)i, uf_find(par, (int32_t)i));
    }
    /* expand flagged boxes, top-down: a flagged box covers its subtree */
    {
        int64_t stack[256];
        int sp = 0;
        if (n > 0) stack[sp++] = 0;
        while (sp > 0) {
            int64_t id = stack[--sp];
            kdnode *nd = &T.node[id];
            if (whole[id]) {
                int32_t first = T.perm[nd->a];
                for (int64_t s = nd->a + 1; s < nd->b; ++s) uf_unite(label, first, T.perm[s]);
                continue;
            }
            if (nd->left >= 0) { stack[sp++] = nd->left; stack[sp++] = nd->left + 1; }
        }
    }
    for (int64_t i = 0; i < n; ++i) label[i] = uf_find(label, (int32_t)i);
    free(whole);
    free(loc);
    kd_free(&T);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* FP64 cross-check of the FoF linking decisions (a report, not a gate)       */

/* The same distance and box bounds evaluated in binary64. Coordinates are
 * float32, so they convert exactly; every step is correctly rounded and
 * monotone, so the computed box bounds bracket every member's computed d2d. */
static inline double d2d(const float *p, const float *q) {
    double dx = (double)p[0] - (double)q[0];
    double dy = (double)p[1] - (double)q[1];
    double dz = (double)p[2] - (double)q[2];
    return (dx * dx + dy * dy) + dz * dz;
}

static inline double box_low64(const float *q, const float *lo, const float *hi) {
    double g[3];
    for (int a = 0; a < 3; ++a) {
        double l = (double)lo[a] - (double)q[a];
        double h = (double)q[a] - (double)hi[a];
        double m = l > h ? l : h;
        g[a] = m > 0.0 ? m : 0.0;
    }
    return (g[0] * g[0] + g[1] * g[1]) + g[2] * g[2];
}

static inline double box_up64(const float *q, const float *lo, const float *hi) {
    double g[3];
    for (int a = 0; a < 3; ++a) {
        double l = (double)q[a] - (double)lo[a];
        double h = (double)hi[a] - (double)q[a];
        g[a] = l > h ? l : h;
    }
    return (g[0] * g[0] + g[1] * g[1]) + g[2] * g[2];
}

/* For the linking length b, compares the float32 predicate d2f <= fl(b*b)
 * with the binary64 predicate d2d <= (double)b * (double)b on every pair.
 * *only32 receives the number of pairs i < j that float32 links and binary64
 * does not, *only64 the reverse, and label64[n] the FoF labels (smallest
 * member index) of the binary64 graph, so that the caller can tell whether the
 * partition itself changes. A kd-tree visit skips boxes where both predicates
 * fail for every member, and takes whole boxes where both hold for every
 * member (no disagreement is possible there); only boxes straddling either
 * threshold are examined pair by pair. */
JZO_API int jzo_fof_f64_report(const float *pts, int64_t n, float b, int64_t *only32,
                               int64_t *only64, int32_t *label64, int nthreads) {
    if (!(b >= 0.0f) || !only32 || !only64) return -1;
    const float b2 = b * b;
    const double B = (double)b * (double)b;
    kdtree T;
    if (kd_build(&T, pts, n, nthreads)) return -2;
    int TH = clamp_threads(nthreads);
    uint8_t *whole = (uint8_t *)calloc((size_t)T.nnode + 1, 1);
    int32_t *loc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1) * (size_t)TH);
    if (!whole || !loc) { free(whole); free(loc); kd_free(&T); return -2; }
    for (int64_t id = 0; id < T.nnode; ++id) {
        kdnode *nd = &T.node[id];
        if (nd->b > nd->a && box_up64(nd->lo, nd->lo, nd->hi) <= B) whole[id] = 1;
    }
    int64_t c32 = 0, c64 = 0;
#pragma omp parallel num_threads(TH) reduction(+ : c32, c64)
    {
        int t = omp_get_thread_num();
        int32_t *par = loc + (size_t)t * (size_t)n;
        for (int64_t i = 0; i < n; ++i) par[i] = (int32_t)i;
        int64_t stack[256];
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            const float *q = pts + 3 * i;
            int sp = 0;
            if (n > 0) stack[sp++] = 0;
            while (sp > 0) {
                int64_t id = stack[--sp];
                kdnode *nd = &T.node[id];
                if (box_low(q, nd->lo, nd->hi) > b2 && box_low64(q, nd->lo, nd->hi) > B) continue;
                if (box_up(q, nd->lo, nd->hi) <= b2 && box_up64(q, nd->lo, nd->hi) <= B) {
                    uf_unite(par, (int32_t)i, T.perm[nd->a]);
#pragma omp atomic write
                    whole[id] = 1;
                    continue;
                }
                if (nd->left < 0) {
                    for (int64_t s = nd->a; s < nd->b; ++s) {
                        int32_t j = T.perm[s];
                        if (j == i) continue;
                        const float *p = pts + 3 * (int64_t)j;
                        int l32 = d2f(q, p) <= b2;
                        int l64 = d2d(q, p) <= B;
                        if (j > i) {
                            c32 += l32 && !l64;
                            c64 += l64 && !l32;
                        }
                        if (l64) uf_unite(par, (int32_t)i, j);
                    }
                } else {
                    stack[sp++] = nd->left;
                    stack[sp++] = nd->left + 1;
                }
            }
        }
    }
    for (int64_t i = 0; i < n; ++i) label64[i] = (int32_t)i;
    for (int t = 0; t < TH; ++t) {
        int32_t *par = loc + (size_t)t * (size_t)n;
        for (int64_t i = 0; i < n; ++i) uf_unite(label64, (int32_t)i, uf_find(par, (int32_t)i));
    }
    {
        int64_t stack[256];
        int sp = 0;
        if (n > 0) stack[sp++] = 0;
        while (sp > 0) {
            int64_t id = stack[--sp];
            kdnode *nd = &T.node[id];
            if (whole[id]) {
                int32_t first = T.perm[nd->a];
                for (int64_t s = nd->a + 1; s < nd->b; ++s) uf_unite(label64, first, T.perm[s]);
                continue;
            }
            if (nd->left >= 0) { stack[sp++] = nd->left; stack[sp++] = nd->left + 1; }
        }
    }
    for (int64_t i = 0; i < n; ++i) label64[i] = uf_find(label64, (int32_t)i);
    *only32 = c32;
    *only64 = c64;
    free(whole);
    free(loc);
    kd_free(&T);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* periodic kd-tree searches                                                  */

/* Bounds of the periodic distance between a point q and an axis-aligned box,
 * made safe for rounding: a wrapped difference fl(fl(q - x) -+ L) can be off
 * from the exact minimum-image difference by a few units of the last place of
 * L, so every per-axis gap is lowered (and every extent raised) by an
 * absolute margin of 2^-21 L, and the sums get a relative margin of 2^-20. */
static inline float per_gap(float q, float lo, float hi, float L) {
    if (q >= lo && q <= hi) return 0.0f;
    float a = lo - q;
    if (a < 0.0f) a += L;
    float b = q - hi;
    if (b < 0.0f) b += L;
    return a < b ? a : b;
}

static inline float per_low(const float *q, const float *lo, const float *hi, float L) {
    const float eps = L * 0x1p-21f;
    float s = 0.0f;
    for (int a = 0; a < 3; ++a) {
        float g = per_gap(q[a], lo[a], hi[a], L) - eps;
        g = g > 0.0f ? g : 0.0f;
        s += g * g;
    }
    return s * (1.0f - 0x1p-20f);
}

static inline float per_up(const float *q, const float *lo, const float *hi, float L) {
    const float eps = L * 0x1p-21f, h = 0.5f * L;
    float s = 0.0f;
    for (int a = 0; a < 3; ++a) {
        float u = fabsf(q[a] - lo[a]);
        float v = fabsf(hi[a] - q[a]);
        u = u > v ? u : v;
        u = (u < h ? u : h) + eps;
        s += u * u;
    }
    return s * (1.0f + 0x1p-20f);
}

/* jzo_knn_kd with the periodic distance: a subtree is skipped only if its
 * (rounding-safe) periodic lower bound exceeds the current k-th distance. */
JZO_API int jzo_knn_kd_per(const float *pts, int64_t n, float L, int k, const int64_t *rows,
                           int64_t nrows, int32_t *idx, float *d2, int nthreads) {
    if (k < 1 || n < 0 || !(L > 0.0f)) return -1;
    const float h = 0.5f * L;
    kdtree T;
    if (kd_build(&T, pts, n, nthreads)) return -2;
    int64_t R = rows ? nrows : n;
#pragma omp parallel num_threads(clamp_threads(nthreads))
    {
        float *bd = (float *)malloc(sizeof(float) * (size_t)k);
        int32_t *bj = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
        int64_t stack[256];
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < R; ++r) {
            int64_t i = rows ? rows[r] : r;
            const float *q = pts + 3 * i;
            int cnt = 0, sp = 0;
            if (n > 0) stack[sp++] = 0;
            while (sp > 0) {
                const kdnode *nd = &T.node[stack[--sp]];
                if (cnt == k && per_low(q, nd->lo, nd->hi, L) > bd[k - 1]) continue;
                if (nd->left < 0) {
                    for (int64_t t = nd->a; t < nd->b; ++t) {
                        int32_t j = T.perm[t];
                        float d = d2f_per(q, pts + 3 * (int64_t)j, L, h);
                        if (cnt == k && !pair_less(d, j, bd[k - 1], bj[k - 1])) continue;
                        int pos = cnt < k ? cnt : k - 1;
                        while (pos > 0 && pair_less(d, j, bd[pos - 1], bj[pos - 1])) {
                            bd[pos] = bd[pos - 1];
                            bj[pos] = bj[pos - 1];
                            --pos;
                        }
                        bd[pos] = d;
                        bj[pos] = j;
                        if (cnt < k) ++cnt;
                    }
                } else {
                    const kdnode *Ln = &T.node[nd->left], *Rn = &T.node[nd->left + 1];
                    float dl = per_low(q, Ln->lo, Ln->hi, L), dr = per_low(q, Rn->lo, Rn->hi, L);
                    if (dl <= dr) { stack[sp++] = nd->left + 1; stack[sp++] = nd->left; }
                    else { stack[sp++] = nd->left; stack[sp++] = nd->left + 1; }
                }
            }
            for (int t = 0; t < k; ++t) {
                idx[r * k + t] = t < cnt ? bj[t] : -1;
                d2[r * k + t] = t < cnt ? bd[t] : INFINITY;
            }
        }
        free(bd);
        free(bj);
    }
    kd_free(&T);
    return 0;
}

/* jzo_fof_kd with the periodic distance and the rounding-safe bounds (a box
 * is taken whole only if its periodic upper bound is within b). */
JZO_API int jzo_fof_kd_per(const float *pts, int64_t n, float L, float b, int32_t *label,
                           int nthreads) {
    if (!(b >= 0.0f) || !(L > 0.0f)) return -1;
    const float b2 = b * b, h = 0.5f * L;
    kdtree T;
    if (kd_build(&T, pts, n, nthreads)) return -2;
    int TH = clamp_threads(nthreads);
    uint8_t *whole = (uint8_t *)calloc((size_t)T.nnode + 1, 1);
    int32_t *loc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1) * (size_t)TH);
    if (!whole || !loc) { free(whole); free(loc); kd_free(&T); return -2; }
    for (int64_t id = 0; id < T.nnode; ++id) {
        kdnode *nd = &T.node[id];
        float ext[3], zero[3] = {0.0f, 0.0f, 0.0f};
        for (int a = 0; a < 3; ++a) ext[a] = nd->hi[a] - nd->lo[a];
        /* largest distance between two points of the box: its extents */
        if (nd->b > nd->a && per_up(zero, zero, ext, L) <= b2) whole[id] = 1;
    }
#pragma omp parallel num_threads(TH)
    {
        int t = omp_get_thread_num();
        int32_t *par = loc + (size_t)t * (size_t)n;
        for (int64_t i = 0; i < n; ++i) par[i] = (int32_t)i;
        int64_t stack[256];
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            const float *q = pts + 3 * i;
            int sp = 0;
            if (n > 0) stack[sp++] = 0;
            while (sp > 0) {
                int64_t id = stack[--sp];
                kdnode *nd = &T.node[id];
                if (per_low(q, nd->lo, nd->hi, L) > b2) continue;
                if (per_up(q, nd->lo, nd->hi, L) <= b2) {
                    uf_unite(par, (int32_t)i, T.perm[nd->a]);
#pragma omp atomic write
                    whole[id] = 1;
                    continue;
                }
                if (nd->left < 0) {
                    for (int64_t s = nd->a; s < nd->b; ++s) {
                        int32_t j = T.perm[s];
                        if (j != i && d2f_per(q, pts + 3 * (int64_t)j, L, h) <= b2)
                            uf_unite(par, (int32_t)i, j);
                    }
                } else {
                    stack[sp++] = nd->left;
                    stack[sp++] = nd->left + 1;
                }
            }
        }
    }
    for (int64_t i = 0; i < n; ++i) label[i] = (int32_t)i;
    for (int t = 0; t < TH; ++t) {
        int32_t *par = loc + (size_t)t * (size_t)n;
        for (int64_t i = 0; i < n; ++i) uf_unite(label, (int32_t)i, uf_find(par, (int32_t)i));
    }
    {
        int64_t stack[256];
        int sp = 0;
        if (n > 0) stack[sp++] = 0;
        while (sp > 0) {
            int64_t id = stack[--sp];
            kdnode *nd = &T.node[id];
            if (whole[id]) {
                int32_t first = T.perm[nd->a];
                for (int64_t s = nd->a + 1; s < nd->b; ++s) uf_unite(label, first, T.perm[s]);
                continue;
            }
            if (nd->left >= 0) { stack[sp++] = nd->left; stack[sp++] = nd->left + 1; }
        }
    }
    for (int64_t i = 0; i < n; ++i) label[i] = uf_find(label, (int32_t)i);
    free(whole);
    free(loc);
    kd_free(&T);
    return 0;
}

JZO_API int jzo_abi_version(void) { return 1; }
