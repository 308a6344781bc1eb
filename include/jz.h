/*
 * jz.h -- C ABI of the MI355X (gfx950) library for exact k-nearest-neighbour
 * search and friends-of-friends (FoF) clustering of 3-D float32 point sets.
 *
 * Method: arXiv 2604.05885 ("jz-tree"). Points are sorted along a Morton
 * (z-order) curve (section "Z-order sort"); a fixed-depth hierarchy of tree
 * planes is built from the gaps between consecutive sorted points (section
 * "Plane based tree-hierarchy", Eq. 7-9); a dual tree walk moves node-pair
 * interaction lists from the coarsest plane down to the leaves (Alg. 1-3,
 * Eq. 14-16), and the leaf stage computes exact kNN (kNN section) or links FoF
 * groups (FoF section, Eq. 18-19).
 *
 * Conventions for every call below:
 *  - Point and output buffers are DEVICE pointers (e.g. a torch tensor's
 *    data_ptr() on the current HIP device); `stream` is a hipStream_t (NULL =
 *    the default stream). The caller owns them.
 *  - Points are float32, row-major [n][3] (x, y, z), 4-byte aligned. They must
 *    be finite.
 *  - Distances are compared as squared distances with the fixed float32
 *    expression dist2 = fl(fl(fl(dx*dx) + fl(dy*dy)) + fl(dz*dz)),
 *    dx = fl(x_i - x_j), no fused multiply-add, subnormals kept. Results are
 *    exact with respect to that expression.
 *  - All calls in this header are synchronous: they return after their work
 *    on `stream` has completed, so that errors (capacity, non-finite input)
 *    can be reported.
 *  - Errors are returned as jz_status; jz_last_error() gives a message
 *    (thread-local, valid until the next call on the same thread).
 *  - A tree may be used by one thread / stream at a time; distinct trees are
 *    independent.
 */
#ifndef JZ_H
#define JZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define JZ_API __attribute__((visibility("default")))
#else
#define JZ_API
#endif

typedef enum jz_status {
    JZ_OK = 0,
    JZ_E_INVALID = 1,      /* bad argument (null pointer, n out of range, k < 1, b < 0 or NaN) */
    JZ_E_NONFINITE = 2,    /* an input coordinate is NaN or infinite */
    JZ_E_UNSUPPORTED = 3,  /* k > JZ_MAX_K */
    JZ_E_CAPACITY = 4,     /* interaction list overflow with auto_regrow = 0 */
    JZ_E_OOM = 5,          /* device allocation failed (jz_knn_fof: also host memory) */
    JZ_E_DEVICE = 6        /* a HIP runtime error */
} jz_status;

/* Optional device allocator. alloc returns NULL on failure; memory must be
 * device memory on the current device, 256-byte aligned. free receives the
 * pointer and the size that alloc was called with. Both may be called from
 * inside any jz_* call. NULL allocator = the library's own caching pool over
 * hipMalloc. */
typedef struct jz_allocator {
    void *ctx;
    void *(*alloc)(void *ctx, size_t bytes, void *stream);
    void (*free)(void *ctx, void *ptr, size_t bytes, void *stream);
} jz_allocator;

/* Build options (tree-plane hierarchy of the paper's section on the plane
 * based hierarchy; defaults follow its Eq. 8-9 and Alg. 1). */
typedef struct jz_build_opts {
    int leaf_max;          /* N_max^(0): most points per leaf. Default 64, range [1, 64]. */
    int coarsen;           /* c in N_max^(p) = N_max^(0) c^p. Default 8, range [2, 64]. */
    int n_target;          /* stop adding planes when N / (N_max^(p)/2) < n_target. Default 1000. */
    int ngr;               /* top nodes per super node (NGR of Alg. 1). Default 32, range [1, 64]. */
    int key_bits;          /* Morton bits per dimension, range [1, 21]; 0 (default): automatic,
                              b = ceil(log2(n) / 3) + 5 bits (at least 10), i.e. cells 32 times
                              finer than the mean point spacing, raised to the most that the
                              radix passes b needs can hold (a pass sorts 8 bits of the key:
                              13 bits and 5 passes at n = 2^24), at most 21. Results never
                              depend on it; fewer bits mean fewer radix-sort passes. */
    float list_per_node;   /* initial interaction-list capacity in entries per node. Default 96.
                              With auto_regrow = 1 the library may start larger, from the list
                              sizes it has seen in this process. */
    int auto_regrow;       /* 1 (default): on list overflow grow and rerun; 0: use exactly
                              list_per_node and return JZ_E_CAPACITY on overflow. */
    int keep_keys;         /* 1: keep the sorted Morton keys for jz_tree_export. Default 0. */
    int sort_max;          /* kNN: longest interaction list put in r_low order before it is
                              walked (so the walk can stop at the first entry beyond its
                              radius); longer lists are read unordered. Default 8192, range
                              [256, 8192]. */
    float period;          /* > 0: the points lie in the periodic cube [0, period)^3 (coordinates
                              outside it: JZ_E_INVALID) and kNN / FoF use the minimum-image
                              distance: each coordinate difference dx = fl(x_i - x_j) becomes
                              fl(dx - period) if dx > fl(period / 2) and fl(dx + period) if
                              dx < -fl(period / 2), then the fixed dist2 expression. The paper's
                              periodic cosmological case. 0 (default): open space. */
    float reg_fmax;        /* > 0: regularization (paper: section on regularization) with
                              f_max = reg_fmax (the paper uses about 50): on every plane, nodes
                              may not exceed f_max times V90, the point-weighted mean volume of
                              the smallest nodes holding 90% of the points, so gaps whose level
                              (volume 2^level of the Morton cell spanning them) exceeds
                              log2(f_max V90) are split as well. Keeps a few points far from the
                              bulk out of huge nodes. 0 (default): off. Results never depend
                              on it. */
} jz_build_opts;

/* Fill *o with the defaults above. */
JZ_API void jz_default_opts(jz_build_opts *o);

typedef struct jz_tree jz_tree;

/* Sort the n points in z-order and build the tree planes (paper: section on
 * z-order trees, Eq. 7-9). `points` is read only during this call; the tree
 * keeps its own sorted copy. n in [0, 2^31 - 2]. opts/alloc may be NULL.
 * On success *out owns device memory until jz_tree_free. Errors:
 * JZ_E_INVALID, JZ_E_NONFINITE, JZ_E_OOM, JZ_E_DEVICE (*out is then NULL). */
JZ_API jz_status jz_build(const float *points, int64_t n, void *stream, const jz_build_opts *opts,
                   const jz_allocator *alloc, jz_tree **out);

/* Largest k of jz_knn. */
#define JZ_MAX_K 256

/* Exact k nearest neighbours of every point, self included (paper: kNN
 * section, Alg. 1-3 and the LeafToLeaf kernel). Row i of idx[n][k] holds the
 * input indices of the k points closest to point i (input order), ascending by
 * (dist2, index); dist2[n][k] holds their squared distances. If k > n the row
 * tail is idx = -1, dist2 = +inf. k in [1, JZ_MAX_K] (larger: JZ_E_UNSUPPORTED);
 * k > 32 runs the leaf stage in passes of 32 neighbours, each continuing after
 * the last (dist2, index) of the pass before, as the paper's LeafToLeaf does
 * above its 32-neighbour limit. idx and dist2 are device buffers of n*k
 * elements. */
JZ_API jz_status jz_knn(jz_tree *t, int k, int32_t *idx, float *dist2, void *stream);

/* ---- separate query and source points ---------------------------------
 * (paper: section on multiple point types) One tree built jointly over the
 * n_src source points and the n_qry query points (both DEVICE float32
 * [n][3], read only during the call): the two arrays are concatenated
 * before the z-order sort, so the hierarchy adapts to both distributions,
 * and every node records how many source points it holds. Nodes are split on
 * the combined count (at most leaf_max points of both types together per
 * leaf). Errors as jz_build; a periodic box (opts->period > 0) is not
 * supported here (JZ_E_UNSUPPORTED). Such a tree takes jz_knn_query only
 * (jz_knn, jz_fof and the catalogue return JZ_E_INVALID on it). */
JZ_API jz_status jz_build_joint(const float *sources, int64_t n_src, const float *queries,
                                int64_t n_qry, void *stream, const jz_build_opts *opts,
                                const jz_allocator *alloc, jz_tree **out);

/* Exact k nearest source points of every query point: row i of
 * idx[n_qry][k] (DEVICE) holds source indices (0-based into `sources`),
 * ascending by (dist2, index), dist2[n_qry][k] their squared distances; a
 * query equal to a source point finds it at distance 0. Rows beyond n_src
 * sources pad with idx = -1, dist2 = +inf. k in [1, JZ_MAX_K]. */
JZ_API jz_status jz_knn_query(jz_tree *t, int k, int32_t *idx, float *dist2, void *stream);

/* Friends-of-friends groups (paper: FoF section, Eq. 18): connected
 * components of the graph linking every pair with dist2 <= fl(b*b).
 * label[n] (device, input order) receives, for each point, the smallest input
 * index in its group. b must be finite and >= 0. */
JZ_API jz_status jz_fof(jz_tree *t, float b, int32_t *label, void *stream);

/* Release the tree and its device memory (NULL is ignored). */
JZ_API void jz_tree_free(jz_tree *t);

/* Size of the fixed device array behind jz_knn_noalloc. */
#define JZ_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/* jz_knn without any device allocation during the call, for callers that
 * cannot allocate there (tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, results and errors as jz_knn on a tree built
 * beforehand with jz_build / jz_forest_build. The call's scratch (walk
 * counters, per-level lists, work items) is carved from one file-scope device
 * array of JZ_NOALLOC_SCRATCH_BYTES (128 MiB) that each GPU the library runs
 * on holds until the process ends; the walk's lists take about 40 bytes per
 * point at k = 16 on clustered data, so about 3e6 points fit there. A call
 * needing more returns JZ_E_CAPACITY (use jz_knn). Calls on one GPU share
 * the array and are serialized by the library (each returns after its work
 * has finished, like jz_knn); the array keeps the last call's contents and
 * every call clears what it needs. */
JZ_API jz_status jz_knn_noalloc(jz_tree *t, int k, int32_t *idx, float *dist2, void *stream);

/* Bytes of device memory the tree holds between calls (sorted points, node
 * planes, splits, top-level lists; 0 for NULL). Scratch memory of a
 * jz_knn / jz_fof call is taken from the allocator during the call and
 * returned before it ends. */
JZ_API int64_t jz_tree_size(const jz_tree *t);

/* ---- batched solving: many independent point sets in one tree ----------
 * (the paper motivates repeated evaluations, e.g. simulation-based inference,
 * in its introduction). Set s holds points[offsets[s] .. offsets[s+1]) of the
 * concatenated array; `offsets` is a HOST array of nsets + 1 non-decreasing
 * values with offsets[0] = 0 and offsets[nsets] = n, nsets in [1, 65536].
 * One sort and one set of kernel launches cover all sets; no node straddles
 * two sets and sets never interact, so every set's result equals what
 * jz_build + jz_knn / jz_fof give for that set alone.
 * On a forest, jz_knn writes set-local neighbour indices (row i of set s is
 * global row offsets[s] + i; entries are indices within set s), and jz_fof
 * uses one linking length for all sets with set-local labels. */
JZ_API jz_status jz_forest_build(const float *points, const int64_t *offsets, int nsets, void *stream,
                          const jz_build_opts *opts, const jz_allocator *alloc, jz_tree **out);

/* FoF on a forest with one linking length per set (b: HOST array of nsets
 * finite values >= 0). label[n] is set-local (smallest index within the set). */
JZ_API jz_status jz_forest_fof(jz_tree *t, const float *b, int32_t *label, void *stream);

/* ---- FoF catalogue ---------------------------------------------------------
 * (paper: FoF section, catalogue reduction) The groups of jz_fof with
 * linking length b, brought into group order and summarized. Group order is
 * a stable sort of the input indices by group label: groups follow their
 * labels (smallest member index) in ascending order, and each group is one
 * contiguous block of ascending input indices (the input-order counterpart
 * of the paper's sort into group order, since every result of this library
 * is in input order). Per group with at least min_members points: */
typedef struct jz_group {
    int32_t label;      /* the group's label: its smallest member index */
    int32_t count;      /* members (the mass, at unit point mass) */
    int64_t first;      /* offset of the group's block in order[] */
    double cm[3];       /* centre of mass: mean member position (binary64 sums) */
    double vcm[3];      /* centre-of-mass velocity: mean member velocity (0 without vel) */
    double r_inertia;   /* inertia radius: RMS distance of the members from cm */
} jz_group;

/* On a tree from jz_build (one set, open space: a periodic tree returns
 * JZ_E_INVALID): label[n] (DEVICE, may be NULL) receives
 * the labels as jz_fof gives them; order[n] (DEVICE) the input indices in
 * group order; groups[max_groups] (DEVICE) the groups with >= min_members
 * (>= 1) points, in label order; *ngroups (HOST) their number. vel: DEVICE
 * float32 [n][3] member velocities in input order, or NULL. If more than
 * max_groups groups qualify, returns JZ_E_CAPACITY with *ngroups set to the
 * number needed (label and order are complete then). The sums are binary64
 * in an order that may vary between calls (atomics), so cm, vcm and
 * r_inertia may differ in the last bits from run to run; label, order,
 * count, first are exact. */
JZ_API jz_status jz_fof_catalogue(jz_tree *t, float b, int min_members, const float *vel,
                                  int32_t *label, int32_t *order, jz_group *groups,
                                  int64_t max_groups, int64_t *ngroups, void *stream);

/* ---- autotuning -----------------------------------------------------------
 * Time the build plus the requested operations on the caller's workload for
 * each candidate setting and return the fastest in *best and its time (ms,
 * best of two runs) in *best_ms. Candidates: leaf_max in {32, 48, 64} x
 * coarsen in {4, 8, 16}, then, from the best of those, n_target in {500,
 * 2000} and then ngr in {16, 64}; other fields are taken from *base or the
 * defaults. (A leaf is one wave of queries, so leaves hold at most 64 points;
 * leaves of up to 16 or 32 points get 4 or 2 lanes per query by themselves.)
 * points / offsets / nsets as for jz_forest_build (offsets may be NULL for one
 * set of n points; then nsets is n). k in [1, JZ_MAX_K] runs kNN, k = 0 skips
 * it; b (HOST, one value per set) runs FoF, NULL skips it. The winner is
 * remembered for the signature (device architecture, k, FoF or not, number
 * of sets, log2 of the point count) for the rest of the process, and later
 * calls with that signature return it without timing. If the environment
 * variable JZ_TUNE_CACHE names a file, winners are also appended to it as one
 * JSON object per line ({"arch", "k", "fof", "sets", "log2n", "leaf_max",
 * "coarsen", "n_target", "ngr", "ms"}), and a signature not yet tuned in this
 * process is looked up there first (the last matching line wins; lines whose
 * options are out of range are ignored). Results of the method never depend on
 * these options. */
JZ_API jz_status jz_autotune(const float *points, const int64_t *offsets, int64_t nsets,
                             int k, const float *b, void *stream, const jz_build_opts *base,
                             jz_build_opts *best, double *best_ms);

/* ---- serving: a continuous-batching request loop -----------------------
 * Requests (kNN or FoF on their own point sets) are submitted at any time from
 * any thread. Worker threads, each with its own HIP stream, repeatedly take
 * the oldest pending request that fits the free part of the device-memory
 * budget and every later pending request of the same kind (same op, same k),
 * as far as the budget and the batch caps allow, solve them as one forest
 * (one sort, one set of launches), and copy each result to its request's
 * output buffers. The oldest pending request may be passed over this way by
 * later ones at most 8 times; after that no batch starts until it fits (no
 * request waits forever behind smaller ones). Requests that arrive
 * while batches run join the next batch a worker forms; batches on different
 * streams overlap on the device. Each result is identical to what
 * jz_build + jz_knn / jz_fof give for that request alone. */
typedef struct jz_server jz_server;

enum { JZ_OP_KNN = 0, JZ_OP_FOF = 1 };

typedef struct jz_request {
    int op;                  /* JZ_OP_KNN or JZ_OP_FOF */
    int k;                   /* kNN: neighbours per point, [1, JZ_MAX_K] */
    float b;                 /* FoF: linking length, finite, >= 0 */
    const float *points;     /* DEVICE [n][3]; must stay valid until the request is done */
    int64_t n;               /* [0, 2^31-2] */
    int32_t *idx;            /* kNN output, DEVICE [n][k] (input order, indices within the request) */
    float *dist2;            /* kNN output, DEVICE [n][k] */
    int32_t *label;          /* FoF output, DEVICE [n] (smallest index within the request's group) */
    void *stream;            /* the caller's hipStream_t (NULL = default stream): jz_server_submit
                                records an event on it, and the request's work starts only after
                                everything queued on it before the call (e.g. the kernels that
                                write `points`). Results are complete once the request is done;
                                the caller orders its later reads after jz_server_wait / _poll. */
} jz_request;

typedef struct jz_server_opts {
    size_t hbm_budget;       /* device bytes the in-flight batches may use (estimated per
                                request from n, op and k). Default 200e9. */
    int streams;             /* worker threads / HIP streams (batches in flight), [1, 16]. Default 4. */
    int64_t max_batch_points;/* most points per batch. Default 2^26. */
    int max_batch_sets;      /* most requests per batch, [1, 65536]. Default 4096. */
    jz_build_opts build;     /* tree options for every batch */
} jz_server_opts;

JZ_API void jz_server_default_opts(jz_server_opts *o);

/* Start the workers on the current HIP device. */
JZ_API jz_status jz_server_create(const jz_server_opts *opts, jz_server **out);

/* Queue a request (copied; the buffers it points to are not). *ticket
 * identifies it. The request reads its points only after the work queued on
 * r->stream before this call has finished (an event is recorded there), so
 * points still being written on that stream are safe to submit. Invalid
 * requests, and requests whose estimated footprint exceeds the whole budget,
 * are rejected here (JZ_E_INVALID / JZ_E_OOM). */
JZ_API jz_status jz_server_submit(jz_server *s, const jz_request *r, uint64_t *ticket);

/* *done = 1 once the request's outputs are complete on the device; then
 * *result holds its status and *done_ns the completion time on the clock of
 * jz_now_ns(). Any output pointer may be NULL. When the request failed, its
 * error message becomes the calling thread's jz_last_error(). */
JZ_API jz_status jz_server_poll(jz_server *s, uint64_t ticket, int *done, jz_status *result,
                                int64_t *done_ns);

/* Block until the request is done (same outputs as jz_server_poll). */
JZ_API jz_status jz_server_wait(jz_server *s, uint64_t ticket, jz_status *result,
                                int64_t *done_ns);

/* Forget a finished ticket (its record is freed). */
JZ_API jz_status jz_server_release(jz_server *s, uint64_t ticket);

typedef struct jz_serve_stats {
    int64_t submitted, completed, failed, batches;
    int64_t points_done;
    int64_t pending;          /* submitted, not yet in a batch */
    int64_t in_flight_bytes;  /* budget in use by running batches */
    int64_t max_batch_sets_seen;
} jz_serve_stats;

JZ_API jz_status jz_server_stats(jz_server *s, jz_serve_stats *st);

/* Finish every queued and running request, stop the workers, free the server. */
JZ_API void jz_server_destroy(jz_server *s);

/* Monotonic clock used for completion times (nanoseconds). */
JZ_API int64_t jz_now_ns(void);

#define JZ_MAX_PLANES 16

typedef struct jz_stats {
    int64_t n;                       /* points */
    int planes;                      /* number of tree planes P */
    int64_t nodes[JZ_MAX_PLANES];    /* nodes per plane (plane 0 = leaves) */
    int64_t super_nodes;             /* super nodes over the top plane */
    /* last jz_knn / jz_fof call on this tree */
    int64_t list_entries[JZ_MAX_PLANES + 1]; /* list entries produced per level (index p = plane p, P = super) */
    int64_t leaf_pairs;              /* leaf-leaf interactions in the leaf list */
    int64_t leaf_pairs_visited;      /* of those, visited before the early exit */
    double evaluations;              /* point-pair distance evaluations in the leaf stage */
    double leaf_ms;                  /* leaf-stage kernel time (ms), when profiling is on */
    double total_ms;                 /* whole call, device time (ms), when profiling is on */
    int reruns;                      /* capacity reruns in the last call */
    int64_t insert_rounds;           /* kNN leaf stage: wave-level top-k insert rounds */
    int64_t tile_steps;              /* kNN leaf stage: wave-level candidate steps */
    int64_t lists_sorted_long;       /* kNN leaf stage: lists longer than the 256 entries staged in
                                        LDS, put in r_low order (in the wave's LDS scratch up to
                                        1024 entries, beforehand in HBM up to sort_max) */
    int64_t lists_unordered;         /* kNN leaf stage: lists longer than sort_max, read unordered */
    /* kNN lists put in r_low order in HBM before they are walked, by the sorter
     * for lists of up to 1024 entries ([0]) and by the one for longer lists, up
     * to sort_max ([1]); index p < JZ_MAX_PLANES: the lists of plane p + 1 read
     * by walk level p; index JZ_MAX_PLANES: the leaf lists read by the leaf
     * stage (only those longer than it sorts itself, 1024 entries). */
    int64_t lists_presorted[JZ_MAX_PLANES + 1][2];
} jz_stats;

/* Statistics of the tree and of its last kNN / FoF call. */
JZ_API jz_status jz_tree_stats(const jz_tree *t, jz_stats *s);

/* jz_knn and jz_fof on one tree in one call, the two running concurrently:
 * both only read the tree, so the FoF half runs from a second host thread on a
 * stream the library keeps per device, while the calling thread runs the kNN
 * half on `stream`. Both start after the work already queued on `stream`, and
 * work queued on `stream` afterwards starts after both. idx, dist2 and label
 * receive exactly what jz_knn(t, k, idx, dist2) and jz_fof(t, b, label) write;
 * the arguments are checked as those two calls check them (a joint tree:
 * JZ_E_INVALID). knn_st and fof_st (HOST, each may be NULL) receive the
 * statistics of each half, as jz_tree_stats reports them after that call
 * alone; jz_tree_stats afterwards reports the kNN half. With a user allocator
 * (jz_build's `alloc`), its callbacks may be called from both threads at once.
 * Errors: the kNN half's status and message if it failed, else the FoF
 * half's. Like jz_knn and jz_fof, the call returns when both halves are
 * done. */
JZ_API jz_status jz_knn_fof(jz_tree *t, int k, int32_t *idx, float *dist2, float b,
                            int32_t *label, void *stream, jz_stats *knn_st, jz_stats *fof_st);

/* Turn device-time measurement of the leaf stage and of whole calls on (1) or
 * off (0) for calls made by this thread. Off by default. */
JZ_API void jz_set_profiling(int on);

/* Copy tree internals to HOST buffers, for tests. Any pointer may be NULL.
 * order[n]: input index of each z-sorted point; keys[n]: sorted Morton keys
 * (only if built with keep_keys = 1, else JZ_E_INVALID); for plane p, spl
 * receives nodes[p] + 1 entries: plane 0 point offsets, plane p > 0 indices
 * into the plane p-1 node array. */
JZ_API jz_status jz_tree_export(const jz_tree *t, int32_t *order, uint64_t *keys, int plane,
                         int32_t *spl);

/* Return the library's cached (currently unused) device memory to the
 * runtime. Trees keep their own memory until jz_tree_free. */
JZ_API void jz_release_cached(void);

/* Thread-local message of the last error (empty string if none). */
JZ_API const char *jz_last_error(void);

/* ABI version of this header (4). */
JZ_API int jz_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* JZ_H */
