// Host-side internals shared by the library's translation units: the tree
// object, device allocation, error reporting and the pipeline entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/jz.h"

struct Node;

// ---------------------------------------------------------------------------
// errors

jz_status jz_fail(jz_status code, const char *fmt, ...);
jz_status jz_hip_fail(hipError_t e, const char *what, const char *file, int line);

#define JZ_HIP(call)                                                          \
    do {                                                                      \
        hipError_t _e = (call);                                               \
        if (_e != hipSuccess) return jz_hip_fail(_e, #call, __FILE__, __LINE__); \
    } while (0)

#define JZ_TRY(call)                       \
    do {                                   \
        jz_status _s = (call);             \
        if (_s != JZ_OK) return _s;        \
    } while (0)

// ---------------------------------------------------------------------------
// device memory

struct AllocCtx {
    bool user = false;
    jz_allocator ua{};
    int device = 0;
};

void *dev_alloc(const AllocCtx &a, size_t bytes, hipStream_t s);
void dev_free(const AllocCtx &a, void *p, size_t bytes, hipStream_t s);
// Before a stream is destroyed: wait for the cached blocks last used on it
// and drop their events (an event last recorded on a destroyed stream must
// not be waited on).
void pool_forget_stream(int device, hipStream_t s);

// A device buffer owned by a tree or by one call.
struct DBuf {
    const AllocCtx *ac = nullptr;
    void *p = nullptr;
    size_t bytes = 0;
    hipStream_t s = nullptr;

    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { release(); }

    jz_status get(const AllocCtx *a, size_t b, hipStream_t st) {
        release();
        ac = a;
        s = st;
        bytes = b;
        if (b == 0) return JZ_OK;
        p = dev_alloc(*a, b, st);
        if (!p) {
            bytes = 0;
            return jz_fail(JZ_E_OOM, "device allocation of %zu bytes failed", b);
        }
        return JZ_OK;
    }
    // keep the buffer if it is already large enough
    jz_status ensure(const AllocCtx *a, size_t b, hipStream_t st) {
        if (p && bytes >= b) {
            s = st;
            return JZ_OK;
        }
        return get(a, b, st);
    }
    void release() {
        if (p) dev_free(*ac, p, bytes, s);
        p = nullptr;
        bytes = 0;
    }
    template <class T>
    T *as() const {
        return static_cast<T *>(p);
    }
};

// ---------------------------------------------------------------------------
// the tree

struct jz_tree {
    AllocCtx ac;
    jz_build_opts opts{};
    int64_t n = 0;

    // independent point sets sharing one tree (a single set for jz_build)
    int nsets = 1;
    std::vector<int64_t> set_off;  // host, nsets + 1
    int set_bits = 0;              // key bits above the Morton bits that hold the set id
    DBuf d_set_off;                // int64 [nsets + 1]

    // sorted points: float4 (x, y, z, input index as int bits)
    DBuf pts4;
    DBuf keys;  // uint64 [n], only with keep_keys

    int P = 0;                       // planes
    int64_t L[JZ_MAX_PLANES] = {};   // nodes per plane
    DBuf nodes[JZ_MAX_PLANES];       // Node [L_p]
    DBuf spl[JZ_MAX_PLANES];         // int [L_p + 1]
    DBuf leaf_base;                  // int [L_0]: first input index of the leaf's set (sets > 1)
    DBuf node_set[JZ_MAX_PLANES];    // int [L_p]: set of each node (sets > 1)

    // super nodes over the top plane (NGR grouping of Alg. 1)
    int64_t S = 0;
    DBuf super_spl;                  // int [S + 1] ranges into the top plane
    std::vector<int> super_set;      // host: set of each super node
    DBuf knn_top_seg, knn_top_list;  // dense super-node list (all pairs within a set)
    DBuf fof_top_seg, fof_top_list;  // dense super-node list (pairs s <= t within a set)

    // separate point types (jz_build_joint): points [0, n_src) are sources,
    // [n_src, n) queries; n_src = -1 otherwise. src_cnt[p][i]: source points
    // in node i of plane p.
    int64_t n_src = -1;
    DBuf src_cnt[JZ_MAX_PLANES];

    jz_stats st{};
};

// create a tree over nsets sets (offsets: host, nsets + 1); on error *out is NULL
jz_status tree_create(const float *points, const int64_t *offsets, int nsets, hipStream_t s,
                      const jz_build_opts *opts, const jz_allocator *alloc, jz_tree **out);

// pipelines (build.hip / knn.hip / fof.hip)
jz_status build_tree(jz_tree *t, const float *points, hipStream_t s);
// per-node source counts of a joint tree (t->n_src set)
jz_status source_counts(jz_tree *t, hipStream_t s);
// run_knn takes its per-call scratch from `scratch` when given (instead of
// the tree's allocator); every buffer it acquires after its fixed ones is a
// level list, acquired top level first and released bottom level first.
jz_status run_knn(jz_tree *t, int k, int32_t *idx, float *dist2, hipStream_t s,
                  const AllocCtx *scratch = nullptr);
// run_fof writes its call statistics to `st_out` when given (else to t->st)
jz_status run_fof(jz_tree *t, const float *b2_set_host, int32_t *label, hipStream_t s,
                  jz_stats *st_out = nullptr);
// the ranges jz_build_opts documents (JZ_E_INVALID with a message otherwise)
jz_status check_opts(const jz_build_opts &o);

bool jz_profiling();

// fill n 64-bit words with zero on stream s (a kernel, not a memset node)
jz_status zero_words(unsigned long long *p, size_t n, hipStream_t s);

// Stable LSD radix sort (8-bit digits) of n (key, value) pairs on the low
// `bits` key bits: k0 / v0 hold the input and, on return, the sorted pairs
// (the DBufs may have traded pointers with the scratch pair k1 / v1).
jz_status radix_sort_pairs(const AllocCtx *ac, DBuf &k0, DBuf &v0, DBuf &k1, DBuf &v1, int64_t n,
                           int bits, hipStream_t s);

// Process-wide memory of interaction-list sizes: the largest entries-per-node
// ratio seen for (operation, k, level), so that later calls on similar data
// start with lists that are large enough.
enum { CAP_KNN = 0, CAP_FOF = 1 };
double cap_hint(int op, int k, int level);
void cap_learn(int op, int k, int level, double ratio);
int64_t initial_cap(const jz_tree *t, int op, int k, int level);

// hipEvents for optional device timing; created only when profiling is on
struct EventSet {
    bool on = false;
    hipEvent_t e[4] = {};
    explicit EventSet(bool want) {
        if (!want) return;
        on = true;
        for (auto &x : e)
            if (hipEventCreate(&x) != hipSuccess) on = false;
    }
    ~EventSet() {
        for (auto &x : e)
            if (x) (void)hipEventDestroy(x);
    }
    hipEvent_t operator[](int i) const { return e[i]; }
};

// Device counters of one walk: [0, JZ_MAX_PLANES) list entries per level,
// [CTR_FLAG] the overflow flag, and from CTR_STATS the leaf-stage statistics,
// each spread over STAT_SLOTS words (a wave adds into slot item % STAT_SLOTS:
// one address shared by every wave serializes the adds in L2 and slows the
// kernel) and summed on the host.
constexpr int STAT_SLOTS = 256;
// Interaction-list space of a level is split into LIST_ARENAS arenas, each
// with its own fill counter: a wave reserves its segment in arena
// (receiver parent % LIST_ARENAS), which spreads the reservation atomics.
constexpr int LIST_ARENAS = 64;
constexpr int CTR_FLAG = JZ_MAX_PLANES * LIST_ARENAS;
constexpr int CTR_STATS = CTR_FLAG + 8;
inline size_t ctr_words(int nstats) { return (size_t)CTR_STATS + (size_t)nstats * STAT_SLOTS; }
// Entries a level asked for: the sum over its arenas, and the size every
// arena must have (the fullest arena times the arena count).
inline void arena_need(const unsigned long long *hc, int level, double &sum, double &need) {
    unsigned long long tot = 0, mx = 0;
    for (int a = 0; a < LIST_ARENAS; ++a) {
        const unsigned long long v = hc[(size_t)level * LIST_ARENAS + a];
        tot += v;
        mx = v > mx ? v : mx;
    }
    sum = (double)tot;
    need = (double)mx * LIST_ARENAS;
}
inline double stat_sum(const unsigned long long *hc, int i) {
    unsigned long long v = 0;
    for (int j = 0; j < STAT_SLOTS; ++j) v += hc[CTR_STATS + (size_t)i * STAT_SLOTS + j];
    return (double)v;
}

// launch helpers
inline unsigned blocks_for(int64_t items, int per_block) {
    int64_t b = (items + per_block - 1) / per_block;
    return (unsigned)(b < 1 ? 1 : b);
}
