// The C ABI (include/jz.h): argument checks, error reporting, the caching
// device pool, and tree lifetime. The pipelines live in build.hip, knn.hip
// and fof.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <tuple>
#include <algorithm>
#include <unordered_map>
#include <vector>

#include "jz_internal.h"

// ---------------------------------------------------------------------------
// errors and per-thread settings

static thread_local std::string g_err;
static thread_local bool g_prof = false;

jz_status jz_fail(jz_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

jz_status jz_hip_fail(hipError_t e, const char *what, const char *file, int line) {
    (void)hipGetLastError();
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return jz_fail(JZ_E_OOM, "%s: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    return jz_fail(JZ_E_DEVICE, "%s: %s (%s:%d)", what, hipGetErrorString(e), file, line);
}

bool jz_profiling() { return g_prof; }

// ---------------------------------------------------------------------------
// learned list capacities

namespace {
std::mutex g_cap_m;
std::map<std::tuple<int, int, int>, double> g_cap;
}  // namespace

double cap_hint(int op, int k, int level) {
    std::lock_guard<std::mutex> lk(g_cap_m);
    auto it = g_cap.find(std::make_tuple(op, k, level));
    return it == g_cap.end() ? 0.0 : it->second;
}

void cap_learn(int op, int k, int level, double ratio) {
    std::lock_guard<std::mutex> lk(g_cap_m);
    double &r = g_cap[std::make_tuple(op, k, level)];
    if (ratio > r) r = ratio;
}

int64_t initial_cap(const jz_tree *t, int op, int k, int level) {
    // with auto_regrow off the capacity is exactly what the options ask for
    const double hint = t->opts.auto_regrow ? 1.15 * cap_hint(op, k, level) : 0.0;
    const double ratio = std::max<double>(t->opts.list_per_node, hint);
    const double c = ratio * (double)t->L[level] + 1024.0;
    return c > (double)INT32_MAX ? (int64_t)INT32_MAX : (int64_t)c;
}

// ---------------------------------------------------------------------------
// Caching device pool. Freed blocks keep an event recorded on the stream that
// last used them; a block is handed to a different stream only after that
// event has completed, so stream order protects every reuse.

namespace {

struct Block {
    void *p;
    size_t bytes;
    hipStream_t s;
    hipEvent_t ev;
};

struct Pool {
    std::mutex m;
    std::multimap<size_t, Block> free;
    std::unordered_map<void *, size_t> live;
};

Pool &pool(int dev) {
    static Pool pools[64];
    return pools[dev & 63];
}

size_t round_size(size_t b) {
    if (b >= (1u << 20)) return (b + (2u << 20) - 1) & ~(size_t)((2u << 20) - 1);
    size_t r = 256;
    while (r < b) r <<= 1;
    return r;
}

// Wait for the work a free block's event marks and destroy the event. An
// event whose wait fails (for instance one last recorded on a stream that no
// longer exists) is replaced by a wait for the whole device, and the error is
// cleared so that it cannot surface in an unrelated later check.
void retire_event(hipEvent_t ev) {
    if (!ev) return;
    if (hipEventSynchronize(ev) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipDeviceSynchronize();
        (void)hipGetLastError();
    }
    if (hipEventDestroy(ev) != hipSuccess) (void)hipGetLastError();
}

void release_all(Pool &P) {
    for (auto &kv : P.free) {
        retire_event(kv.second.ev);
        (void)hipFree(kv.second.p);
    }
    P.free.clear();
}

}  // namespace

void *dev_alloc(const AllocCtx &a, size_t bytes, hipStream_t s) {
    if (a.user) return a.ua.alloc(a.ua.ctx, bytes, (void *)s);
    Pool &P = pool(a.device);
    const size_t want = round_size(bytes);
    Block blk{};
    bool found = false;
    {
        std::lock_guard<std::mutex> lk(P.m);
        auto it = P.free.lower_bound(want);
        if (it != P.free.end() && it->first <= 2 * want) {
            blk = it->second;
            P.free.erase(it);
            found = true;
        }
    }
    if (found) {
        if (blk.ev) {
            if (blk.s != s) {
                retire_event(blk.ev);
            } else if (hipEventDestroy(blk.ev) != hipSuccess) {
                (void)hipGetLastError();
            }
        }
        std::lock_guard<std::mutex> lk(P.m);
        P.live[blk.p] = blk.bytes;
        return blk.p;
    }
    void *p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        std::lock_guard<std::mutex> lk(P.m);
        release_all(P);
        if (hipMalloc(&p, want) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    std::lock_guard<std::mutex> lk(P.m);
    P.live[p] = want;
    return p;
}

void dev_free(const AllocCtx &a, void *p, size_t bytes, hipStream_t s) {
    if (!p) return;
    if (a.user) {
        a.ua.free(a.ua.ctx, p, bytes, (void *)s);
        return;
    }
    Pool &P = pool(a.device);
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
        if (hipEventRecord(ev, s) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipStreamSynchronize(s);
            (void)hipEventDestroy(ev);
            ev = nullptr;
        }
    } else {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(s);
        ev = nullptr;
    }
    std::lock_guard<std::mutex> lk(P.m);
    auto it = P.live.find(p);
    const size_t real = it != P.live.end() ? it->second : round_size(bytes);
    if (it != P.live.end()) P.live.erase(it);
    P.free.emplace(real, Block{p, real, s, ev});
}

void pool_forget_stream(int device, hipStream_t s) {
    Pool &P = pool(device);
    std::lock_guard<std::mutex> lk(P.m);
    for (auto &kv : P.free) {
        if (kv.second.s != s) continue;
        retire_event(kv.second.ev);
        kv.second.ev = nullptr;
        kv.second.s = nullptr;
    }
}

// ---------------------------------------------------------------------------

jz_status make_tree_impl(const float *points, const int64_t *offsets, int nsets, int64_t n,
                         void *stream, const jz_build_opts *opts, const jz_allocator *alloc,
                         jz_tree **out);

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else if (prev == dev) prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// The stream the FoF half of jz_knn_fof runs on: one per device, created on
// first use and kept until the process ends (the pool keeps, for blocks freed
// on it, events recorded on it).
hipStream_t side_stream(int dev, jz_status &st) {
    static std::mutex m;
    static hipStream_t streams[64] = {};
    std::lock_guard<std::mutex> lk(m);
    hipStream_t &x = streams[dev & 63];
    if (!x) {
        const hipError_t e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking);
        if (e != hipSuccess) {
            x = nullptr;
            st = jz_hip_fail(e, "hipStreamCreateWithFlags", __FILE__, __LINE__);
        }
    }
    return x;
}

struct EventGuard {
    hipEvent_t e = nullptr;
    ~EventGuard() {
        if (e && hipEventDestroy(e) != hipSuccess) (void)hipGetLastError();
    }
};

}  // namespace

jz_status check_opts(const jz_build_opts &o) {
    if (o.leaf_max < 1 || o.leaf_max > 64) return jz_fail(JZ_E_INVALID, "leaf_max must be in [1, 64]");
    if (o.coarsen < 2 || o.coarsen > 64) return jz_fail(JZ_E_INVALID, "coarsen must be in [2, 64]");
    if (o.n_target < 1) return jz_fail(JZ_E_INVALID, "n_target must be >= 1");
    if (o.ngr < 1 || o.ngr > 64) return jz_fail(JZ_E_INVALID, "ngr must be in [1, 64]");
    if (o.key_bits < 0 || o.key_bits > 21) return jz_fail(JZ_E_INVALID, "key_bits must be in [0, 21]");
    if (!(o.list_per_node >= 1.0f) || !std::isfinite(o.list_per_node))
        return jz_fail(JZ_E_INVALID, "list_per_node must be finite and >= 1");
    if (o.sort_max < 256 || o.sort_max > 8192)
        return jz_fail(JZ_E_INVALID, "sort_max must be in [256, 8192]");
    if (!(o.period >= 0.0f) || !std::isfinite(o.period))
        return jz_fail(JZ_E_INVALID, "period must be finite and >= 0");
    if (!(o.reg_fmax >= 0.0f) || !std::isfinite(o.reg_fmax))
        return jz_fail(JZ_E_INVALID, "reg_fmax must be finite and >= 0");
    return JZ_OK;
}

jz_status tree_create(const float *points, const int64_t *offsets, int nsets, hipStream_t s,
                      const jz_build_opts *opts, const jz_allocator *alloc, jz_tree **out) {
    return make_tree_impl(points, offsets, nsets, offsets[nsets], (void *)s, opts, alloc, out);
}

jz_status make_tree_impl(const float *points, const int64_t *offsets, int nsets, int64_t n,
                         void *stream, const jz_build_opts *opts, const jz_allocator *alloc,
                         jz_tree **out) {
    if (!out) return jz_fail(JZ_E_INVALID, "out is NULL");
    *out = nullptr;
    if (n < 0 || n > (int64_t)INT32_MAX - 1) return jz_fail(JZ_E_INVALID, "n must be in [0, 2^31-2]");
    if (n > 0 && !points) return jz_fail(JZ_E_INVALID, "points is NULL");
    if (alloc && (!alloc->alloc || !alloc->free))
        return jz_fail(JZ_E_INVALID, "allocator needs both alloc and free");
    jz_build_opts o;
    jz_default_opts(&o);
    if (opts) o = *opts;
    JZ_TRY(check_opts(o));
    jz_tree *t = new (std::nothrow) jz_tree();
    if (!t) return jz_fail(JZ_E_OOM, "host allocation failed");
    int dev = 0;
    const hipError_t de = hipGetDevice(&dev);
    if (de != hipSuccess) {
        (void)hipGetLastError();
        delete t;
        return jz_fail(JZ_E_DEVICE, "no HIP device (hipGetDevice: %s)", hipGetErrorString(de));
    }
    t->ac.device = dev;
    if (alloc) {
        t->ac.user = true;
        t->ac.ua = *alloc;
    }
    t->opts = o;
    t->n = n;
    t->nsets = nsets;
    t->set_off.assign(offsets, offsets + nsets + 1);
    int sb = 0;
    while ((1 << sb) < nsets) ++sb;
    t->set_bits = sb;
    hipStream_t s = (hipStream_t)stream;
    jz_status st = t->d_set_off.get(&t->ac, (nsets + 1) * sizeof(int64_t), s);
    if (st == JZ_OK) {
        hipError_t e = hipMemcpyAsync(t->d_set_off.p, t->set_off.data(), (nsets + 1) * sizeof(int64_t),
                                      hipMemcpyHostToDevice, s);
        if (e != hipSuccess) st = jz_hip_fail(e, "hipMemcpyAsync(set offsets)", __FILE__, __LINE__);
    }
    if (st == JZ_OK) st = build_tree(t, points, s);
    if (st != JZ_OK) {
        (void)hipStreamSynchronize(s);
        delete t;
        return st;
    }
    t->st.n = n;
    *out = t;
    return JZ_OK;
}

extern "C" {

void jz_default_opts(jz_build_opts *o) {
    if (!o) return;
    o->leaf_max = 64;
    o->coarsen = 8;
    o->n_target = 1000;
    o->ngr = 32;
    o->key_bits = 0;
    o->list_per_node = 96.0f;
    o->auto_regrow = 1;
    o->keep_keys = 0;
    o->sort_max = 8192;
    o->period = 0.0f;
    o->reg_fmax = 0.0f;
}

jz_status jz_build(const float *points, int64_t n, void *stream, const jz_build_opts *opts,
                   const jz_allocator *alloc, jz_tree **out) {
    g_err.clear();
    const int64_t off[2] = {0, n < 0 ? 0 : n};
    return make_tree_impl(points, off, 1, n, stream, opts, alloc, out);
}

jz_status jz_forest_build(const float *points, const int64_t *offsets, int nsets, void *stream,
                          const jz_build_opts *opts, const jz_allocator *alloc, jz_tree **out) {
    g_err.clear();
    if (out) *out = nullptr;
    if (!offsets) return jz_fail(JZ_E_INVALID, "offsets is NULL");
    if (nsets < 1 || nsets > 65536) return jz_fail(JZ_E_INVALID, "nsets must be in [1, 65536]");
    if (offsets[0] != 0) return jz_fail(JZ_E_INVALID, "offsets[0] must be 0");
    for (int i = 0; i < nsets; ++i)
        if (offsets[i + 1] < offsets[i]) return jz_fail(JZ_E_INVALID, "offsets must be non-decreasing");
    return make_tree_impl(points, offsets, nsets, offsets[nsets], stream, opts, alloc, out);
}

jz_status jz_build_joint(const float *sources, int64_t n_src, const float *queries,
                         int64_t n_qry, void *stream, const jz_build_opts *opts,
                         const jz_allocator *alloc, jz_tree **out) {
    g_err.clear();
    if (out) *out = nullptr;
    if (!out) return jz_fail(JZ_E_INVALID, "out is NULL");
    if (n_src < 0 || n_qry < 0 || n_src + n_qry > (int64_t)INT32_MAX - 1)
        return jz_fail(JZ_E_INVALID, "n_src, n_qry must be >= 0 with n_src + n_qry <= 2^31-2");
    if ((n_src > 0 && !sources) || (n_qry > 0 && !queries))
        return jz_fail(JZ_E_INVALID, "points are NULL");
    if (alloc && (!alloc->alloc || !alloc->free))
        return jz_fail(JZ_E_INVALID, "allocator needs both alloc and free");
    if (opts && opts->period != 0.0f)
        return jz_fail(JZ_E_UNSUPPORTED, "a joint tree takes open space (period 0)");
    const int64_t n = n_src + n_qry;
    hipStream_t s = (hipStream_t)stream;
    AllocCtx ac;
    if (hipGetDevice(&ac.device) != hipSuccess) {
        (void)hipGetLastError();
        return jz_fail(JZ_E_DEVICE, "no HIP device");
    }
    if (alloc) {
        ac.user = true;
        ac.ua = *alloc;
    }
    // one array over both types: sources first, then queries
    DBuf cat;
    JZ_TRY(cat.get(&ac, (size_t)n * 3 * sizeof(float), s));
    if (n_src)
        JZ_HIP(hipMemcpyAsync(cat.p, sources, (size_t)n_src * 3 * sizeof(float),
                              hipMemcpyDeviceToDevice, s));
    if (n_qry)
        JZ_HIP(hipMemcpyAsync(cat.as<float>() + 3 * n_src, queries, (size_t)n_qry * 3 * sizeof(float),
                              hipMemcpyDeviceToDevice, s));
    const int64_t off[2] = {0, n};
    JZ_TRY(make_tree_impl(cat.as<float>(), off, 1, n, stream, opts, alloc, out));
    jz_tree *t = *out;
    t->n_src = n_src;
    jz_status st = n > 0 ? source_counts(t, s) : JZ_OK;
    if (st == JZ_OK) {
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = jz_hip_fail(e, "hipStreamSynchronize", __FILE__, __LINE__);
    }
    if (st != JZ_OK) {
        delete t;
        *out = nullptr;
    }
    return st;
}

jz_status jz_knn_query(jz_tree *t, int k, int32_t *idx, float *dist2, void *stream) {
    g_err.clear();
    if (!t) return jz_fail(JZ_E_INVALID, "tree is NULL");
    if (t->n_src < 0) return jz_fail(JZ_E_INVALID, "the tree has no query points (jz_build_joint)");
    if (k < 1) return jz_fail(JZ_E_INVALID, "k must be >= 1");
    if (k > JZ_MAX_K) return jz_fail(JZ_E_UNSUPPORTED, "k > %d is not supported", JZ_MAX_K);
    if (t->n > t->n_src && (!idx || !dist2)) return jz_fail(JZ_E_INVALID, "output is NULL");
    DeviceGuard g(t->ac.device);
    return run_knn(t, k, idx, dist2, (hipStream_t)stream);
}

jz_status jz_knn(jz_tree *t, int k, int32_t *idx, float *dist2, void *stream) {
    g_err.clear();
    if (!t) return jz_fail(JZ_E_INVALID, "tree is NULL");
    if (t->n_src >= 0) return jz_fail(JZ_E_INVALID, "a joint tree takes jz_knn_query");
    if (k < 1) return jz_fail(JZ_E_INVALID, "k must be >= 1");
    if (k > JZ_MAX_K) return jz_fail(JZ_E_UNSUPPORTED, "k > %d is not supported", JZ_MAX_K);
    if (t->n > 0 && (!idx || !dist2)) return jz_fail(JZ_E_INVALID, "output is NULL");
    DeviceGuard g(t->ac.device);
    return run_knn(t, k, idx, dist2, (hipStream_t)stream);
}

jz_status jz_fof(jz_tree *t, float b, int32_t *label, void *stream) {
    g_err.clear();
    if (!t) return jz_fail(JZ_E_INVALID, "tree is NULL");
    if (t->n_src >= 0) return jz_fail(JZ_E_INVALID, "FoF takes a tree from jz_build");
    if (!(b >= 0.0f) || !std::isfinite(b)) return jz_fail(JZ_E_INVALID, "b must be finite and >= 0");
    if (t->n > 0 && !label) return jz_fail(JZ_E_INVALID, "label is NULL");
    DeviceGuard g(t->ac.device);
    std::vector<float> b2(t->nsets, b * b);
    return run_fof(t, b2.data(), label, (hipStream_t)stream);
}

// kNN and FoF only read the tree and write disjoint outputs, so the FoF half
// runs from a second host thread on the library's side stream while this
// thread runs the kNN half on `stream`: each half keeps its own host-side
// rerun checks, and the walk levels of one, which fill few waves, overlap
// the other's work. Both halves start after the work queued on `stream` and
// `stream` waits for both.
jz_status jz_knn_fof(jz_tree *t, int k, int32_t *idx, float *dist2, float b, int32_t *label,
                     void *stream, jz_stats *knn_st, jz_stats *fof_st) {
    g_err.clear();
    if (!t) return jz_fail(JZ_E_INVALID, "tree is NULL");
    if (t->n_src >= 0) return jz_fail(JZ_E_INVALID, "jz_knn_fof takes a tree from jz_build");
    if (k < 1) return jz_fail(JZ_E_INVALID, "k must be >= 1");
    if (k > JZ_MAX_K) return jz_fail(JZ_E_UNSUPPORTED, "k > %d is not supported", JZ_MAX_K);
    if (!(b >= 0.0f) || !std::isfinite(b)) return jz_fail(JZ_E_INVALID, "b must be finite and >= 0");
    if (t->n > 0 && (!idx || !dist2 || !label)) return jz_fail(JZ_E_INVALID, "output is NULL");
    const int dev = t->ac.device;
    DeviceGuard g(dev);
    const hipStream_t s = (hipStream_t)stream;
    jz_status st = JZ_OK;
    const hipStream_t s2 = side_stream(dev, st);
    if (!s2) return st;
    EventGuard e_in, e_out;
    JZ_HIP(hipEventCreateWithFlags(&e_in.e, hipEventDisableTiming));
    JZ_HIP(hipEventCreateWithFlags(&e_out.e, hipEventDisableTiming));
    JZ_HIP(hipEventRecord(e_in.e, s));
    JZ_HIP(hipStreamWaitEvent(s2, e_in.e, 0));

    jz_stats fst = t->st;  // the tree's own fields; run_fof fills the call's
    const std::vector<float> b2(t->nsets, b * b);
    const bool prof = g_prof;
    jz_status f_status = JZ_OK;
    std::string f_msg;
    // (no exception may leave a thread: a failed host allocation becomes a status)
    auto fof_half = [&]() {
        g_prof = prof;  // (thread-local settings of the calling thread)
        DeviceGuard g2(dev);
        try {
            f_status = run_fof(t, b2.data(), label, s2, &fst);
        } catch (...) {
            f_status = jz_fail(JZ_E_OOM, "host allocation failed in the FoF half");
        }
        if (f_status != JZ_OK) f_msg = g_err;
    };
    std::thread th;
    bool threaded = true;
    try {
        th = std::thread(fof_half);
    } catch (...) {
        threaded = false;  // no thread to be had: the halves run one after the other
    }
    jz_status k_status;
    try {
        k_status = run_knn(t, k, idx, dist2, s);
    } catch (...) {
        k_status = jz_fail(JZ_E_OOM, "host allocation failed in the kNN half");
    }
    if (threaded) th.join();
    else fof_half();
    // `stream` waits for the FoF half whatever either half returned
    const hipError_t e1 = hipEventRecord(e_out.e, s2);
    const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(s, e_out.e, 0) : e1;
    if (knn_st) *knn_st = t->st;
    if (fof_st) *fof_st = fst;
    if (k_status != JZ_OK) return k_status;
    if (f_status != JZ_OK) return jz_fail(f_status, "%s", f_msg.c_str());
    if (e2 != hipSuccess) return jz_hip_fail(e2, "ordering the FoF half before later work", __FILE__, __LINE__);
    return JZ_OK;
}

jz_status jz_forest_fof(jz_tree *t, const float *b, int32_t *label, void *stream) {
    g_err.clear();
    if (!t) return jz_fail(JZ_E_INVALID, "tree is NULL");
    if (!b) return jz_fail(JZ_E_INVALID, "b is NULL");
    std::vector<float> b2(t->nsets);
    for (int i = 0; i < t->nsets; ++i) {
        if (!(b[i] >= 0.0f) || !std::isfinite(b[i]))
            return jz_fail(JZ_E_INVALID, "b[%d] must be finite and >= 0", i);
        b2[i] = b[i] * b[i];
    }
    if (t->n > 0 && !label) return jz_fail(JZ_E_INVALID, "label is NULL");
    DeviceGuard g(t->ac.device);
    return run_fof(t, b2.data(), label, (hipStream_t)stream);
}

void jz_tree_free(jz_tree *t) {
    if (!t) return;
    DeviceGuard g(t->ac.device);
    delete t;
}

int64_t jz_tree_size(const jz_tree *t) {
    if (!t) return 0;
    size_t b = t->d_set_off.bytes + t->pts4.bytes + t->keys.bytes + t->leaf_base.bytes +
               t->super_spl.bytes + t->knn_top_seg.bytes + t->knn_top_list.bytes +
               t->fof_top_seg.bytes + t->fof_top_list.bytes;
    for (int p = 0; p < JZ_MAX_PLANES; ++p)
        b += t->nodes[p].bytes + t->spl[p].bytes + t->node_set[p].bytes + t->src_cnt[p].bytes;
    return (int64_t)b;
}

jz_status jz_tree_stats(const jz_tree *t, jz_stats *s) {
    if (!t || !s) return jz_fail(JZ_E_INVALID, "NULL argument");
    *s = t->st;
    return JZ_OK;
}

void jz_set_profiling(int on) { g_prof = on != 0; }

jz_status jz_tree_export(const jz_tree *t, int32_t *order, uint64_t *keys, int plane,
                         int32_t *spl) {
    g_err.clear();
    if (!t) return jz_fail(JZ_E_INVALID, "tree is NULL");
    DeviceGuard g(t->ac.device);
    const int64_t n = t->n;
    if (order && n > 0) {
        std::vector<float> tmp(4 * n);
        JZ_HIP(hipMemcpy(tmp.data(), t->pts4.p, n * 4 * sizeof(float), hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < n; ++i) std::memcpy(order + i, &tmp[4 * i + 3], sizeof(int32_t));
    }
    if (keys && n > 0) {
        if (!t->keys.p) return jz_fail(JZ_E_INVALID, "tree was built without keep_keys");
        JZ_HIP(hipMemcpy(keys, t->keys.p, n * sizeof(uint64_t), hipMemcpyDeviceToHost));
    }
    if (spl) {
        if (plane < 0 || plane >= t->P) return jz_fail(JZ_E_INVALID, "plane out of range");
        JZ_HIP(hipMemcpy(spl, t->spl[plane].p, (t->L[plane] + 1) * sizeof(int32_t),
                         hipMemcpyDeviceToHost));
    }
    return JZ_OK;
}

void jz_release_cached(void) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    Pool &P = pool(dev);
    std::lock_guard<std::mutex> lk(P.m);
    release_all(P);
}

const char *jz_last_error(void) { return g_err.c_str(); }

int jz_abi_version(void) { return 4; }

}  // extern "C"
