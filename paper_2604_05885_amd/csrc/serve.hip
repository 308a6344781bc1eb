// Continuous-batching request loop (jz_server_* in include/jz.h).
//
// Submitted requests wait in one FIFO queue. Each worker thread owns a HIP
// stream; when free it takes the oldest request that fits the free part of
// the device-memory budget and every later pending request of the same kind
// (op, k) while the budget and the batch caps allow, solves them as one
// forest (one sort, one launch per stage for all of them), copies each result
// to its request's buffers, and marks the requests done with a completion
// time. The oldest request may be passed over by later, smaller ones at most
// MAX_BYPASS times; then the workers wait until it fits. Requests arriving during a
// batch join the next batch a worker forms, and batches of different workers
// overlap on the device. Sets in a forest never interact and every result is
// exact, so a request's result does not depend on the batch it ran in.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "jz_internal.h"

namespace {

int64_t steady_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Req {
    uint64_t ticket = 0;
    jz_request r{};
    hipEvent_t ready = nullptr;  // recorded on the caller's stream at submission
    size_t bytes = 0;
    bool done = false;
    jz_status status = JZ_OK;
    std::string msg;  // the worker's error message when status != JZ_OK
    int64_t t_done = 0;
    int bypassed = 0;  // batches started ahead of it while it was the oldest
};

constexpr int MAX_BYPASS = 8;     // times the oldest request may be passed over
constexpr int ADMIT_WINDOW = 64;  // pending requests looked at for one that fits

// Device bytes a request adds to a batch (an upper estimate): the tree build
// (input copy, keys and values twice, sorted float4 copy, planes) about 150 B
// per point, the interaction lists about 60 B per point, and the batch's
// output staging (8k B per point for kNN, 4 B for FoF labels).
size_t footprint(const jz_request &r) {
    const double n = (double)r.n;
    double b = 150.0 * n + 60.0 * n + (double)(1 << 20);
    b += r.op == JZ_OP_KNN ? 8.0 * r.k * n : 4.0 * n;
    return (size_t)b;
}

jz_status check_request(const jz_request *r) {
    if (!r) return jz_fail(JZ_E_INVALID, "request is NULL");
    if (r->n < 0 || r->n > (int64_t)INT32_MAX - 1)
        return jz_fail(JZ_E_INVALID, "n must be in [0, 2^31-2]");
    if (r->op == JZ_OP_KNN) {
        if (r->k < 1) return jz_fail(JZ_E_INVALID, "k must be >= 1");
        if (r->k > JZ_MAX_K) return jz_fail(JZ_E_UNSUPPORTED, "k > %d is not supported", JZ_MAX_K);
        if (r->n > 0 && (!r->idx || !r->dist2)) return jz_fail(JZ_E_INVALID, "kNN outputs are NULL");
    } else if (r->op == JZ_OP_FOF) {
        if (!(r->b >= 0.0f) || !std::isfinite(r->b))
            return jz_fail(JZ_E_INVALID, "b must be finite and >= 0");
        if (r->n > 0 && !r->label) return jz_fail(JZ_E_INVALID, "FoF output is NULL");
    } else {
        return jz_fail(JZ_E_INVALID, "unknown op");
    }
    if (r->n > 0 && !r->points) return jz_fail(JZ_E_INVALID, "points is NULL");
    return JZ_OK;
}

}  // namespace

struct jz_server {
    jz_server_opts o{};
    int device = 0;
    std::mutex m;
    std::condition_variable cv_work, cv_done;
    std::deque<Req *> pending;
    std::unordered_map<uint64_t, Req *> reqs;
    uint64_t next_ticket = 1;
    size_t in_use = 0;
    bool stop = false;
    std::vector<std::thread> workers;
    jz_serve_stats st{};
};

namespace {

// Solve one batch on stream s. All requests have the same op (and k).
jz_status run_batch(jz_server *S, const std::vector<Req *> &batch, hipStream_t s) {
    const int nsets = (int)batch.size();
    const jz_request &h = batch[0]->r;
    AllocCtx ac;
    ac.device = S->device;
    std::vector<int64_t> off(nsets + 1, 0);
    for (int i = 0; i < nsets; ++i) off[i + 1] = off[i] + batch[i]->r.n;
    const int64_t n = off[nsets];
    const bool single = nsets == 1;
    // the caller's work on its stream up to each submission (writes of the
    // points, or the copy that made them contiguous) comes first
    for (Req *q : batch)
        if (q->ready) JZ_HIP(hipStreamWaitEvent(s, q->ready, 0));
    // inputs: a single request is used in place, a batch is concatenated
    DBuf pts;
    const float *p = h.points;
    if (!single) {
        JZ_TRY(pts.get(&ac, (size_t)n * 3 * sizeof(float), s));
        for (int i = 0; i < nsets; ++i)
            if (batch[i]->r.n)
                JZ_HIP(hipMemcpyAsync(pts.as<float>() + 3 * off[i], batch[i]->r.points,
                                      batch[i]->r.n * 3 * sizeof(float), hipMemcpyDeviceToDevice, s));
        p = pts.as<float>();
    }
    jz_tree *t = nullptr;
    JZ_TRY(tree_create(p, off.data(), nsets, s, &S->o.build, nullptr, &t));
    jz_status st = JZ_OK;
    if (h.op == JZ_OP_KNN) {
        const int k = h.k;
        DBuf oi, od;
        int32_t *idx = h.idx;
        float *d2 = h.dist2;
        if (!single) {
            st = oi.get(&ac, (size_t)n * k * sizeof(int32_t), s);
            if (st == JZ_OK) st = od.get(&ac, (size_t)n * k * sizeof(float), s);
            idx = oi.as<int32_t>();
            d2 = od.as<float>();
        }
        if (st == JZ_OK) st = run_knn(t, k, idx, d2, s);
        if (st == JZ_OK && !single) {
            for (int i = 0; i < nsets && st == JZ_OK; ++i) {
                const size_t rows = (size_t)batch[i]->r.n * k;
                if (!rows) continue;
                hipError_t e = hipMemcpyAsync(batch[i]->r.idx, idx + off[i] * k,
                                              rows * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(batch[i]->r.dist2, d2 + off[i] * k, rows * sizeof(float),
                                       hipMemcpyDeviceToDevice, s);
                if (e != hipSuccess) st = jz_hip_fail(e, "hipMemcpyAsync(kNN result)", __FILE__, __LINE__);
            }
        }
    } else {
        std::vector<float> b2(nsets);
        for (int i = 0; i < nsets; ++i) b2[i] = batch[i]->r.b * batch[i]->r.b;
        DBuf lab;
        int32_t *label = h.label;
        if (!single) {
            st = lab.get(&ac, (size_t)n * sizeof(int32_t), s);
            label = lab.as<int32_t>();
        }
        if (st == JZ_OK) st = run_fof(t, b2.data(), label, s);
        if (st == JZ_OK && !single) {
            for (int i = 0; i < nsets && st == JZ_OK; ++i) {
                if (!batch[i]->r.n) continue;
                hipError_t e = hipMemcpyAsync(batch[i]->r.label, label + off[i],
                                              batch[i]->r.n * sizeof(int32_t),
                                              hipMemcpyDeviceToDevice, s);
                if (e != hipSuccess) st = jz_hip_fail(e, "hipMemcpyAsync(FoF result)", __FILE__, __LINE__);
            }
        }
    }
    if (st == JZ_OK) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = jz_hip_fail(e, "hipStreamSynchronize", __FILE__, __LINE__);
    } else {
        (void)hipStreamSynchronize(s);
    }
    delete t;
    return st;
}

// The request a new batch starts from: the oldest that fits the free budget
// (within the first ADMIT_WINDOW), unless the oldest has been passed over
// MAX_BYPASS times already; nullptr if none may start now.
Req *first_fit(const jz_server *S) {
    if (S->pending.empty()) return nullptr;
    const size_t avail = S->o.hbm_budget - S->in_use;
    Req *head = S->pending.front();
    if (head->bytes <= avail) return head;
    if (head->bypassed >= MAX_BYPASS) return nullptr;
    int scanned = 0;
    for (Req *q : S->pending) {
        if (++scanned > ADMIT_WINDOW) break;
        if (q->bytes <= avail) return q;
    }
    return nullptr;
}

bool can_start(const jz_server *S) { return first_fit(S) != nullptr; }

void worker(jz_server *S) {
    (void)hipSetDevice(S->device);
    hipStream_t stream = nullptr;
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        stream = nullptr;
    }
    std::unique_lock<std::mutex> lk(S->m);
    for (;;) {
        S->cv_work.wait(lk, [&] { return can_start(S) || (S->stop && S->pending.empty()); });
        if (S->pending.empty()) break;  // stopping and drained
        // the oldest request that fits and the later ones of the same kind
        // that fit too
        std::vector<Req *> batch;
        const Req *head = first_fit(S);
        if (head != S->pending.front()) S->pending.front()->bypassed++;
        const size_t avail = S->o.hbm_budget - S->in_use;
        size_t bytes = 0;
        int64_t pts = 0;
        int scanned = 0;
        for (auto it = S->pending.begin(); it != S->pending.end() && scanned < 65536; ++scanned) {
            Req *q = *it;
            const bool same = q->r.op == head->r.op && (q->r.op != JZ_OP_KNN || q->r.k == head->r.k);
            if (same && bytes + q->bytes <= avail &&
                (batch.empty() || pts + q->r.n <= S->o.max_batch_points)) {
                batch.push_back(q);
                bytes += q->bytes;
                pts += q->r.n;
                it = S->pending.erase(it);
                if ((int)batch.size() >= S->o.max_batch_sets) break;
            } else {
                ++it;
            }
        }
        S->in_use += bytes;
        S->st.pending = (int64_t)S->pending.size();
        S->st.in_flight_bytes = (int64_t)S->in_use;
        S->st.batches++;
        if ((int64_t)batch.size() > S->st.max_batch_sets_seen)
            S->st.max_batch_sets_seen = (int64_t)batch.size();
        lk.unlock();
        const jz_status rs = stream ? run_batch(S, batch, stream)
                                    : jz_fail(JZ_E_DEVICE, "no HIP stream for this worker");
        const std::string err = rs == JZ_OK ? std::string() : std::string(jz_last_error());
        lk.lock();
        S->in_use -= bytes;
        S->st.in_flight_bytes = (int64_t)S->in_use;
        const int64_t t = steady_ns();
        for (Req *q : batch) {
            q->done = true;
            q->status = rs;
            q->msg = err;
            q->t_done = t;
            if (rs == JZ_OK) {
                S->st.completed++;
                S->st.points_done += q->r.n;
            } else {
                S->st.failed++;
            }
        }
        S->cv_done.notify_all();
        S->cv_work.notify_all();
    }
    lk.unlock();
    if (stream) {
        (void)hipStreamSynchronize(stream);
        pool_forget_stream(S->device, stream);
        (void)hipStreamDestroy(stream);
        (void)hipGetLastError();
    }
}

}  // namespace

extern "C" {

void jz_server_default_opts(jz_server_opts *o) {
    if (!o) return;
    o->hbm_budget = (size_t)200e9;
    o->streams = 4;
    o->max_batch_points = (int64_t)1 << 26;
    o->max_batch_sets = 4096;
    jz_default_opts(&o->build);
}

int64_t jz_now_ns(void) { return steady_ns(); }

jz_status jz_server_create(const jz_server_opts *opts, jz_server **out) {
    if (!out) return jz_fail(JZ_E_INVALID, "out is NULL");
    *out = nullptr;
    jz_server_opts o;
    jz_server_default_opts(&o);
    if (opts) o = *opts;
    if (o.streams < 1 || o.streams > 16) return jz_fail(JZ_E_INVALID, "streams must be in [1, 16]");
    if (o.max_batch_sets < 1 || o.max_batch_sets > 65536)
        return jz_fail(JZ_E_INVALID, "max_batch_sets must be in [1, 65536]");
    if (o.max_batch_points < 1) return jz_fail(JZ_E_INVALID, "max_batch_points must be >= 1");
    if (o.hbm_budget == 0) return jz_fail(JZ_E_INVALID, "hbm_budget must be > 0");
    int dev = 0;
    const hipError_t de = hipGetDevice(&dev);
    if (de != hipSuccess) {
        (void)hipGetLastError();
        return jz_fail(JZ_E_DEVICE, "no HIP device (hipGetDevice: %s)", hipGetErrorString(de));
    }
    jz_server *S = new (std::nothrow) jz_server();
    if (!S) return jz_fail(JZ_E_OOM, "host allocation failed");
    S->o = o;
    S->device = dev;
    for (int i = 0; i < o.streams; ++i) S->workers.emplace_back(worker, S);
    *out = S;
    return JZ_OK;
}

jz_status jz_server_submit(jz_server *S, const jz_request *r, uint64_t *ticket) {
    if (!S) return jz_fail(JZ_E_INVALID, "server is NULL");
    JZ_TRY(check_request(r));
    const size_t bytes = footprint(*r);
    if (bytes > S->o.hbm_budget)
        return jz_fail(JZ_E_OOM, "request needs about %zu bytes, more than the budget %zu", bytes,
                       S->o.hbm_budget);
    Req *q = new (std::nothrow) Req();
    if (!q) return jz_fail(JZ_E_OOM, "host allocation failed");
    q->r = *r;
    q->bytes = bytes;
    if (r->n > 0) {
        hipError_t e = hipEventCreateWithFlags(&q->ready, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(q->ready, (hipStream_t)r->stream);
        if (e != hipSuccess) {
            if (q->ready) (void)hipEventDestroy(q->ready);
            delete q;
            return jz_hip_fail(e, "recording the submission event", __FILE__, __LINE__);
        }
    }
    std::lock_guard<std::mutex> lk(S->m);
    if (S->stop) {
        if (q->ready) (void)hipEventDestroy(q->ready);
        delete q;
        return jz_fail(JZ_E_INVALID, "server is stopping");
    }
    q->ticket = S->next_ticket++;
    S->reqs[q->ticket] = q;
    S->st.submitted++;
    if (r->n == 0) {
        q->done = true;
        q->t_done = steady_ns();
        S->st.completed++;
    } else {
        S->pending.push_back(q);
        S->st.pending = (int64_t)S->pending.size();
        S->cv_work.notify_one();
    }
    if (ticket) *ticket = q->ticket;
    return JZ_OK;
}

jz_status jz_server_poll(jz_server *S, uint64_t ticket, int *done, jz_status *result,
                         int64_t *done_ns) {
    if (!S) return jz_fail(JZ_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(S->m);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return jz_fail(JZ_E_INVALID, "unknown ticket");
    const Req *q = it->second;
    if (done) *done = q->done ? 1 : 0;
    if (q->done) {
        if (result) *result = q->status;
        if (done_ns) *done_ns = q->t_done;
        // the failed request's message becomes this thread's last error
        if (q->status != JZ_OK) (void)jz_fail(q->status, "%s", q->msg.c_str());
    }
    return JZ_OK;
}

jz_status jz_server_wait(jz_server *S, uint64_t ticket, jz_status *result, int64_t *done_ns) {
    if (!S) return jz_fail(JZ_E_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(S->m);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return jz_fail(JZ_E_INVALID, "unknown ticket");
    Req *q = it->second;
    S->cv_done.wait(lk, [&] { return q->done; });
    if (result) *result = q->status;
    if (q->status != JZ_OK) (void)jz_fail(q->status, "%s", q->msg.c_str());
    if (done_ns) *done_ns = q->t_done;
    return JZ_OK;
}

jz_status jz_server_release(jz_server *S, uint64_t ticket) {
    if (!S) return jz_fail(JZ_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(S->m);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return jz_fail(JZ_E_INVALID, "unknown ticket");
    if (!it->second->done) return jz_fail(JZ_E_INVALID, "request is not done");
    if (it->second->ready) (void)hipEventDestroy(it->second->ready);
    delete it->second;
    S->reqs.erase(it);
    return JZ_OK;
}

jz_status jz_server_stats(jz_server *S, jz_serve_stats *st) {
    if (!S || !st) return jz_fail(JZ_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(S->m);
    *st = S->st;
    st->pending = (int64_t)S->pending.size();
    return JZ_OK;
}

void jz_server_destroy(jz_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->m);
        S->stop = true;
    }
    S->cv_work.notify_all();
    for (auto &th : S->workers) th.join();
    for (auto &kv : S->reqs) {
        if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
        delete kv.second;
    }
    delete S;
}

}  // extern "C"
