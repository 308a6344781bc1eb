// Autotuner (jz_autotune in include/jz.h): times candidate tree options on the
// caller's workload and remembers the fastest per workload signature.
#include <hip/hip_runtime.h>

#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "jz_internal.h"

namespace {

using Sig = std::tuple<int, int, int64_t, int>;  // k, FoF, sets, log2 n
std::mutex g_tune_m;
std::map<Sig, std::pair<jz_build_opts, double>> g_tuned;

// one timed run: build + kNN and/or FoF; returns device time in ms
jz_status time_once(const float *points, const std::vector<int64_t> &off, int k,
                    const std::vector<float> &b2, hipStream_t s, const jz_build_opts &o,
                    int32_t *idx, float *d2, int32_t *lab, double *ms) {
    hipEvent_t e0, e1;
    JZ_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return jz_fail(JZ_E_DEVICE, "hipEventCreate failed");
    }
    jz_status st = hipEventRecord(e0, s) == hipSuccess ? JZ_OK : JZ_E_DEVICE;
    jz_tree *t = nullptr;
    if (st == JZ_OK) st = tree_create(points, off.data(), (int)off.size() - 1, s, &o, nullptr, &t);
    if (st == JZ_OK && k > 0) st = run_knn(t, k, idx, d2, s);
    if (st == JZ_OK && !b2.empty()) st = run_fof(t, b2.data(), lab, s);
    delete t;
    if (st == JZ_OK && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess) {
        float f = 0;
        (void)hipEventElapsedTime(&f, e0, e1);
        *ms = f;
    } else if (st == JZ_OK) {
        st = jz_fail(JZ_E_DEVICE, "event timing failed");
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

}  // namespace

extern "C" jz_status jz_autotune(const float *points, const int64_t *offsets, int64_t nsets,
                                 int k, const float *b, void *stream, const jz_build_opts *base,
                                 jz_build_opts *best, double *best_ms) {
    if (!best) return jz_fail(JZ_E_INVALID, "best is NULL");
    if (k < 0 || k > JZ_MAX_K) return jz_fail(JZ_E_INVALID, "k must be in [0, %d]", JZ_MAX_K);
    if (k == 0 && !b) return jz_fail(JZ_E_INVALID, "nothing to tune (k = 0 and b = NULL)");
    std::vector<int64_t> off;
    if (offsets) {
        if (nsets < 1 || nsets > 65536) return jz_fail(JZ_E_INVALID, "nsets must be in [1, 65536]");
        off.assign(offsets, offsets + nsets + 1);
        if (off[0] != 0) return jz_fail(JZ_E_INVALID, "offsets[0] must be 0");
        for (int64_t i = 0; i < nsets; ++i)
            if (off[i + 1] < off[i]) return jz_fail(JZ_E_INVALID, "offsets must be non-decreasing");
    } else {
        if (nsets < 0) return jz_fail(JZ_E_INVALID, "n must be >= 0");
        off = {0, nsets};
    }
    const int64_t n = off.back();
    if (n < 0 || n > (int64_t)INT32_MAX - 1) return jz_fail(JZ_E_INVALID, "n out of range");
    if (n > 0 && !points) return jz_fail(JZ_E_INVALID, "points is NULL");
    const int sets = (int)off.size() - 1;
    std::vector<float> b2;
    if (b) {
        b2.resize(sets);
        for (int i = 0; i < sets; ++i) {
            if (!(b[i] >= 0.0f) || !std::isfinite(b[i]))
                return jz_fail(JZ_E_INVALID, "b[%d] must be finite and >= 0", i);
            b2[i] = b[i] * b[i];
        }
    }
    const Sig sig{k, b ? 1 : 0, (int64_t)sets, n > 0 ? (int)std::floor(std::log2((double)n)) : 0};
    {
        std::lock_guard<std::mutex> lk(g_tune_m);
        auto it = g_tuned.find(sig);
        if (it != g_tuned.end()) {
            *best = it->second.first;
            if (best_ms) *best_ms = it->second.second;
            return JZ_OK;
        }
    }
    jz_build_opts o0;
    jz_default_opts(&o0);
    if (base) o0 = *base;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    JZ_HIP(hipGetDevice(&dev));
    AllocCtx ac;
    ac.device = dev;
    DBuf oi, od, ol;
    if (k > 0) {
        JZ_TRY(oi.get(&ac, (size_t)n * k * sizeof(int32_t), s));
        JZ_TRY(od.get(&ac, (size_t)n * k * sizeof(float), s));
    }
    if (b) JZ_TRY(ol.get(&ac, (size_t)n * sizeof(int32_t), s));
    double bestt = INFINITY;
    jz_build_opts bo = o0;
    for (int leaf : {32, 48, 64}) {
        for (int c : {4, 8}) {
            jz_build_opts o = o0;
            o.leaf_max = leaf;
            o.coarsen = c;
            double tmin = INFINITY;
            for (int rep = 0; rep < 2; ++rep) {
                double ms = 0;
                JZ_TRY(time_once(points, off, k, b2, s, o, oi.as<int32_t>(), od.as<float>(),
                                 ol.as<int32_t>(), &ms));
                tmin = std::min(tmin, ms);
            }
            if (tmin < bestt) {
                bestt = tmin;
                bo = o;
            }
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_m);
        g_tuned[sig] = {bo, bestt};
    }
    *best = bo;
    if (best_ms) *best_ms = bestt;
    return JZ_OK;
}
