// Autotuner (jz_autotune in include/jz.h): times candidate tree options on the
// caller's workload and remembers the fastest per workload signature, in the
// process and, when JZ_TUNE_CACHE names a file, in that file (one JSON object
// per line), so that later processes reuse it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "jz_internal.h"

namespace {

using Sig = std::tuple<std::string, int, int, int64_t, int>;  // arch, k, FoF, sets, log2 n
std::mutex g_tune_m;
std::map<Sig, std::pair<jz_build_opts, double>> g_tuned;

std::string device_arch(int dev) {
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    std::string a = pr.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

const char *cache_path() {
    const char *p = std::getenv("JZ_TUNE_CACHE");
    return p && *p ? p : nullptr;
}

// the cached entry for sig in the file, if any (the last matching line wins)
bool cache_lookup(const Sig &sig, const jz_build_opts &o0, jz_build_opts *o, double *ms) {
    const char *path = cache_path();
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char arch[32] = {0};
        int k = 0, fof = 0, lg = 0, leaf = 0, coarsen = 0, nt = 0, ngr = 0;
        long long sets = 0;
        double t = 0;
        if (std::sscanf(line,
                        "{\"arch\":\"%31[^\"]\",\"k\":%d,\"fof\":%d,\"sets\":%lld,\"log2n\":%d,"
                        "\"leaf_max\":%d,\"coarsen\":%d,\"n_target\":%d,\"ngr\":%d,\"ms\":%lf}",
                        arch, &k, &fof, &sets, &lg, &leaf, &coarsen, &nt, &ngr, &t) != 10)
            continue;
        if (Sig{arch, k, fof, (int64_t)sets, lg} != sig) continue;
        jz_build_opts c = o0;
        c.leaf_max = leaf;
        c.coarsen = coarsen;
        c.n_target = nt;
        c.ngr = ngr;
        if (check_opts(c) != JZ_OK) continue;
        *o = c;
        *ms = t;
        found = true;
    }
    std::fclose(f);
    return found;
}

void cache_store(const Sig &sig, const jz_build_opts &o, double ms) {
    const char *path = cache_path();
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    char line[512];
    std::snprintf(line, sizeof line,
                  "{\"arch\":\"%s\",\"k\":%d,\"fof\":%d,\"sets\":%lld,\"log2n\":%d,"
                  "\"leaf_max\":%d,\"coarsen\":%d,\"n_target\":%d,\"ngr\":%d,\"ms\":%.6f}\n",
                  std::get<0>(sig).c_str(), std::get<1>(sig), std::get<2>(sig),
                  (long long)std::get<3>(sig), std::get<4>(sig), o.leaf_max, o.coarsen, o.n_target,
                  o.ngr, ms);
    std::fputs(line, f);  // one write per line: appends from several processes do not interleave
    std::fclose(f);
}

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
    jz_build_opts o0;
    jz_default_opts(&o0);
    if (base) o0 = *base;
    JZ_TRY(check_opts(o0));
    int dev = 0;
    JZ_HIP(hipGetDevice(&dev));
    const Sig sig{device_arch(dev), k, b ? 1 : 0, (int64_t)sets,
                  n > 0 ? (int)std::floor(std::log2((double)n)) : 0};
    {
        std::lock_guard<std::mutex> lk(g_tune_m);
        auto it = g_tuned.find(sig);
        if (it == g_tuned.end()) {
            jz_build_opts c;
            double t = 0;
            if (cache_lookup(sig, o0, &c, &t)) it = g_tuned.emplace(sig, std::make_pair(c, t)).first;
        }
        if (it != g_tuned.end()) {
            *best = it->second.first;
            if (best_ms) *best_ms = it->second.second;
            return JZ_OK;
        }
    }
    hipStream_t s = (hipStream_t)stream;
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
    // best of two timed runs of each candidate
    auto try_opts = [&](const jz_build_opts &o) -> jz_status {
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
        return JZ_OK;
    };
    // leaf size x coarsening on a grid (a leaf is one wave of queries, so
    // at most 64 points), then the stop rule of the planes and the super-node
    // width around the best of those
    for (int leaf : {32, 48, 64}) {
        for (int c : {4, 8, 16}) {
            jz_build_opts o = o0;
            o.leaf_max = leaf;
            o.coarsen = c;
            JZ_TRY(try_opts(o));
        }
    }
    const jz_build_opts grid_best = bo;
    for (int nt : {500, 2000}) {
        jz_build_opts o = grid_best;
        o.n_target = nt;
        JZ_TRY(try_opts(o));
    }
    const jz_build_opts nt_best = bo;
    for (int g : {16, 64}) {
        jz_build_opts o = nt_best;
        o.ngr = g;
        JZ_TRY(try_opts(o));
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_m);
        g_tuned[sig] = {bo, bestt};
        cache_store(sig, bo, bestt);
    }
    *best = bo;
    if (best_ms) *best_ms = bestt;
    return JZ_OK;
}
