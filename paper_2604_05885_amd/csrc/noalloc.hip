// jz_knn_noalloc: exact kNN on a built tree without any device allocation
// during the call. Its per-call scratch (walk counters, per-level segment
// tables and interaction lists, work items) is carved from `scratch`, a
// file-scope device array of JZ_NOALLOC_SCRATCH_BYTES that every GPU the
// library runs on holds until the process ends. The kernels are those of
// jz_knn; only where their scratch comes from differs.
#include <hip/hip_runtime.h>

#include <mutex>

#include "jz_internal.h"

namespace {

constexpr size_t kScratchBytes = JZ_NOALLOC_SCRATCH_BYTES;
constexpr size_t kAlign = 256;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Per device: the address of that device's copy of `scratch` (in host code
// the array's name is only a stand-in, never a device address), and a lock
// that serializes calls on the device (they share the array).
struct DeviceScratch {
    std::once_flag once;
    hipError_t err = hipSuccess;
    unsigned char *ptr = nullptr;
    std::mutex m;
};

DeviceScratch &device_scratch(int dev) {
    static DeviceScratch d[kMaxDevices];
    return d[dev];
}

// Hands out the region in stack order: a release of the most recent block
// returns its space, any other release is ignored until the call ends.
struct Bump {
    unsigned char *base = nullptr;
    size_t used = 0;
    size_t peak_need = 0;  // largest request that did not fit, for the message
    size_t stack[64];
    int depth = 0;
};

void *bump_alloc(void *ctx, size_t bytes, void *) {
    Bump *b = static_cast<Bump *>(ctx);
    const size_t start = (b->used + kAlign - 1) & ~(kAlign - 1);
    if (bytes > kScratchBytes || start > kScratchBytes - bytes || b->depth == 64) {
        if (start + bytes > b->peak_need) b->peak_need = start + bytes;
        return nullptr;
    }
    b->stack[b->depth++] = b->used;
    b->used = start + bytes;
    return b->base + start;
}

void bump_free(void *ctx, void *p, size_t bytes, void *) {
    Bump *b = static_cast<Bump *>(ctx);
    if (b->depth == 0) return;
    const size_t start = (size_t)(static_cast<unsigned char *>(p) - b->base);
    if (start + bytes == b->used) b->used = b->stack[--b->depth];
}

}  // namespace

extern "C" JZ_API jz_status jz_knn_noalloc(jz_tree *t, int k, int32_t *idx, float *dist2,
                                           void *stream) {
    if (!t) return jz_fail(JZ_E_INVALID, "tree is NULL");
    if (t->n_src >= 0) return jz_fail(JZ_E_INVALID, "a joint tree takes jz_knn_query");
    if (k < 1) return jz_fail(JZ_E_INVALID, "k must be >= 1");
    if (k > JZ_MAX_K) return jz_fail(JZ_E_UNSUPPORTED, "k > %d is not supported", JZ_MAX_K);
    if (t->n > 0 && (!idx || !dist2)) return jz_fail(JZ_E_INVALID, "output is NULL");
    const int dev = t->ac.device;
    if (dev < 0 || dev >= kMaxDevices) return jz_fail(JZ_E_INVALID, "device %d out of range", dev);
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) {
        (void)hipGetLastError();
        return jz_fail(JZ_E_DEVICE, "no HIP device");
    }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) {
        (void)hipGetLastError();
        return jz_fail(JZ_E_DEVICE, "cannot select device %d", dev);
    }
    DeviceScratch &ds = device_scratch(dev);
    // once per device, with that device current: the device address of its
    // copy of the array
    std::call_once(ds.once, [&] {
        ds.err = hipGetSymbolAddress(reinterpret_cast<void **>(&ds.ptr), HIP_SYMBOL(scratch));
        if (ds.err != hipSuccess) {
            (void)hipGetLastError();
            ds.ptr = nullptr;
        }
    });
    jz_status st;
    if (!ds.ptr) {
        st = jz_fail(JZ_E_DEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                     hipGetErrorString(ds.err));
    } else {
        std::lock_guard<std::mutex> lk(ds.m);
        Bump b;
        b.base = ds.ptr;
        AllocCtx ac;
        ac.device = dev;
        ac.user = true;
        ac.ua.ctx = &b;
        ac.ua.alloc = bump_alloc;
        ac.ua.free = bump_free;
        st = run_knn(t, k, idx, dist2, (hipStream_t)stream, &ac);
        if (st == JZ_E_OOM)
            st = jz_fail(JZ_E_CAPACITY,
                         "jz_knn_noalloc: this call needs more than the %zu bytes of the "
                         "library's fixed scratch (at least %zu); use jz_knn",
                         kScratchBytes, b.peak_need);
    }
    if (prev != dev) (void)hipSetDevice(prev);
    return st;
}
