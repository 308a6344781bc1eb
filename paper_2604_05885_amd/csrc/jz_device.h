// Device helpers for the gfx950 kernels: node records, rigorous float32
// distance bounds, wave64 primitives, union-find and launch mapping.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define JZ_WAVE 64

// One tree node (32 bytes): tight bounding box of its points, the first point
// (z-order position) and the number of points.
struct __align__(16) Node {
    float lo[3];
    int start;
    float hi[3];
    int count;
};

// ---------------------------------------------------------------------------
// Fixed float32 distance. Built with -ffp-contract=off: no FMA contraction.

__device__ __forceinline__ float dist2_pts(float ax, float ay, float az, float bx, float by,
                                           float bz) {
    float dx = ax - bx;
    float dy = ay - by;
    float dz = az - bz;
    float xx = dx * dx;
    float yy = dy * dy;
    float zz = dz * dz;
    float s = xx + yy;
    return s + zz;
}

// Node-node bounds (paper Eq. 14-16, here on tight member boxes instead of
// Morton cells). Every operation is correctly rounded and monotone on
// non-negative values, so for any member pair (p in a, q in b) the computed
// dist2_pts(p, q) lies in [box_low2(a, b), box_up2(a, b)] exactly.
__device__ __forceinline__ float box_low2(const Node &a, const Node &b) {
    float gx = fmaxf(fmaxf(a.lo[0] - b.hi[0], b.lo[0] - a.hi[0]), 0.0f);
    float gy = fmaxf(fmaxf(a.lo[1] - b.hi[1], b.lo[1] - a.hi[1]), 0.0f);
    float gz = fmaxf(fmaxf(a.lo[2] - b.hi[2], b.lo[2] - a.hi[2]), 0.0f);
    float xx = gx * gx;
    float yy = gy * gy;
    float zz = gz * gz;
    float s = xx + yy;
    return s + zz;
}

__device__ __forceinline__ float box_up2(const Node &a, const Node &b) {
    float ux = fmaxf(a.hi[0] - b.lo[0], b.hi[0] - a.lo[0]);
    float uy = fmaxf(a.hi[1] - b.lo[1], b.hi[1] - a.lo[1]);
    float uz = fmaxf(a.hi[2] - b.lo[2], b.hi[2] - a.lo[2]);
    float xx = ux * ux;
    float yy = uy * uy;
    float zz = uz * uz;
    float s = xx + yy;
    return s + zz;
}

// ---------------------------------------------------------------------------
// wave64 primitives

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    return (lane_id() == 0) ? 0ull : (~0ull >> (64 - lane_id()));
}

// A value that every active lane of the wave holds, moved to a scalar
// register. The compiler cannot tell that values read from LDS, reduced with
// shuffles or derived from threadIdx.x / 64 are wave-uniform; marking them
// gives scalar loop control, scalar loads and fewer vector instructions.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ unsigned uni(unsigned v) {
    return (unsigned)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ unsigned long long uni(unsigned long long v) {
    const unsigned lo = uni((unsigned)v), hi = uni((unsigned)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ float uni(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// inclusive prefix sum over the 64 lanes
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(v, o, 64);
        if (l >= o) v += t;
    }
    return v;
}

// Order LDS traffic of one wave: everything written before is visible to the
// wave's later reads (the wave's lanes run in lockstep; the fence makes the
// compiler wait for outstanding LDS operations and keeps them in order).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// coherent (L2) loads/stores for data other waves update concurrently

__device__ __forceinline__ int ld_acq(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_rel(int *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Lock-free union-find over z-order point indices (paper, FoF section: link
// the higher root to the lower one with compare-and-swap, retry on failure).
// Invariant: par[x] <= x, so the forest has no cycles and a root is the
// smallest z-index of its group.

__device__ __forceinline__ int uf_find(int *par, int x) {
    while (true) {
        int p = ld_acq(par + x);
        if (p == x) return x;
        int gp = ld_acq(par + p);
        if (gp == p) return p;
        st_rel(par + x, gp);  // path halving: gp is an ancestor of x
        x = gp;
    }
}

__device__ __forceinline__ void uf_union(int *par, int a, int b) {
    while (true) {
        a = uf_find(par, a);
        b = uf_find(par, b);
        if (a == b) return;
        if (a > b) {
            int t = a;
            a = b;
            b = t;
        }
        int old = atomicCAS(par + b, b, a);
        if (old == b) return;
        b = old;
    }
}

// ---------------------------------------------------------------------------
// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2). Remap so that each XCD works on runs of XCD_RUN consecutive
// workgroups, the runs dealt to the XCDs in turn: neighbouring z-order nodes
// (which share source data) stay in the same L2, while the cost of dense and
// sparse regions spreads evenly over the XCDs (one contiguous range per XCD
// leaves the XCD with the densest range finishing last). Workgroups past the
// last complete round of runs take one contiguous range per XCD.
// Kernels that give each work item one wave run WPB waves per workgroup. A
// workgroup keeps its registers and LDS until its slowest wave ends, so with
// waves of uneven cost one wave per workgroup keeps the most waves resident.
constexpr int WPB = 1;
constexpr int XCD_RUN = 16 / WPB;
__device__ __forceinline__ int xcd_block(int bid, int nblocks) {
    constexpr int per = 8 * XCD_RUN;
    const int full = nblocks / per;
    const int x = bid & 7;
    if (bid < full * per) {
        const int i = bid >> 3;
        return ((i / XCD_RUN) * 8 + x) * XCD_RUN + (i % XCD_RUN);
    }
    const int b = (bid - full * per) >> 3, n = nblocks - full * per;
    const int q = n >> 3, r = n & 7;
    return full * per + x * q + (x < r ? x : r) + b;
}

__device__ __forceinline__ unsigned bitlen64(uint64_t v) { return v ? 64u - __clzll(v) : 0u; }
__device__ __forceinline__ unsigned bitlen32(uint32_t v) { return v ? 32u - __clz(v) : 0u; }
