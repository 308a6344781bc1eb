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
// Periodic cube [0, L)^3 (build option `period`): the minimum-image
// difference moves a coordinate difference by one period when it lies beyond
// half of it (h = fl(L / 2)), and dist2 is the fixed expression of the
// wrapped differences. PER = false is the open box above.

template <bool PER>
__device__ __forceinline__ float wrap_diff(float d, float L, float h) {
    if constexpr (PER) {
        d = d > h ? d - L : d;
        d = d < -h ? d + L : d;
    }
    return d;
}

template <bool PER>
__device__ __forceinline__ float dist2_m(float ax, float ay, float az, float bx, float by,
                                         float bz, float L, float h) {
    float dx = wrap_diff<PER>(ax - bx, L, h);
    float dy = wrap_diff<PER>(ay - by, L, h);
    float dz = wrap_diff<PER>(az - bz, L, h);
    float xx = dx * dx;
    float yy = dy * dy;
    float zz = dz * dz;
    float s = xx + yy;
    return s + zz;
}

// Periodic bounds are not exact like the open ones: a wrapped difference
// fl(fl(x - y) -+ L) may be off from the exact minimum-image difference by a
// few units in the last place of L. Per axis the gap is lowered (the extent
// raised) by 2^-21 L, and the sums get a relative margin of 2^-20, so the
// bounds still bracket every computed member distance.
__device__ __forceinline__ float per_gap(float dmin, float dmax, float L) {
    // smallest |d + mL| over d in [dmin, dmax], m in {-1, 0, 1}
    const float g0 = fmaxf(fmaxf(dmin, -dmax), 0.0f);
    const float g1 = fmaxf(fmaxf(dmin - L, L - dmax), 0.0f);
    const float g2 = fmaxf(fmaxf(dmin + L, -(dmax + L)), 0.0f);
    return fminf(g0, fminf(g1, g2));
}
__device__ __forceinline__ float per_low_sum(float gx, float gy, float gz, float L) {
    const float eps = L * 0x1p-21f;
    gx = fmaxf(gx - eps, 0.0f);
    gy = fmaxf(gy - eps, 0.0f);
    gz = fmaxf(gz - eps, 0.0f);
    const float xx = gx * gx, yy = gy * gy, zz = gz * gz;
    const float s = xx + yy;
    return (s + zz) * (1.0f - 0x1p-20f);
}
__device__ __forceinline__ float per_up_sum(float ux, float uy, float uz, float L) {
    const float eps = L * 0x1p-21f, h = 0.5f * L;
    ux = fminf(ux, h) + eps;
    uy = fminf(uy, h) + eps;
    uz = fminf(uz, h) + eps;
    const float xx = ux * ux, yy = uy * uy, zz = uz * uz;
    const float s = xx + yy;
    return (s + zz) * (1.0f + 0x1p-20f);
}

// node-node bounds in the chosen metric
template <bool PER>
__device__ __forceinline__ float box_low2_m(const Node &a, const Node &b, float L) {
    if constexpr (!PER) {
        return box_low2(a, b);
    } else {
        return per_low_sum(per_gap(a.lo[0] - b.hi[0], a.hi[0] - b.lo[0], L),
                           per_gap(a.lo[1] - b.hi[1], a.hi[1] - b.lo[1], L),
                           per_gap(a.lo[2] - b.hi[2], a.hi[2] - b.lo[2], L), L);
    }
}
template <bool PER>
__device__ __forceinline__ float box_up2_m(const Node &a, const Node &b, float L) {
    if constexpr (!PER) {
        return box_up2(a, b);
    } else {
        return per_up_sum(fmaxf(a.hi[0] - b.lo[0], b.hi[0] - a.lo[0]),
                          fmaxf(a.hi[1] - b.lo[1], b.hi[1] - a.lo[1]),
                          fmaxf(a.hi[2] - b.lo[2], b.hi[2] - a.lo[2]), L);
    }
}
// point-box lower bound in the chosen metric (box given by its corners)
template <bool PER>
__device__ __forceinline__ float point_low2_m(float qx, float qy, float qz, float lx, float ly,
                                              float lz, float hx, float hy, float hz, float L) {
    if constexpr (!PER) {
        const float gx = fmaxf(fmaxf(lx - qx, qx - hx), 0.0f);
        const float gy = fmaxf(fmaxf(ly - qy, qy - hy), 0.0f);
        const float gz = fmaxf(fmaxf(lz - qz, qz - hz), 0.0f);
        const float xx = gx * gx;
        const float yy = gy * gy;
        const float zz = gz * gz;
        const float s = xx + yy;
        return s + zz;
    } else {
        return per_low_sum(per_gap(qx - hx, qx - lx, L), per_gap(qy - hy, qy - ly, L),
                           per_gap(qz - hz, qz - lz, L), L);
    }
}

// ---------------------------------------------------------------------------
// Work-group and work-item indices read straight from the hardware registers
// and the dispatch packet. The device library's accessors behind blockIdx,
// threadIdx, gridDim and blockDim are not inlined into code built with a
// different IEEE mode (the leaf-stage files): there they become calls, each
// with a stack frame, and in the largest kernels the registers live across
// them spill to scratch memory.
__device__ __forceinline__ unsigned blk_x() { return __builtin_amdgcn_workgroup_id_x(); }
__device__ __forceinline__ unsigned tid_x() { return __builtin_amdgcn_workitem_id_x(); }
// dispatch packet: workgroup_size_x (16 bits) at byte 4, grid_size_x (work
// items, 32 bits) at byte 12
typedef const __attribute__((address_space(4))) uint16_t dispatch_u16;
typedef const __attribute__((address_space(4))) uint32_t dispatch_u32;
__device__ __forceinline__ unsigned bdim_x() {
    return ((dispatch_u16 *)__builtin_amdgcn_dispatch_ptr())[2];
}
__device__ __forceinline__ unsigned nblk_x() {
    const unsigned wg = ((dispatch_u16 *)__builtin_amdgcn_dispatch_ptr())[2];
    const unsigned gs = ((dispatch_u32 *)__builtin_amdgcn_dispatch_ptr())[3];
    return (gs + wg - 1) / wg;
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

// Cross-lane reductions without LDS round trips: DPP permutations inside
// each row of 16 lanes (xor 1, xor 2, the mirror inside 8 lanes and inside 16
// lanes pair every lane with a partner until the row is combined), then the
// gfx950 row swaps (lanes l and l ^ 16, then l and l ^ 32). Every lane ends
// with the reduction over the wave (or over the stated group). All lanes of
// the wave must be active.
constexpr int DPP_XOR1 = 0xB1;         // quad_perm [1, 0, 3, 2]
constexpr int DPP_XOR2 = 0x4E;         // quad_perm [2, 3, 0, 1]
constexpr int DPP_HALF_MIRROR = 0x141; // lane i <-> 7 - i inside each 8
constexpr int DPP_MIRROR = 0x140;      // lane i <-> 15 - i inside each 16
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
// the value of lane l ^ 16 (a) and of lane l ^ 32 (b)
__device__ __forceinline__ int swap16_i(int v) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (__lane_id() & 16) ? r[0] : r[1];
}
__device__ __forceinline__ int swap32_i(int v) {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (__lane_id() & 32) ? r[0] : r[1];
}
__device__ __forceinline__ float swap16_f(float v) { return __int_as_float(swap16_i(__float_as_int(v))); }
__device__ __forceinline__ double swap16_d(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint64_t lo = (uint32_t)swap16_i((int)(uint32_t)b), hi = (uint32_t)swap16_i((int)(b >> 32));
    return __builtin_bit_cast(double, (hi << 32) | lo);
}
__device__ __forceinline__ double swap32_d(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint64_t lo = (uint32_t)swap32_i((int)(uint32_t)b), hi = (uint32_t)swap32_i((int)(b >> 32));
    return __builtin_bit_cast(double, (hi << 32) | lo);
}
__device__ __forceinline__ float swap32_f(float v) { return __int_as_float(swap32_i(__float_as_int(v))); }

// reduction over each group of 8 lanes (lanes 8g .. 8g + 7)
__device__ __forceinline__ float group8_min(float v) {
    v = fminf(v, dpp_f<DPP_XOR1>(v));
    v = fminf(v, dpp_f<DPP_XOR2>(v));
    return fminf(v, dpp_f<DPP_HALF_MIRROR>(v));
}
__device__ __forceinline__ float group8_max(float v) {
    v = fmaxf(v, dpp_f<DPP_XOR1>(v));
    v = fmaxf(v, dpp_f<DPP_XOR2>(v));
    return fmaxf(v, dpp_f<DPP_HALF_MIRROR>(v));
}
// wave-wide reductions (result in every lane)
__device__ __forceinline__ int wave_max_i(int v) {
    v = max(v, dpp_i<DPP_XOR1>(v));
    v = max(v, dpp_i<DPP_XOR2>(v));
    v = max(v, dpp_i<DPP_HALF_MIRROR>(v));
    v = max(v, dpp_i<DPP_MIRROR>(v));
    v = max(v, swap16_i(v));
    return max(v, swap32_i(v));
}
__device__ __forceinline__ float wave_max_f(float v) {
    v = fmaxf(v, dpp_f<DPP_XOR1>(v));
    v = fmaxf(v, dpp_f<DPP_XOR2>(v));
    v = fmaxf(v, dpp_f<DPP_HALF_MIRROR>(v));
    v = fmaxf(v, dpp_f<DPP_MIRROR>(v));
    v = fmaxf(v, swap16_f(v));
    return fmaxf(v, swap32_f(v));
}
__device__ __forceinline__ int wave_min_i(int v) {
    v = min(v, dpp_i<DPP_XOR1>(v));
    v = min(v, dpp_i<DPP_XOR2>(v));
    v = min(v, dpp_i<DPP_HALF_MIRROR>(v));
    v = min(v, dpp_i<DPP_MIRROR>(v));
    v = min(v, swap16_i(v));
    return min(v, swap32_i(v));
}
// minimum over each aligned group of G lanes (G a power of 2, wave-uniform)
__device__ __forceinline__ float group_min_f(float v, int G) {
    if (G >= 2) v = fminf(v, dpp_f<DPP_XOR1>(v));
    if (G >= 4) v = fminf(v, dpp_f<DPP_XOR2>(v));
    if (G >= 8) v = fminf(v, dpp_f<DPP_HALF_MIRROR>(v));
    if (G >= 16) v = fminf(v, dpp_f<DPP_MIRROR>(v));
    if (G >= 32) v = fminf(v, swap16_f(v));
    if (G >= 64) v = fminf(v, swap32_f(v));
    return v;
}
__device__ __forceinline__ unsigned wave_or(unsigned v) {
    int x = (int)v;
    x |= dpp_i<DPP_XOR1>(x);
    x |= dpp_i<DPP_XOR2>(x);
    x |= dpp_i<DPP_HALF_MIRROR>(x);
    x |= dpp_i<DPP_MIRROR>(x);
    x |= swap16_i(x);
    x |= swap32_i(x);
    return (unsigned)x;
}
__device__ __forceinline__ int wave_sum_i(int v) {
    v += dpp_i<DPP_XOR1>(v);
    v += dpp_i<DPP_XOR2>(v);
    v += dpp_i<DPP_HALF_MIRROR>(v);
    v += dpp_i<DPP_MIRROR>(v);
    v += swap16_i(v);
    return v + swap32_i(v);
}

__device__ __forceinline__ float wave_max(float v) { return wave_max_f(v); }
__device__ __forceinline__ float wave_min(float v) { return group_min_f(v, 64); }
__device__ __forceinline__ int wave_max_int(int v) { return wave_max_i(v); }
__device__ __forceinline__ int wave_sum(int v) { return wave_sum_i(v); }

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

// The same operations with parent pointers read through this CU's and this
// XCD's caches (device-scope reads go past the per-XCD L2 to memory): a read
// may return an older value, never a wrong one, because a parent only ever
// moves to an ancestor. An older parent is still an ancestor, an older root
// is still a member of the group, and equal roots, however old, mean one
// group (groups only merge). Every write stays device-coherent: the
// path-halving store puts an ancestor (found from possibly older reads) into
// a node that is not a root, which only the halving itself ever rewrites, and
// the compare-and-swap on a root fails on a stale guess and returns the
// current parent, which is smaller, so union's retry loop ends (the larger of
// its two ids strictly decreases).
__device__ __forceinline__ int ld_cached(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ int uf_find_c(int *par, int x) {
    while (true) {
        int p = ld_cached(par + x);
        if (p == x) return x;
        int gp = ld_cached(par + p);
        if (gp == p) return p;
        st_rel(par + x, gp);
        x = gp;
    }
}
__device__ __forceinline__ void uf_union_c(int *par, int a, int b) {
    while (true) {
        a = uf_find_c(par, a);
        b = uf_find_c(par, b);
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
