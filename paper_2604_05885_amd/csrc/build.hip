// Tree construction on gfx950 (paper: section "Z-order trees").
//
//  1. bounding box + finiteness check
//  2. Morton keys (21 bits per dimension, dimension 0 most significant in
//     each bit triple; set id above them for forests) fused with the digit
//     histograms of every radix pass
//  3. stable LSD radix sort of (key, input index), one kernel per 8-bit digit
//     with decoupled look-back across tiles (one read + one write per pass)
//  4. gather of the sorted points into float4 (x, y, z, input index)
//  5. leaf plane: gap levels (Eq. 7 on keys) and the windowed test
//     n > N_max^(0) over +-N_max^(0) neighbouring gaps, compacted in order
//  6. exact node sizes n at the leaf splits by galloping binary search
//     (the left/right search of the plane-hierarchy section)
//  7. coarser planes: keep the splits with n > N_max^(p) (Eq. 8)
//  8. node geometry: tight member boxes, first point, count
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

#include "jz_device.h"
#include "jz_internal.h"

namespace {

constexpr int kSentinelLevel = 255;
constexpr int kBoundaryLevel = 254;

// float <-> order-preserving int for atomic min/max
__device__ __forceinline__ int f2o(float f) {
    int i = __float_as_int(f);
    return i >= 0 ? i : i ^ 0x7FFFFFFF;
}
__device__ __forceinline__ float o2f(int i) { return __int_as_float(i >= 0 ? i : i ^ 0x7FFFFFFF); }

// bbox[0..2] = min (ordered int), bbox[3..5] = max, bbox[6] = non-finite flag
__global__ __launch_bounds__(256) void k_bbox(const float *__restrict__ pts, int64_t n,
                                              int *__restrict__ bbox) {
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float v = pts[3 * i + a];
            bad |= !isfinite(v);
            lo[a] = fminf(lo[a], v);
            hi[a] = fmaxf(hi[a], v);
        }
    }
    // one atomic per block and value (same-address atomics serialize in L2)
    __shared__ float s_v[4][7];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = wave_min(lo[a]);
        hi[a] = wave_max(hi[a]);
    }
    bad = wave_sum(bad);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) {
        s_v[w][0] = lo[0]; s_v[w][1] = lo[1]; s_v[w][2] = lo[2];
        s_v[w][3] = hi[0]; s_v[w][4] = hi[1]; s_v[w][5] = hi[2];
        s_v[w][6] = bad ? 1.0f : 0.0f;
    }
    __syncthreads();
    if (threadIdx.x < 7) {
        const int a = threadIdx.x;
        float v = s_v[0][a];
        for (int ww = 1; ww < 4; ++ww) v = a < 3 ? fminf(v, s_v[ww][a]) : fmaxf(v, s_v[ww][a]);
        if (a < 3) atomicMin(bbox + a, f2o(v));
        else if (a < 6) atomicMax(bbox + a, f2o(v));
        else if (v != 0.0f) atomicOr(bbox + 6, 1);
    }
}

__device__ __forceinline__ uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1fffffull;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}

constexpr int kMaxPass = 8;

// Morton key + input index, and the digit histograms of all radix passes.
// Quantization per dimension: q = min(2^bits - 1, trunc(fl(fl(x - lo) * inv)))
// with inv = fl(2^bits / ext), ext = the largest extent of the bounding box.
__global__ __launch_bounds__(256) void k_morton(const float *__restrict__ pts, int64_t n,
                                                const int *__restrict__ bbox, int bits,
                                                const int64_t *__restrict__ set_off, int nsets,
                                                int npass, uint64_t *__restrict__ keys,
                                                uint32_t *__restrict__ vals,
                                                uint32_t *__restrict__ hist) {
    __shared__ uint32_t s_h[kMaxPass * 256];
    for (int i = threadIdx.x; i < npass * 256; i += blockDim.x) s_h[i] = 0;
    __syncthreads();
    float lo[3], ext = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = o2f(bbox[a]);
        ext = fmaxf(ext, o2f(bbox[3 + a]) - lo[a]);
    }
    float inv = ext > 0.0f ? (float)(1u << bits) / ext : 0.0f;
    if (!isfinite(inv)) inv = 0.0f;
    const uint32_t qmax = (1u << bits) - 1u;
    const int bits3 = 3 * bits;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint32_t q[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float t = (pts[3 * i + a] - lo[a]) * inv;
            uint32_t u = (t >= 0.0f) ? (uint32_t)fminf(t, 4294967040.0f) : 0u;
            q[a] = u < qmax ? u : qmax;
        }
        uint64_t key = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
        if (nsets > 1) {
            int lo_s = 0, hi_s = nsets - 1;  // largest s with set_off[s] <= i
            while (lo_s < hi_s) {
                int m = (lo_s + hi_s + 1) >> 1;
                if (set_off[m] <= i) lo_s = m; else hi_s = m - 1;
            }
            key |= (uint64_t)lo_s << bits3;
        }
        keys[i] = key;
        vals[i] = (uint32_t)i;
        for (int p = 0; p < npass; ++p) atomicAdd(&s_h[p * 256 + ((key >> (8 * p)) & 255u)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < npass * 256; i += blockDim.x)
        if (s_h[i]) atomicAdd(hist + i, s_h[i]);
}

// exclusive scan of each pass's 256 digit counts (one block per pass)
__global__ __launch_bounds__(256) void k_hist_scan(const uint32_t *__restrict__ hist,
                                                   uint32_t *__restrict__ doff) {
    __shared__ int s_w[4];
    const int p = blockIdx.x, t = threadIdx.x;
    int v = (int)hist[p * 256 + t];
    int inc = wave_incl_scan(v);
    if (lane_id() == 63) s_w[t >> 6] = inc;
    __syncthreads();
    int add = 0;
    for (int w = 0; w < (t >> 6); ++w) add += s_w[w];
    doff[p * 256 + t] = (uint32_t)(inc - v + add);
}

constexpr int RS_THREADS = 256;
constexpr int RS_WAVES = RS_THREADS / 64;
constexpr int RS_ITEMS = 24;  // 6144 keys per tile: two tiles fill a CU's LDS
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;
constexpr uint64_t FLAG_AGG = 1ull << 62;
constexpr uint64_t FLAG_INC = 2ull << 62;
constexpr uint64_t VAL_MASK = (1ull << 62) - 1;

__device__ __forceinline__ uint64_t ld_u64(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_u64(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One stable counting pass over the 8-bit digit at `shift`. Tiles take their
// id from an atomic counter (so every lower id belongs to a workgroup that has
// started); each tile ranks its keys per wave with ballots, publishes its digit
// counts, looks back over earlier tiles for its global offsets, stages the
// tile in LDS in digit order and writes it out with coalesced runs.
__global__ __launch_bounds__(RS_THREADS) void k_onesweep(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint64_t *__restrict__ kout,
    uint32_t *__restrict__ vout, int64_t n, int shift, const uint32_t *__restrict__ doff,
    uint64_t *__restrict__ status, int *__restrict__ tile_ctr) {
    __shared__ uint64_t s_k[RS_TILE];
    __shared__ uint32_t s_v[RS_TILE];
    __shared__ uint32_t s_wh[RS_WAVES][256];
    __shared__ uint32_t s_excl[256];
    __shared__ uint64_t s_gb[256];
    __shared__ int s_tmp[RS_WAVES];
    __shared__ int s_tile;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) s_tile = atomicAdd(tile_ctr, 1);
    for (int i = tid; i < RS_WAVES * 256; i += RS_THREADS) (&s_wh[0][0])[i] = 0;
    __syncthreads();
    const int tile = s_tile;
    const int64_t base = (int64_t)tile * RS_TILE;
    const int tn = (int)((n - base) < RS_TILE ? (n - base) : RS_TILE);

    uint64_t k[RS_ITEMS];
    uint32_t v[RS_ITEMS];
    uint32_t rk[RS_ITEMS];
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int li = w * (RS_ITEMS * 64) + i * 64 + lane;
        const bool valid = li < tn;
        k[i] = valid ? kin[base + li] : 0ull;
        v[i] = valid ? vin[base + li] : 0u;
    }
    const uint64_t ltm = lanemask_lt();
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int li = w * (RS_ITEMS * 64) + i * 64 + lane;
        const bool valid = li < tn;
        const uint32_t d = (uint32_t)(k[i] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t before = s_wh[w][d];
        rk[i] = (d << 16) | (before + (uint32_t)__popcll(peers & ltm));
        const bool leader = valid && ((peers & ltm) == 0ull);
        wave_lds_sync();
        if (leader) s_wh[w][d] = before + (uint32_t)__popcll(peers);
        wave_lds_sync();
    }
    __syncthreads();

    // per digit: wave prefix, tile total, look-back over earlier tiles
    const uint32_t c0 = s_wh[0][tid], c1 = s_wh[1][tid], c2 = s_wh[2][tid], c3 = s_wh[3][tid];
    const uint32_t tot = c0 + c1 + c2 + c3;
    s_wh[0][tid] = 0;
    s_wh[1][tid] = c0;
    s_wh[2][tid] = c0 + c1;
    s_wh[3][tid] = c0 + c1 + c2;
    uint64_t *mine = status + (size_t)tile * 256 + tid;
    uint64_t excl = 0;
    if (tile == 0) {
        st_u64(mine, FLAG_INC | tot);
    } else {
        st_u64(mine, FLAG_AGG | tot);
        int j = tile - 1;
        while (true) {
            const uint64_t sv = ld_u64(status + (size_t)j * 256 + tid);
            const uint64_t flag = sv >> 62;
            if (flag == 0) {  // predecessor not published yet
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            excl += sv & VAL_MASK;
            if (flag == 2 || j == 0) break;
            --j;
        }
        st_u64(mine, FLAG_INC | (excl + tot));
    }
    s_gb[tid] = (uint64_t)doff[tid] + excl;
    {
        const int vi = (int)tot;
        const int inc = wave_incl_scan(vi);
        if (lane == 63) s_tmp[w] = inc;
        __syncthreads();
        int add = 0;
        for (int ww = 0; ww < w; ++ww) add += s_tmp[ww];
        s_excl[tid] = (uint32_t)(inc - vi + add);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int li = w * (RS_ITEMS * 64) + i * 64 + lane;
        if (li < tn) {
            const uint32_t d = rk[i] >> 16;
            const uint32_t pos = s_excl[d] + s_wh[w][d] + (rk[i] & 0xffffu);
            s_k[pos] = k[i];
            s_v[pos] = v[i];
        }
    }
    __syncthreads();
    for (int e = tid; e < tn; e += RS_THREADS) {
        const uint64_t key = s_k[e];
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        const uint64_t dest = s_gb[d] + (uint64_t)(e - (int)s_excl[d]);
        kout[dest] = key;
        vout[dest] = s_v[e];
    }
}

// digit histograms of npass 8-bit passes over n 64-bit keys
__global__ __launch_bounds__(256) void k_digit_hist(const uint64_t *__restrict__ keys, int64_t n,
                                                    int npass, uint32_t *__restrict__ hist) {
    __shared__ uint32_t s_h[kMaxPass * 256];
    for (int i = threadIdx.x; i < npass * 256; i += blockDim.x) s_h[i] = 0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t key = keys[i];
        for (int p = 0; p < npass; ++p) atomicAdd(&s_h[p * 256 + ((key >> (8 * p)) & 255u)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < npass * 256; i += blockDim.x)
        if (s_h[i]) atomicAdd(hist + i, s_h[i]);
}

__global__ __launch_bounds__(256) void k_gather(const float *__restrict__ pts,
                                                const uint32_t *__restrict__ order, int64_t n,
                                                float4 *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t j = order[i];
    out[i] = make_float4(pts[3 * (int64_t)j], pts[3 * (int64_t)j + 1], pts[3 * (int64_t)j + 2],
                         __int_as_float((int)j));
}

// Level of gap g (between sorted points g-1 and g), Eq. 7 on keys extended by
// the sorted position: 32 + bitlen(key xor) for different keys, bitlen of the
// position xor for equal keys, 254 where the set changes, 255 at both ends.
__device__ __forceinline__ int gap_level(const uint64_t *__restrict__ keys, int64_t n, int64_t g,
                                         int bits3, int has_sets) {
    if (g <= 0 || g >= n) return kSentinelLevel;
    const uint64_t x = keys[g - 1] ^ keys[g];
    if (has_sets && (x >> bits3)) return kBoundaryLevel;
    if (x) return 32 + (int)bitlen64(x);
    return (int)bitlen64((uint64_t)(g - 1) ^ (uint64_t)g);
}

// level of the smallest node holding sorted points i < j
__device__ __forceinline__ int pair_level(const uint64_t *__restrict__ keys, int64_t i, int64_t j,
                                          int bits3, int has_sets) {
    const uint64_t x = keys[i] ^ keys[j];
    if (has_sets && (x >> bits3)) return kBoundaryLevel;
    if (x) return 32 + (int)bitlen64(x);
    return (int)bitlen64((uint64_t)i ^ (uint64_t)j);
}

constexpr int LF_TILE = 1024;
constexpr int LF_MAXW = 64;

// Leaf-plane split flags: gap g is a split iff the node spanning it holds
// more than nmax0 points, i.e. the nearest strictly greater gap on one side
// lies farther than the window, or both lie within it but r - l > nmax0.
// The nearest greater gaps are found by binary lifting over a table of range
// maxima of the tile (mx[k][i] = max of the 2^k levels from i), so every
// thread takes the same ~2 x 7 steps instead of a scan of up to 2 x nmax0.
constexpr int LF_SPAN = LF_TILE + 2 * LF_MAXW + 2;
constexpr int LF_LOG = 7;  // 2^6 = LF_MAXW: levels 0..6
__global__ __launch_bounds__(256) void k_leaf_flags(const uint64_t *__restrict__ keys, int64_t n,
                                                    int bits3, int has_sets, int nmax0,
                                                    uint8_t *__restrict__ flags,
                                                    int *__restrict__ blk_cnt) {
    __shared__ uint8_t s_mx[LF_LOG][LF_SPAN];
    __shared__ int s_c[4];
    const int W = nmax0;
    const int span = LF_TILE + 2 * W + 1;
    const int64_t g0 = (int64_t)blockIdx.x * LF_TILE;
    for (int t = threadIdx.x; t < span; t += blockDim.x)
        s_mx[0][t] = (uint8_t)gap_level(keys, n, g0 - W + t, bits3, has_sets);
    __syncthreads();
    for (int k = 1; k < LF_LOG; ++k) {
        const int h = 1 << (k - 1);
        for (int t = threadIdx.x; t + 2 * h <= span; t += blockDim.x)
            s_mx[k][t] = max(s_mx[k - 1][t], s_mx[k - 1][t + h]);
        __syncthreads();
    }
    int cnt = 0;
    for (int t = threadIdx.x; t < LF_TILE; t += blockDim.x) {
        const int64_t g = g0 + t;
        if (g > n) break;
        const int c = t + W;  // g's position in the tile
        const int lv = s_mx[0][c];
        uint8_t f;
        if (lv >= kBoundaryLevel) {
            f = 1;
        } else {
            // left: move cur down while [cur - 2^k, cur) holds no greater level
            int cur = c;
            for (int k = LF_LOG - 1; k >= 0; --k)
                if (cur - (1 << k) >= c - W && s_mx[k][cur - (1 << k)] <= lv) cur -= 1 << k;
            const int dl = cur - 1 >= c - W ? c - (cur - 1) : 0;
            int dr = 0;
            if (dl) {
                // right: move cur up while [cur, cur + 2^k) holds no greater level
                cur = c + 1;
                for (int k = LF_LOG - 1; k >= 0; --k)
                    if (cur + (1 << k) - 1 <= c + W && s_mx[k][cur] <= lv) cur += 1 << k;
                dr = cur <= c + W ? cur - c : 0;
            }
            f = (dl == 0 || dr == 0 || dl + dr > nmax0) ? 1 : 0;
        }
        flags[g] = f;
        cnt += f;
    }
    cnt = wave_sum(cnt);
    if (lane_id() == 0) s_c[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) blk_cnt[blockIdx.x] = s_c[0] + s_c[1] + s_c[2] + s_c[3];
}

// exclusive offsets of per-block counts; total to *total (one block)
__global__ __launch_bounds__(1024) void k_scan_counts(const int *__restrict__ cnt, int nb,
                                                      int *__restrict__ off,
                                                      int *__restrict__ total) {
    __shared__ int s_w[16];
    const int t = threadIdx.x;
    const int per = (nb + 1023) / 1024;
    const int b0 = t * per;
    int sum = 0;
    for (int i = 0; i < per; ++i)
        if (b0 + i < nb) sum += cnt[b0 + i];
    const int inc = wave_incl_scan(sum);
    if (lane_id() == 63) s_w[t >> 6] = inc;
    __syncthreads();
    int add = 0;
    for (int w = 0; w < (t >> 6); ++w) add += s_w[w];
    int run = inc - sum + add;
    for (int i = 0; i < per; ++i)
        if (b0 + i < nb) {
            off[b0 + i] = run;
            run += cnt[b0 + i];
        }
    if (t == 1023) *total = inc + add;
}

// ordered compaction of flagged items: out[pos] = item, out2[pos] = map[item]
__global__ __launch_bounds__(256) void k_compact(const uint8_t *__restrict__ flags,
                                                 int64_t nitems_max,
                                                 const int *__restrict__ nitems_dev,
                                                 const int *__restrict__ off,
                                                 int *__restrict__ out,
                                                 const int *__restrict__ map,
                                                 int *__restrict__ out2) {
    __shared__ int s_w[4];
    const int64_t nitems = nitems_dev ? (int64_t)(*nitems_dev) : nitems_max;
    const int64_t base = (int64_t)blockIdx.x * LF_TILE;
    int run = off[blockIdx.x];
    const int t = threadIdx.x, w = t >> 6;
    for (int c = 0; c < LF_TILE / 256; ++c) {
        const int64_t item = base + c * 256 + t;
        const bool f = item < nitems && flags[item];
        const uint64_t m = __ballot(f);
        const int pre = __popcll(m & lanemask_lt());
        if (lane_id() == 0) s_w[w] = __popcll(m);
        __syncthreads();
        int add = 0, tot = 0;
        for (int ww = 0; ww < 4; ++ww) {
            if (ww < w) add += s_w[ww];
            tot += s_w[ww];
        }
        if (f) {
            const int pos = run + add + pre;
            out[pos] = (int)item;
            if (map) out2[pos] = map[item];
        }
        run += tot;
        __syncthreads();
    }
}

// Exact size of the node spanning each leaf split (galloping search for the
// nearest strictly greater gap on both sides). Sentinels and set boundaries
// get INT_MAX so that they stay splits on every plane.
__global__ __launch_bounds__(256) void k_split_sizes(const uint64_t *__restrict__ keys, int64_t n,
                                                     int bits3, int has_sets,
                                                     const int *__restrict__ spl0,
                                                     const int *__restrict__ cnt0, int gallop0,
                                                     int *__restrict__ nsz,
                                                     uint8_t *__restrict__ slv) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t m = *cnt0;  // L0 + 1 entries
    if (s >= m) return;
    const int64_t g = spl0[s];
    const int lv = gap_level(keys, n, g, bits3, has_sets);
    slv[s] = (uint8_t)lv;
    if (lv >= kBoundaryLevel) {
        nsz[s] = INT_MAX;
        return;
    }
    // left: first j in [0, g-1] with pair_level(j, g) <= lv (monotone in j)
    int64_t good = g - 1, bad = -1, step = gallop0;
    while (good - bad > 1) {
        const int64_t j = good - step;
        if (j <= bad) break;
        if (pair_level(keys, j, g, bits3, has_sets) <= lv) {
            good = j;
            step <<= 1;
        } else {
            bad = j;
            break;
        }
    }
    while (good - bad > 1) {
        const int64_t mid = bad + (good - bad) / 2;
        if (pair_level(keys, mid, g, bits3, has_sets) <= lv) good = mid; else bad = mid;
    }
    const int64_t lb = good;
    // right: first j in [g, n) with pair_level(g-1, j) > lv, else n
    good = g;
    bad = n;
    step = gallop0;
    while (bad - good > 1) {
        const int64_t j = good + step;
        if (j >= bad) break;
        if (pair_level(keys, g - 1, j, bits3, has_sets) <= lv) {
            good = j;
            step <<= 1;
        } else {
            bad = j;
            break;
        }
    }
    while (bad - good > 1) {
        const int64_t mid = good + (bad - good) / 2;
        if (pair_level(keys, g - 1, mid, bits3, has_sets) <= lv) good = mid; else bad = mid;
    }
    const int64_t rb = bad;
    nsz[s] = (int)(rb - lb);
}

// Plane p flags over the plane p-1 splits: keep the ends and every split
// whose node size exceeds N_max^(p).
__global__ __launch_bounds__(256) void k_plane_flags(const int *__restrict__ lsi_prev,
                                                     const int *__restrict__ cnt_prev,
                                                     const int *__restrict__ nsz, int64_t nmax,
                                                     const uint8_t *__restrict__ slv, int lvl_max,
                                                     uint8_t *__restrict__ flags,
                                                     int *__restrict__ blk_cnt) {
    __shared__ int s_c[4];
    const int64_t m = *cnt_prev;
    int cnt = 0;
    const int64_t base = (int64_t)blockIdx.x * LF_TILE;
    for (int t = threadIdx.x; t < LF_TILE; t += blockDim.x) {
        const int64_t j = base + t;
        if (j >= m) break;
        const int ls = lsi_prev[j];
        const uint8_t f = (j == 0 || j == m - 1 || (int64_t)nsz[ls] > nmax ||
                           (int)slv[ls] > lvl_max) ? 1 : 0;
        flags[j] = f;
        cnt += f;
    }
    cnt = wave_sum(cnt);
    if (lane_id() == 0) s_c[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) blk_cnt[blockIdx.x] = s_c[0] + s_c[1] + s_c[2] + s_c[3];
}

// Regularization (paper: section on regularization): points per node level
// over the nodes of a plane. Node i spans the sorted points between leaf
// splits lsi[i] and lsi[i + 1] (lsi = NULL: the leaf plane itself); its level
// is that of its first and last point (the largest gap level inside it).
__global__ __launch_bounds__(256) void k_level_hist(const uint64_t *__restrict__ keys,
                                                    const int *__restrict__ spl0,
                                                    const int *__restrict__ lsi,
                                                    const int *__restrict__ cnt, int bits3,
                                                    int has_sets,
                                                    unsigned long long *__restrict__ hist) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i + 1 >= *cnt) return;
    const int64_t a = spl0[lsi ? lsi[i] : i], e = spl0[lsi ? lsi[i + 1] : i + 1];
    const int lv = e - a > 1 ? pair_level(keys, a, e - 1, bits3, has_sets) : 0;
    atomicAdd(hist + lv, (unsigned long long)(e - a));
}

// leaf plane: also split every gap whose level exceeds lvl_max; per-block
// counts as k_leaf_flags
__global__ __launch_bounds__(256) void k_reg_leaf_flags(const uint64_t *__restrict__ keys,
                                                        int64_t n, int bits3, int has_sets,
                                                        int lvl_max, uint8_t *__restrict__ flags,
                                                        int *__restrict__ blk_cnt) {
    __shared__ int s_c[4];
    int cnt = 0;
    const int64_t g0 = (int64_t)blockIdx.x * LF_TILE;
    for (int t = threadIdx.x; t < LF_TILE; t += blockDim.x) {
        const int64_t g = g0 + t;
        if (g > n) break;
        uint8_t f = flags[g];
        if (!f && gap_level(keys, n, g, bits3, has_sets) > lvl_max) {
            f = 1;
            flags[g] = 1;
        }
        cnt += f;
    }
    cnt = wave_sum(cnt);
    if (lane_id() == 0) s_c[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) blk_cnt[blockIdx.x] = s_c[0] + s_c[1] + s_c[2] + s_c[3];
}

__global__ void k_iota(int *__restrict__ a, const int *__restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < *cnt) a[i] = (int)i;
}

// leaves: one wave per leaf, lanes over its points
__global__ __launch_bounds__(256) void k_leaf_geom(const float4 *__restrict__ pts,
                                                   const int *__restrict__ spl, int64_t L,
                                                   Node *__restrict__ nodes) {
    const int64_t a = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (a >= L) return;
    const int s0 = spl[a], s1 = spl[a + 1];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = s0 + lane_id(); i < s1; i += 64) {
        const float4 p = pts[i];
        lo[0] = fminf(lo[0], p.x); hi[0] = fmaxf(hi[0], p.x);
        lo[1] = fminf(lo[1], p.y); hi[1] = fmaxf(hi[1], p.y);
        lo[2] = fminf(lo[2], p.z); hi[2] = fmaxf(hi[2], p.z);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        lo[d] = wave_min(lo[d]);
        hi[d] = wave_max(hi[d]);
    }
    if (lane_id() == 0) {
        Node nd;
        nd.lo[0] = lo[0]; nd.lo[1] = lo[1]; nd.lo[2] = lo[2];
        nd.hi[0] = hi[0]; nd.hi[1] = hi[1]; nd.hi[2] = hi[2];
        nd.start = s0;
        nd.count = s1 - s0;
        nodes[a] = nd;
    }
}

// coarser planes: one wave per node, lanes over its children
__global__ __launch_bounds__(256) void k_node_geom(const Node *__restrict__ child,
                                                   const int *__restrict__ spl, int64_t L,
                                                   Node *__restrict__ nodes) {
    const int64_t a = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (a >= L) return;
    const int c0 = spl[a], c1 = spl[a + 1];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int cnt = 0;
    for (int c = c0 + lane_id(); c < c1; c += 64) {
        const Node ch = child[c];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            lo[d] = fminf(lo[d], ch.lo[d]);
            hi[d] = fmaxf(hi[d], ch.hi[d]);
        }
        cnt += ch.count;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        lo[d] = wave_min(lo[d]);
        hi[d] = wave_max(hi[d]);
    }
    cnt = wave_sum(cnt);
    if (lane_id() == 0) {
        Node nd;
        nd.lo[0] = lo[0]; nd.lo[1] = lo[1]; nd.lo[2] = lo[2];
        nd.hi[0] = hi[0]; nd.hi[1] = hi[1]; nd.hi[2] = hi[2];
        nd.start = child[c0].start;
        nd.count = cnt;
        nodes[a] = nd;
    }
}

// set of each node (from the key of its first point) and, for leaves, the
// first input index of that set
__global__ void k_node_sets(const Node *__restrict__ nodes, int64_t L,
                            const uint64_t *__restrict__ keys, int bits3,
                            const int64_t *__restrict__ set_off, int *__restrict__ set_of,
                            int *__restrict__ base_of) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= L) return;
    const int s = (int)(keys[nodes[a].start] >> bits3);
    set_of[a] = s;
    if (base_of) base_of[a] = (int)set_off[s];
}

}  // namespace

// ---------------------------------------------------------------------------

// The onesweep passes over the low 8 * npass key bits, with the exclusive
// digit offsets in doff; (kin, vin) -> sorted pairs, swapping with
// (kout, vout) after every pass (the result is where the last pass wrote).
static jz_status onesweep_passes(const AllocCtx *ac, uint64_t *&kin, uint32_t *&vin,
                                 uint64_t *&kout, uint32_t *&vout, int64_t n, int npass,
                                 const uint32_t *doff, hipStream_t s) {
    const int64_t ntiles = (n + RS_TILE - 1) / RS_TILE;
    DBuf d_status;
    const size_t per_pass = (size_t)ntiles * 256;
    JZ_TRY(d_status.get(ac, (per_pass * npass) * sizeof(uint64_t) + 64 * sizeof(int), s));
    JZ_TRY(zero_words(d_status.as<unsigned long long>(), d_status.bytes / 8, s));
    int *ctrs = reinterpret_cast<int *>(d_status.as<uint64_t>() + per_pass * npass);
    for (int p = 0; p < npass; ++p) {
        k_onesweep<<<(unsigned)ntiles, RS_THREADS, 0, s>>>(
            kin, vin, kout, vout, n, 8 * p, doff + 256 * p, d_status.as<uint64_t>() + per_pass * p,
            ctrs + p);
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    JZ_HIP(hipGetLastError());
    return JZ_OK;
}

jz_status radix_sort_pairs(const AllocCtx *ac, DBuf &k0, DBuf &v0, DBuf &k1, DBuf &v1, int64_t n,
                           int bits, hipStream_t s) {
    if (n <= 1 || bits <= 0) return JZ_OK;
    const int npass = std::min(kMaxPass, (bits + 7) / 8);
    DBuf d_hist, d_doff;
    JZ_TRY(d_hist.get(ac, kMaxPass * 256 * sizeof(uint32_t), s));
    JZ_TRY(d_doff.get(ac, kMaxPass * 256 * sizeof(uint32_t), s));
    JZ_TRY(zero_words(d_hist.as<unsigned long long>(), d_hist.bytes / 8, s));
    k_digit_hist<<<std::min<unsigned>(blocks_for(n, 256 * 8), 2048), 256, 0, s>>>(
        k0.as<uint64_t>(), n, npass, d_hist.as<uint32_t>());
    k_hist_scan<<<npass, 256, 0, s>>>(d_hist.as<uint32_t>(), d_doff.as<uint32_t>());
    uint64_t *kin = k0.as<uint64_t>(), *kout = k1.as<uint64_t>();
    uint32_t *vin = v0.as<uint32_t>(), *vout = v1.as<uint32_t>();
    JZ_TRY(onesweep_passes(ac, kin, vin, kout, vout, n, npass, d_doff.as<uint32_t>(), s));
    if (kin != k0.as<uint64_t>()) {
        std::swap(k0.p, k1.p);
        std::swap(v0.p, v1.p);
    }
    return JZ_OK;
}

namespace {

// source points per leaf (one wave per leaf: a leaf holds at most 64 points)
__global__ __launch_bounds__(256) void k_src_count_leaf(const Node *__restrict__ leaves, int64_t L,
                                                        const float4 *__restrict__ pts, int n_src,
                                                        int *__restrict__ cnt) {
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (i >= L) return;
    const Node a = leaves[i];
    const int lane = lane_id();
    const bool src = lane < a.count && __float_as_int(pts[a.start + lane].w) < n_src;
    const uint64_t m = __ballot(src);
    if (lane == 0) cnt[i] = (int)__popcll(m);
}

// source points per node of a coarser plane: the sum over its children
__global__ __launch_bounds__(256) void k_src_count_up(const int *__restrict__ child,
                                                      const int *__restrict__ spl, int64_t L,
                                                      int *__restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L) return;
    int s = 0;
    for (int c = spl[i]; c < spl[i + 1]; ++c) s += child[c];
    cnt[i] = s;
}

}  // namespace

jz_status source_counts(jz_tree *t, hipStream_t s) {
    for (int p = 0; p < t->P; ++p) {
        JZ_TRY(t->src_cnt[p].get(&t->ac, (size_t)t->L[p] * sizeof(int), s));
        if (p == 0)
            k_src_count_leaf<<<blocks_for(t->L[0] * 64, 256), 256, 0, s>>>(
                t->nodes[0].as<Node>(), t->L[0], t->pts4.as<float4>(), (int)t->n_src,
                t->src_cnt[0].as<int>());
        else
            k_src_count_up<<<blocks_for(t->L[p], 256), 256, 0, s>>>(
                t->src_cnt[p - 1].as<int>(), t->spl[p].as<int>(), t->L[p], t->src_cnt[p].as<int>());
    }
    JZ_HIP(hipGetLastError());
    return JZ_OK;
}

// Regularization: the largest node level of a plane from its histogram of
// points per node level. V90 is the point-weighted mean volume (2^level) of
// the smallest nodes that together hold 90% of the points; nodes may not
// exceed f_max * V90, i.e. levels above floor(log2(f_max * V90)) are split.
static int reg_level_max(const unsigned long long *hist, double f_max) {
    double total = 0;
    for (int l = 0; l < 256; ++l) total += (double)hist[l];
    if (total <= 0) return 1000;
    double cum = 0, wsum = 0;
    for (int l = 0; l < 256 && cum < 0.9 * total; ++l) {
        cum += (double)hist[l];
        wsum += (double)hist[l] * std::ldexp(1.0, l);
    }
    const double v90 = wsum / cum;
    return (int)std::floor(std::log2(f_max * v90));
}

static int plan_planes(int64_t n, const jz_build_opts &o) {
    int P = 1;
    double nmax = (double)o.leaf_max;
    while (P < JZ_MAX_PLANES) {
        nmax *= o.coarsen;
        if ((double)n / (nmax / 2.0) < (double)o.n_target) break;
        ++P;
    }
    return P;
}

jz_status build_tree(jz_tree *t, const float *points, hipStream_t s) {
    const int64_t n = t->n;
    const AllocCtx *ac = &t->ac;
    const jz_build_opts &o = t->opts;
    t->P = 0;
    if (n == 0) return JZ_OK;

    const int has_sets = t->nsets > 1;
    // automatic key bits: 5 more per dimension than an even split of n
    // points needs (cells 32 times finer than the mean spacing), raised to
    // as many as the radix passes those need can hold (a pass sorts 8 key
    // bits; set bits come first), at most 21
    int bits = o.key_bits;
    if (bits == 0) {
        int lg = 0;
        while (lg < 62 && ((int64_t)1 << lg) < n) ++lg;
        const int b0 = std::max(10, (lg + 2) / 3 + 5);
        const int np = (3 * b0 + t->set_bits + 7) / 8;
        bits = std::min(21, std::max(b0, (8 * np - t->set_bits) / 3));
    }
    const int max_bits = (63 - t->set_bits) / 3;
    if (bits > max_bits) bits = max_bits;
    const int bits3 = 3 * bits;
    const int total_bits = bits3 + t->set_bits;
    const int npass = (total_bits + 7) / 8;

    // 1-2: bbox, keys, histograms
    DBuf d_bbox, d_hist, d_doff, k0, k1, v0, v1;
    JZ_TRY(d_bbox.get(ac, 8 * sizeof(int), s));
    JZ_TRY(d_hist.get(ac, kMaxPass * 256 * sizeof(uint32_t), s));
    JZ_TRY(d_doff.get(ac, kMaxPass * 256 * sizeof(uint32_t), s));
    JZ_TRY(k0.get(ac, n * sizeof(uint64_t), s));
    JZ_TRY(k1.get(ac, n * sizeof(uint64_t), s));
    JZ_TRY(v0.get(ac, n * sizeof(uint32_t), s));
    JZ_TRY(v1.get(ac, n * sizeof(uint32_t), s));
    {
        const int init[8] = {INT_MAX, INT_MAX, INT_MAX, INT_MIN, INT_MIN, INT_MIN, 0, 0};
        JZ_HIP(hipMemcpyAsync(d_bbox.p, init, sizeof(init), hipMemcpyHostToDevice, s));
    }
    JZ_TRY(zero_words(d_hist.as<unsigned long long>(), d_hist.bytes / 8, s));
    const unsigned gb = std::min<unsigned>(blocks_for(n, 256), 1024);
    k_bbox<<<gb, 256, 0, s>>>(points, n, d_bbox.as<int>());
    k_morton<<<std::min<unsigned>(blocks_for(n, 256 * 8), 2048), 256, 0, s>>>(
        points, n, d_bbox.as<int>(), bits, t->d_set_off.as<int64_t>(), t->nsets, npass,
        k0.as<uint64_t>(), v0.as<uint32_t>(), d_hist.as<uint32_t>());
    k_hist_scan<<<npass, 256, 0, s>>>(d_hist.as<uint32_t>(), d_doff.as<uint32_t>());
    JZ_HIP(hipGetLastError());

    // 3: radix sort
    {
        uint64_t *kin = k0.as<uint64_t>(), *kout = k1.as<uint64_t>();
        uint32_t *vin = v0.as<uint32_t>(), *vout = v1.as<uint32_t>();
        JZ_TRY(onesweep_passes(ac, kin, vin, kout, vout, n, npass, d_doff.as<uint32_t>(), s));
        // sorted data is in (kin, vin)
        if (kin != k0.as<uint64_t>()) {
            std::swap(k0.p, k1.p);
            std::swap(v0.p, v1.p);
        }
    }
    const uint64_t *keys = k0.as<uint64_t>();
    const uint32_t *order = v0.as<uint32_t>();

    // 4: sorted points
    JZ_TRY(t->pts4.get(ac, n * sizeof(float4), s));
    k_gather<<<blocks_for(n, 256), 256, 0, s>>>(points, order, n, t->pts4.as<float4>());

    // 5: leaf plane
    const int64_t ngaps = n + 1;
    const unsigned nb = blocks_for(ngaps, LF_TILE);
    DBuf d_flags, d_bcnt, d_boff, d_cnt;
    JZ_TRY(d_flags.get(ac, ngaps, s));
    JZ_TRY(d_bcnt.get(ac, (size_t)nb * sizeof(int), s));
    JZ_TRY(d_boff.get(ac, (size_t)nb * sizeof(int), s));
    JZ_TRY(d_cnt.get(ac, (JZ_MAX_PLANES + 2) * sizeof(int), s));
    int *cnts = d_cnt.as<int>();
    JZ_TRY(t->spl[0].get(ac, ngaps * sizeof(int), s));
    k_leaf_flags<<<nb, 256, 0, s>>>(keys, n, bits3, has_sets, o.leaf_max, d_flags.as<uint8_t>(),
                                    d_bcnt.as<int>());
    k_scan_counts<<<1, 1024, 0, s>>>(d_bcnt.as<int>(), (int)nb, d_boff.as<int>(), cnts + 0);
    k_compact<<<nb, 256, 0, s>>>(d_flags.as<uint8_t>(), ngaps, nullptr, d_boff.as<int>(),
                                 t->spl[0].as<int>(), nullptr, nullptr);
    JZ_HIP(hipGetLastError());
    // regularization: the largest level each plane's nodes may have
    const bool reg = o.reg_fmax > 0.0f;
    DBuf d_hist2;
    int lvl_max = 1000;
    auto plane_level_max = [&](const int *lsi, const int *cnt_dev) -> jz_status {
        JZ_TRY(zero_words(d_hist2.as<unsigned long long>(), 256, s));
        k_level_hist<<<blocks_for(ngaps, 256), 256, 0, s>>>(keys, t->spl[0].as<int>(), lsi,
                                                            cnt_dev, bits3, has_sets,
                                                            d_hist2.as<unsigned long long>());
        unsigned long long h[256];
        JZ_HIP(hipMemcpyAsync(h, d_hist2.p, sizeof(h), hipMemcpyDeviceToHost, s));
        JZ_HIP(hipStreamSynchronize(s));
        lvl_max = std::max(lvl_max == 1000 ? 0 : lvl_max, reg_level_max(h, o.reg_fmax));
        return JZ_OK;
    };
    if (reg) {
        JZ_TRY(d_hist2.get(ac, 256 * sizeof(unsigned long long), s));
        JZ_TRY(plane_level_max(nullptr, cnts + 0));
        k_reg_leaf_flags<<<nb, 256, 0, s>>>(keys, n, bits3, has_sets, lvl_max,
                                            d_flags.as<uint8_t>(), d_bcnt.as<int>());
        k_scan_counts<<<1, 1024, 0, s>>>(d_bcnt.as<int>(), (int)nb, d_boff.as<int>(), cnts + 0);
        k_compact<<<nb, 256, 0, s>>>(d_flags.as<uint8_t>(), ngaps, nullptr, d_boff.as<int>(),
                                     t->spl[0].as<int>(), nullptr, nullptr);
        JZ_HIP(hipGetLastError());
    }
    int host_hdr[8];
    JZ_HIP(hipMemcpyAsync(host_hdr, cnts, sizeof(int), hipMemcpyDeviceToHost, s));
    JZ_HIP(hipMemcpyAsync(host_hdr + 1, d_bbox.as<int>(), 7 * sizeof(int), hipMemcpyDeviceToHost,
                          s));
    JZ_HIP(hipStreamSynchronize(s));
    if (host_hdr[7]) return jz_fail(JZ_E_NONFINITE, "input contains NaN or infinite coordinates");
    if (o.period > 0.0f) {
        // the periodic cube is [0, period)^3
        auto of = [](int v) {
            const int i = v >= 0 ? v : v ^ 0x7FFFFFFF;
            float f;
            std::memcpy(&f, &i, sizeof(f));
            return f;
        };
        for (int a = 0; a < 3; ++a)
            if (!(of(host_hdr[1 + a]) >= 0.0f) || !(of(host_hdr[4 + a]) < o.period))
                return jz_fail(JZ_E_INVALID, "with period %g every coordinate must lie in "
                               "[0, %g)", (double)o.period, (double)o.period);
    }
    const int64_t m0 = host_hdr[0];  // L0 + 1
    t->L[0] = m0 - 1;

    // 6-7: node sizes at leaf splits, coarser planes
    const int P = plan_planes(n, o);
    DBuf d_nsz, d_slv, lsiA, lsiB;
    JZ_TRY(d_nsz.get(ac, m0 * sizeof(int), s));
    JZ_TRY(d_slv.get(ac, m0, s));
    k_split_sizes<<<blocks_for(m0, 256), 256, 0, s>>>(keys, n, bits3, has_sets, t->spl[0].as<int>(),
                                                     cnts + 0, o.leaf_max, d_nsz.as<int>(),
                                                     d_slv.as<uint8_t>());
    if (P > 1) {
        JZ_TRY(lsiA.get(ac, m0 * sizeof(int), s));
        JZ_TRY(lsiB.get(ac, m0 * sizeof(int), s));
        k_iota<<<blocks_for(m0, 256), 256, 0, s>>>(lsiA.as<int>(), cnts + 0);
        const unsigned nbp = blocks_for(m0, LF_TILE);
        int64_t nmax = o.leaf_max;
        for (int p = 1; p < P; ++p) {
            nmax *= o.coarsen;
            JZ_TRY(t->spl[p].get(ac, m0 * sizeof(int), s));
            // with regularization a plane is selected twice: by counts, then
            // also splitting the levels above its nodes' lvl_max
            for (int pass = 0; pass < (reg ? 2 : 1); ++pass) {
                k_plane_flags<<<nbp, 256, 0, s>>>(lsiA.as<int>(), cnts + p - 1, d_nsz.as<int>(),
                                                  nmax, d_slv.as<uint8_t>(),
                                                  pass ? lvl_max : 1000, d_flags.as<uint8_t>(),
                                                  d_bcnt.as<int>());
                k_scan_counts<<<1, 1024, 0, s>>>(d_bcnt.as<int>(), (int)nbp, d_boff.as<int>(),
                                                 cnts + p);
                k_compact<<<nbp, 256, 0, s>>>(d_flags.as<uint8_t>(), m0, cnts + p - 1,
                                              d_boff.as<int>(), t->spl[p].as<int>(),
                                              lsiA.as<int>(), lsiB.as<int>());
                if (reg && pass == 0) JZ_TRY(plane_level_max(lsiB.as<int>(), cnts + p));
            }
            std::swap(lsiA.p, lsiB.p);
        }
        JZ_HIP(hipGetLastError());
        int hc[JZ_MAX_PLANES];
        JZ_HIP(hipMemcpyAsync(hc, cnts, P * sizeof(int), hipMemcpyDeviceToHost, s));
        JZ_HIP(hipStreamSynchronize(s));
        for (int p = 0; p < P; ++p) t->L[p] = hc[p] - 1;
    }
    t->P = P;

    // 8: geometry
    for (int p = 0; p < P; ++p) {
        JZ_TRY(t->nodes[p].get(ac, t->L[p] * sizeof(Node), s));
        if (p == 0)
            k_leaf_geom<<<blocks_for(t->L[0] * 64, 256), 256, 0, s>>>(
                t->pts4.as<float4>(), t->spl[0].as<int>(), t->L[0], t->nodes[0].as<Node>());
        else
            k_node_geom<<<blocks_for(t->L[p] * 64, 256), 256, 0, s>>>(
                t->nodes[p - 1].as<Node>(), t->spl[p].as<int>(), t->L[p], t->nodes[p].as<Node>());
    }
    JZ_HIP(hipGetLastError());

    // super nodes over the top plane, per set
    const int T = P - 1;
    const int64_t LT = t->L[T];
    std::vector<int> top_set(LT, 0);
    if (has_sets) {
        JZ_TRY(t->leaf_base.get(ac, t->L[0] * sizeof(int), s));
        for (int p = 0; p < P; ++p) {
            JZ_TRY(t->node_set[p].get(ac, t->L[p] * sizeof(int), s));
            k_node_sets<<<blocks_for(t->L[p], 256), 256, 0, s>>>(
                t->nodes[p].as<Node>(), t->L[p], keys, bits3, t->d_set_off.as<int64_t>(),
                t->node_set[p].as<int>(), p == 0 ? t->leaf_base.as<int>() : nullptr);
        }
        JZ_HIP(hipMemcpyAsync(top_set.data(), t->node_set[T].p, LT * sizeof(int),
                              hipMemcpyDeviceToHost, s));
        JZ_HIP(hipStreamSynchronize(s));
    }
    std::vector<int> sspl;
    t->super_set.clear();
    for (int64_t a = 0; a < LT;) {
        int64_t b = a;
        while (b < LT && top_set[b] == top_set[a]) ++b;
        for (int64_t c = a; c < b; c += o.ngr) {
            sspl.push_back((int)c);
            t->super_set.push_back(top_set[a]);
        }
        a = b;
    }
    t->S = (int64_t)sspl.size();
    sspl.push_back((int)LT);
    // dense lists over the super nodes of each set
    std::vector<int2> kseg(t->S), fseg(t->S), klist, flist;
    for (int64_t a = 0; a < t->S;) {
        int64_t b = a;
        while (b < t->S && t->super_set[b] == t->super_set[a]) ++b;
        for (int64_t i = a; i < b; ++i) {
            kseg[i] = make_int2((int)klist.size(), (int)(b - a));
            for (int64_t j = a; j < b; ++j) klist.push_back(make_int2((int)j, 0));
            fseg[i] = make_int2((int)flist.size(), (int)(b - i));
            for (int64_t j = i; j < b; ++j) flist.push_back(make_int2((int)j, 0));
        }
        a = b;
    }
    JZ_TRY(t->super_spl.get(ac, sspl.size() * sizeof(int), s));
    JZ_TRY(t->knn_top_seg.get(ac, kseg.size() * sizeof(int2), s));
    JZ_TRY(t->knn_top_list.get(ac, klist.size() * sizeof(int2), s));
    JZ_TRY(t->fof_top_seg.get(ac, fseg.size() * sizeof(int2), s));
    JZ_TRY(t->fof_top_list.get(ac, flist.size() * sizeof(int2), s));
    JZ_HIP(hipMemcpyAsync(t->super_spl.p, sspl.data(), sspl.size() * sizeof(int),
                          hipMemcpyHostToDevice, s));
    JZ_HIP(hipMemcpyAsync(t->knn_top_seg.p, kseg.data(), kseg.size() * sizeof(int2),
                          hipMemcpyHostToDevice, s));
    JZ_HIP(hipMemcpyAsync(t->knn_top_list.p, klist.data(), klist.size() * sizeof(int2),
                          hipMemcpyHostToDevice, s));
    JZ_HIP(hipMemcpyAsync(t->fof_top_seg.p, fseg.data(), fseg.size() * sizeof(int2),
                          hipMemcpyHostToDevice, s));
    JZ_HIP(hipMemcpyAsync(t->fof_top_list.p, flist.data(), flist.size() * sizeof(int2),
                          hipMemcpyHostToDevice, s));
    if (o.keep_keys) {
        JZ_TRY(t->keys.get(ac, n * sizeof(uint64_t), s));
        JZ_HIP(hipMemcpyAsync(t->keys.p, keys, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
    }
    JZ_HIP(hipStreamSynchronize(s));

    // stats
    t->st.n = n;
    t->st.planes = P;
    for (int p = 0; p < JZ_MAX_PLANES; ++p) t->st.nodes[p] = p < P ? t->L[p] : 0;
    t->st.super_nodes = t->S;
    return JZ_OK;
}
