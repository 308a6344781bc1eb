// FoF catalogue reduction (paper: FoF section, "Catalogue reduction"): after
// the groups are found, the points are brought into group order by a stable
// sort on the group label, and each group with at least min_members points
// gets its summary statistics.
//
//  1. keys = label (the smallest member index), values = input index; a
//     stable radix sort on the label bits gives group order: groups by
//     ascending label, members of a group as one block of ascending input
//     indices
//  2. member counts per label; group starts (a key differing from the one
//     before); the starts of groups with >= min_members members compacted in
//     order: group g = (label, first position, count)
//  3. centre of mass (and of velocity): per-wave sums over the runs of one
//     group (positions are in group order, so a wave meets few groups), one
//     binary64 atomic per group, component and wave
//  4. inertia radius: the same over |x - cm|^2, then sqrt(sum / count)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <vector>

#include "jz_device.h"
#include "jz_internal.h"

namespace {

constexpr int CAT_BLOCK = 1024;  // positions per compaction block

__global__ __launch_bounds__(256) void k_cat_keys(const int32_t *__restrict__ label, int64_t n,
                                                  uint64_t *__restrict__ keys,
                                                  uint32_t *__restrict__ vals,
                                                  int *__restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int l = label[i];
    keys[i] = (uint64_t)(uint32_t)l;
    vals[i] = (uint32_t)i;
    atomicAdd(count + l, 1);
}

__device__ __forceinline__ bool cat_start(const uint64_t *keys, const int *count, int64_t j,
                                          int min_members) {
    return (j == 0 || keys[j] != keys[j - 1]) && count[keys[j]] >= min_members;
}

// qualifying group starts per block of CAT_BLOCK positions
__global__ __launch_bounds__(256) void k_cat_block_counts(const uint64_t *__restrict__ keys,
                                                          const int *__restrict__ count, int64_t n,
                                                          int min_members, int *__restrict__ bcnt) {
    __shared__ int s_c[4];
    const int64_t b0 = (int64_t)blockIdx.x * CAT_BLOCK;
    int c = 0;
    for (int t = threadIdx.x; t < CAT_BLOCK; t += 256) {
        const int64_t j = b0 + t;
        if (j < n && cat_start(keys, count, j, min_members)) ++c;
    }
    c = wave_sum_i(c);
    if (lane_id() == 0) s_c[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) bcnt[blockIdx.x] = s_c[0] + s_c[1] + s_c[2] + s_c[3];
}

// exclusive scan of nb block counts by one workgroup; total in *total
__global__ __launch_bounds__(1024) void k_cat_scan(const int *__restrict__ bcnt, int nb,
                                                   int *__restrict__ boff,
                                                   long long *__restrict__ total) {
    __shared__ int s_w[16];
    __shared__ int s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int c0 = 0; c0 < nb; c0 += 1024) {
        const int i = c0 + (int)threadIdx.x;
        const int v = i < nb ? bcnt[i] : 0;
        const int inc = wave_incl_scan(v);
        if (lane_id() == 63) s_w[threadIdx.x >> 6] = inc;
        __syncthreads();
        int add = s_carry;
        for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) add += s_w[w];
        if (i < nb) boff[i] = add + inc - v;
        __syncthreads();
        if (threadIdx.x == 1023) s_carry = add + inc;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = s_carry;
}

// the qualifying groups in order: label, first position, count; gidx[label]
// = group number (gidx is -1 elsewhere)
__global__ __launch_bounds__(256) void k_cat_compact(const uint64_t *__restrict__ keys,
                                                     const int *__restrict__ count, int64_t n,
                                                     int min_members, const int *__restrict__ boff,
                                                     jz_group *__restrict__ groups,
                                                     int64_t max_groups, int *__restrict__ gidx) {
    __shared__ int s_w[4];
    const int64_t b0 = (int64_t)blockIdx.x * CAT_BLOCK;
    int base = boff[blockIdx.x];
    for (int t0 = 0; t0 < CAT_BLOCK; t0 += 256) {
        const int64_t j = b0 + t0 + threadIdx.x;
        const bool st = j < n && cat_start(keys, count, j, min_members);
        const uint64_t m = __ballot(st);
        const int w = threadIdx.x >> 6;
        if (lane_id() == 0) s_w[w] = __popcll(m);
        __syncthreads();
        int off = base;
        for (int ww = 0; ww < w; ++ww) off += s_w[ww];
        if (st) {
            const int g = off + __popcll(m & lanemask_lt());
            const int l = (int)keys[j];
            gidx[l] = g;
            if (g < max_groups) {
                jz_group gr{};
                gr.label = l;
                gr.count = count[l];
                gr.first = j;
                groups[g] = gr;
            }
        }
        base += s_w[0] + s_w[1] + s_w[2] + s_w[3];
        __syncthreads();
    }
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Pass 1 (second = false): sums of positions (and velocities) per group.
// Pass 2 (second = true): sums of |x - cm|^2 per group, cm from pass 1.
// acc[g] holds 8 doubles: sx, sy, sz, svx, svy, svz, sd2, unused.
__global__ __launch_bounds__(256) void k_cat_sums(const uint64_t *__restrict__ keys,
                                                  const uint32_t *__restrict__ order, int64_t n,
                                                  const int *__restrict__ gidx,
                                                  const float *__restrict__ pts,
                                                  const float *__restrict__ vel, bool second,
                                                  const jz_group *__restrict__ groups,
                                                  double *__restrict__ acc) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int g = -1;
    double x = 0, y = 0, z = 0, a = 0, b = 0, c = 0;
    if (j < n) {
        g = gidx[keys[j]];
        if (g >= 0) {
            const int64_t i = order[j];
            x = pts[3 * i];
            y = pts[3 * i + 1];
            z = pts[3 * i + 2];
            if (second) {
                const jz_group &gr = groups[g];
                const double dx = x - gr.cm[0], dy = y - gr.cm[1], dz = z - gr.cm[2];
                x = (dx * dx + dy * dy) + dz * dz;
            } else if (vel) {
                a = vel[3 * i];
                b = vel[3 * i + 1];
                c = vel[3 * i + 2];
            }
        }
    }
    uint64_t pending = __ballot(g >= 0);
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int g0 = __builtin_amdgcn_readlane(g, leader);
        const bool mine = g == g0;
        pending &= ~__ballot(mine);
        double *dst = acc + (size_t)g0 * 8;
        if (second) {
            const double s = wave_sum_d(mine ? x : 0.0);
            if (lane_id() == leader) atomicAdd(dst + 6, s);
        } else {
            const double sx = wave_sum_d(mine ? x : 0.0);
            const double sy = wave_sum_d(mine ? y : 0.0);
            const double sz = wave_sum_d(mine ? z : 0.0);
            if (lane_id() == leader) {
                atomicAdd(dst + 0, sx);
                atomicAdd(dst + 1, sy);
                atomicAdd(dst + 2, sz);
            }
            if (vel) {
                const double sa = wave_sum_d(mine ? a : 0.0);
                const double sb = wave_sum_d(mine ? b : 0.0);
                const double sc = wave_sum_d(mine ? c : 0.0);
                if (lane_id() == leader) {
                    atomicAdd(dst + 3, sa);
                    atomicAdd(dst + 4, sb);
                    atomicAdd(dst + 5, sc);
                }
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_cat_finish(jz_group *__restrict__ groups, int64_t ng,
                                                    const double *__restrict__ acc, bool second) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    jz_group &gr = groups[g];
    const double *a = acc + (size_t)g * 8;
    const double c = (double)gr.count;
    if (!second) {
        for (int d = 0; d < 3; ++d) {
            gr.cm[d] = a[d] / c;
            gr.vcm[d] = a[3 + d] / c;
        }
    } else {
        gr.r_inertia = sqrt(a[6] / c);
    }
}

// the tree's sorted points back in input order, as float [n][3]
__global__ __launch_bounds__(256) void k_cat_unsort(const float4 *__restrict__ pts4, int64_t n,
                                                    float *__restrict__ xyz) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 p = pts4[i];
    const int64_t o = __float_as_int(p.w);
    xyz[3 * o] = p.x;
    xyz[3 * o + 1] = p.y;
    xyz[3 * o + 2] = p.z;
}

__global__ __launch_bounds__(256) void k_fill_i32(int *__restrict__ p, int64_t n, int v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

extern "C" JZ_API jz_status jz_fof_catalogue(jz_tree *t, float b, int min_members,
                                             const float *vel, int32_t *label, int32_t *order,
                                             jz_group *groups, int64_t max_groups,
                                             int64_t *ngroups, void *stream) {
    jz_fail(JZ_OK, "");
    if (!t) return jz_fail(JZ_E_INVALID, "tree is NULL");
    if (!ngroups) return jz_fail(JZ_E_INVALID, "ngroups is NULL");
    *ngroups = 0;
    if (t->nsets != 1 || t->n_src >= 0)
        return jz_fail(JZ_E_INVALID, "the catalogue takes a single-set tree from jz_build");
    if (t->opts.period > 0.0f)
        return jz_fail(JZ_E_INVALID, "the catalogue is for open space (a periodic group's centre "
                       "of mass depends on how it is unwrapped)");
    if (!(b >= 0.0f) || !std::isfinite(b)) return jz_fail(JZ_E_INVALID, "b must be finite and >= 0");
    if (min_members < 1) return jz_fail(JZ_E_INVALID, "min_members must be >= 1");
    if (max_groups < 0 || (max_groups > 0 && !groups))
        return jz_fail(JZ_E_INVALID, "groups is NULL");
    const int64_t n = t->n;
    if (n > 0 && !order) return jz_fail(JZ_E_INVALID, "order is NULL");
    if (n == 0) return JZ_OK;
    hipStream_t s = (hipStream_t)stream;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) {
        (void)hipGetLastError();
        return jz_fail(JZ_E_DEVICE, "no HIP device");
    }
    struct Restore {
        int prev, dev;
        ~Restore() {
            if (prev != dev) (void)hipSetDevice(prev);
        }
    } restore{prev, t->ac.device};
    if (prev != t->ac.device) JZ_HIP(hipSetDevice(t->ac.device));
    const AllocCtx *ac = &t->ac;

    // group labels (input order)
    DBuf d_label;
    int32_t *lab = label;
    if (!lab) {
        JZ_TRY(d_label.get(ac, (size_t)n * sizeof(int32_t), s));
        lab = d_label.as<int32_t>();
    }
    const float b2 = b * b;
    JZ_TRY(run_fof(t, &b2, lab, s));

    // 1: group order
    DBuf k0, v0, k1, v1, d_count;
    JZ_TRY(k0.get(ac, (size_t)n * sizeof(uint64_t), s));
    JZ_TRY(v0.get(ac, (size_t)n * sizeof(uint32_t), s));
    JZ_TRY(k1.get(ac, (size_t)n * sizeof(uint64_t), s));
    JZ_TRY(v1.get(ac, (size_t)n * sizeof(uint32_t), s));
    JZ_TRY(d_count.get(ac, (size_t)n * sizeof(int), s));
    k_fill_i32<<<blocks_for(n, 256), 256, 0, s>>>(d_count.as<int>(), n, 0);
    k_cat_keys<<<blocks_for(n, 256), 256, 0, s>>>(lab, n, k0.as<uint64_t>(), v0.as<uint32_t>(),
                                                  d_count.as<int>());
    JZ_HIP(hipGetLastError());
    int bits = 0;
    while (bits < 31 && ((int64_t)1 << bits) < n) ++bits;
    JZ_TRY(radix_sort_pairs(ac, k0, v0, k1, v1, n, bits, s));
    JZ_HIP(hipMemcpyAsync(order, v0.p, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));

    // 2: qualifying groups
    const int nb = (int)((n + CAT_BLOCK - 1) / CAT_BLOCK);
    DBuf d_bcnt, d_boff, d_total, d_gidx;
    JZ_TRY(d_bcnt.get(ac, (size_t)nb * sizeof(int), s));
    JZ_TRY(d_boff.get(ac, (size_t)nb * sizeof(int), s));
    JZ_TRY(d_total.get(ac, sizeof(long long), s));
    JZ_TRY(d_gidx.get(ac, (size_t)n * sizeof(int), s));
    k_fill_i32<<<blocks_for(n, 256), 256, 0, s>>>(d_gidx.as<int>(), n, -1);
    k_cat_block_counts<<<nb, 256, 0, s>>>(k0.as<uint64_t>(), d_count.as<int>(), n, min_members,
                                          d_bcnt.as<int>());
    k_cat_scan<<<1, 1024, 0, s>>>(d_bcnt.as<int>(), nb, d_boff.as<int>(),
                                  d_total.as<long long>());
    k_cat_compact<<<nb, 256, 0, s>>>(k0.as<uint64_t>(), d_count.as<int>(), n, min_members,
                                     d_boff.as<int>(), groups, max_groups, d_gidx.as<int>());
    JZ_HIP(hipGetLastError());
    long long G = 0;
    JZ_HIP(hipMemcpyAsync(&G, d_total.p, sizeof(G), hipMemcpyDeviceToHost, s));
    JZ_HIP(hipStreamSynchronize(s));
    *ngroups = G;
    if (G > max_groups)
        return jz_fail(JZ_E_CAPACITY, "%lld groups have at least %d members; groups holds %lld",
                       G, min_members, (long long)max_groups);
    if (G == 0) return JZ_OK;

    // 3-4: centre of mass (and velocity), inertia radius
    DBuf d_acc, d_xyz;
    JZ_TRY(d_xyz.get(ac, (size_t)n * 3 * sizeof(float), s));
    k_cat_unsort<<<blocks_for(n, 256), 256, 0, s>>>(t->pts4.as<float4>(), n, d_xyz.as<float>());
    const float *points = d_xyz.as<float>();
    JZ_TRY(d_acc.get(ac, (size_t)G * 8 * sizeof(double), s));
    JZ_TRY(zero_words(d_acc.as<unsigned long long>(), (size_t)G * 8, s));
    for (int pass = 0; pass < 2; ++pass) {
        k_cat_sums<<<blocks_for(n, 256), 256, 0, s>>>(k0.as<uint64_t>(), v0.as<uint32_t>(), n,
                                                      d_gidx.as<int>(), points, vel, pass == 1,
                                                      groups, d_acc.as<double>());
        k_cat_finish<<<blocks_for(G, 256), 256, 0, s>>>(groups, G, d_acc.as<double>(), pass == 1);
    }
    JZ_HIP(hipGetLastError());
    JZ_HIP(hipStreamSynchronize(s));
    return JZ_OK;
}
