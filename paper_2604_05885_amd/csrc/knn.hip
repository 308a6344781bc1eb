// Exact kNN by a dual walk over the tree planes (paper: kNN section, Alg. 1-3,
// Eq. 14-16, and the implementation-details subsection on r_low ordering).
//
// Level step (one wave per work item: a receiving parent and up to 8 of its
// children; lanes = those children):
//   pass 1  FindRmax: register heap of (d_up^2, count); R = smallest radius
//           whose cumulative count reaches k (Alg. 3)
//   pass 2  count children pairs with d_low^2 <= R
//   pass 3  insert them (with r_low = d_low^2) into the next list, at an
//           offset reserved with one atomic per wave
// The paper's separate Count / prefix-sum / Insert launches become one kernel.
// Each receiver's source list is read in r_low order (sorted in LDS when
// short, in HBM before the level when long) so that the early exit
// "r_low > max over lanes of R" can drop the rest of the list.
//
// Leaf stage (one wave per receiving leaf; lanes = its query points): source
// leaves in r_low order, each staged in LDS as float4 (x, y, z, index); every
// lane keeps its top-k as packed (dist2 bits, index) u64 keys in registers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <type_traits>
#include <vector>

#include "jz_device.h"
#include "jz_internal.h"

namespace {

constexpr int LCAP = 256;  // list entries staged (and sorted) in LDS per wave
constexpr int prev_pow2(int x) {
    int m = 1;
    while (m * 2 <= x) m *= 2;
    return m;
}
constexpr uint64_t PAD_KEY = (0x7f800000ull << 32) | 0xffffffffull;  // (+inf, no index)

__device__ __forceinline__ uint64_t list_key(int2 e) {
    return ((uint64_t)(uint32_t)e.y << 32) | (uint32_t)e.x;  // r_low >= 0: bits order as floats
}

// Stage a receiver's list in LDS and sort it ascending by (r_low, source).
__device__ void stage_sorted(const int2 *__restrict__ src, int len, uint64_t *L) {
    int M = 1;
    while (M < len) M <<= 1;
    for (int i = lane_id(); i < M; i += 64) L[i] = i < len ? list_key(src[i]) : ~0ull;
    wave_lds_sync();
    for (int k = 2; k <= M; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lane_id(); i < (M >> 1); i += 64) {
                const int a = ((i & ~(j - 1)) << 1) | (i & (j - 1));
                const int b = a + j;
                const uint64_t x = L[a], y = L[b];
                const bool up = (a & k) == 0;
                if ((x > y) == up) {
                    L[a] = y;
                    L[b] = x;
                }
            }
            wave_lds_sync();
        }
    }
}

// Order a receiver's list by (r_low, source). A list of at most LCAP entries
// is staged in L. A longer one, of at most scap entries, is sorted in the
// LDS scratch that begins with L (the wave's other buffers, not yet in use)
// and written back whole, in order, over its segment in HBM (the segment
// belongs to this receiver alone); its first LCAP entries stay in L. The
// segment stays a permutation of the list, so a level that is run again
// after a capacity overflow reads the same list. A list of at most
// presorted entries was already put in order in HBM (k_sort_lists): only its
// first LCAP entries are staged. Either way the list then reads in r_low
// order and the walk can stop at the first entry beyond its radius. Returns
// false (list left as it is, read unordered) for a longer list.
__device__ bool stage_list(int2 *__restrict__ gl, int len, uint64_t *S, int scap,
                           int presorted) {
    if (len > scap) {
        if (len > presorted) return false;
        for (int i = lane_id(); i < LCAP; i += 64) S[i] = list_key(gl[i]);
        wave_lds_sync();
        return true;
    }
    stage_sorted(gl, len, S);
    if (len > LCAP) {
        for (int i = lane_id(); i < len; i += 64) {
            const uint64_t e = S[i];
            gl[i] = make_int2((int)(uint32_t)e, (int)(uint32_t)(e >> 32));
        }
        // the wave reads entries from LCAP on back later, from other lanes:
        // wait until the stores have reached L2 (the wave's own, so this
        // CU's L2) and drop this CU's vector L1, which may still hold the
        // lines as they were loaded above. (A workgroup-scope fence compiles
        // to nothing in a one-wave workgroup; an agent-scope one would also
        // write back and invalidate L2, which the other XCDs never read.)
        __asm__ volatile("s_waitcnt vmcnt(0)\n\tbuffer_inv sc0" ::: "memory");
    }
    wave_lds_sync();
    return true;
}

// Lists longer than a wave can sort in its LDS scratch are put in order in
// HBM before they are walked: k_find_long collects the receivers whose list
// length lies in (min_len, mid] and in (mid, max_len], and k_sort_lists
// sorts each such list in place in LDS, one workgroup per list: one wave for
// lists of at most SORT_MID entries, SORT_WAVES waves for longer ones (up to
// SORT_MAX).
constexpr int SORT_MID = 1024;
constexpr int SORT_MAX = 8192;
constexpr int SORT_WAVES = 8;

__global__ __launch_bounds__(64) void k_find_long(const int2 *__restrict__ seg, int n,
                                                  int min_len, int mid, int max_len,
                                                  int *__restrict__ ids_a,
                                                  unsigned long long *__restrict__ count_a,
                                                  int *__restrict__ ids_b,
                                                  unsigned long long *__restrict__ count_b) {
    const int lane = lane_id();
    const int i = blk_x() * 64 + lane;
    const int len = i < n ? seg[i].y : 0;
    const bool la = len > min_len && len <= mid, lb = len > mid && len <= max_len;
    const uint64_t ma = __ballot(la), mb = __ballot(lb);
    if (ma) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(count_a, (unsigned long long)__popcll(ma));
        base = uni((unsigned long long)__shfl(base, 0, 64));
        if (la) ids_a[base + __popcll(ma & lanemask_lt())] = i;
    }
    if (mb) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(count_b, (unsigned long long)__popcll(mb));
        base = uni((unsigned long long)__shfl(base, 0, 64));
        if (lb) ids_b[base + __popcll(mb & lanemask_lt())] = i;
    }
}

// The receivers whose lists are longer than min_len, in any order: the leaf
// stage runs them first, so that these long waves overlap the rest of the
// launch instead of trailing it.
__global__ __launch_bounds__(64) void k_long_first(const int2 *__restrict__ seg, int n,
                                                   int min_len, int *__restrict__ ids,
                                                   unsigned long long *__restrict__ count) {
    const int lane = lane_id();
    const int i = blk_x() * 64 + lane;
    const bool l = i < n && seg[i].y > min_len;
    const uint64_t m = __ballot(l);
    if (!m) return;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(count, (unsigned long long)__popcll(m));
    base = uni((unsigned long long)__shfl(base, 0, 64));
    if (l) ids[base + __popcll(m & lanemask_lt())] = i;
}

// Bitonic sort of each listed segment by (r_low, source), in CAP keys of LDS,
// by NW waves. A compare-exchange step of pair distance j touches, for pair
// indices in one aligned range of PW = M / 2 / NW pairs, only the elements of
// one aligned range of 2 PW: steps with j <= PW run wave by wave without a
// workgroup barrier, so only the few steps of larger j pay one.
template <int CAP, int NW>
__global__ __launch_bounds__(64 * NW) void k_sort_lists(int2 *__restrict__ list,
                                                        const int2 *__restrict__ seg,
                                                        const int *__restrict__ ids,
                                                        const unsigned long long *__restrict__ count) {
    __shared__ uint64_t s[CAP];
    constexpr int NT = 64 * NW;
    const int tid = tid_x(), lane = tid & 63, w = tid >> 6;
    const long long nl = (long long)*count;
    for (long long jl = blk_x(); jl < nl; jl += nblk_x()) {
        const int2 sg = seg[ids[jl]];
        int2 *g = list + sg.x;
        const int len = sg.y;
        int M = 2 * NW;
        while (M < len) M <<= 1;
        for (int i = tid; i < M; i += NT) s[i] = i < len ? list_key(g[i]) : ~0ull;
        __syncthreads();
        const int PW = (M >> 1) / NW;
        for (int k = 2; k <= M; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                const bool wide = j > PW;
                // a wide step reads what other waves wrote in the steps before
                if (wide) __syncthreads();
                const int i0 = wide ? tid : w * PW + lane;
                const int i1 = wide ? (M >> 1) : (w + 1) * PW;
                const int di = wide ? NT : 64;
                for (int i = i0; i < i1; i += di) {
                    const int a = ((i & ~(j - 1)) << 1) | (i & (j - 1));
                    const int b = a + j;
                    const uint64_t x = s[a], y = s[b];
                    const bool up = (a & k) == 0;
                    if ((x > y) == up) {
                        s[a] = y;
                        s[b] = x;
                    }
                }
                if (wide || NW == 1) __syncthreads();
                else wave_lds_sync();
            }
        }
        __syncthreads();
        for (int i = tid; i < len; i += NT) {
            const uint64_t e = s[i];
            g[i] = make_int2((int)(uint32_t)e, (int)(uint32_t)(e >> 32));
        }
        __syncthreads();
    }
}

// Entry t of a receiver's list: from LDS for the first LCAP entries of an
// ordered list, else from HBM.
__device__ __forceinline__ void list_entry(bool staged, const uint64_t *L, const int2 *g, int t,
                                           int &src, float &rl) {
    if (staged && t < LCAP) {
        const uint64_t e = L[t];
        src = (int)(uint32_t)e;
        rl = __uint_as_float((uint32_t)(e >> 32));
    } else {
        const int2 e = g[t];
        src = e.x;
        rl = __int_as_float(e.y);
    }
}

// Register heap of (radius, count), sorted by radius. Inserting pushes the
// largest entry out; its count is merged into the last slot at its (larger)
// radius, which keeps "at least C points within radius r" true for every
// prefix.
template <int NR>
__device__ __forceinline__ void heap_insert(float (&hr)[NR], int (&hc)[NR], float r, int c) {
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const bool sw = r < hr[i];
        const float tr = sw ? hr[i] : r;
        const int tc = sw ? hc[i] : c;
        hr[i] = sw ? r : hr[i];
        hc[i] = sw ? c : hc[i];
        r = tr;
        c = tc;
    }
    if (c > 0) {
        hr[NR - 1] = r;
        hc[NR - 1] += c;
    }
}

// smallest radius whose cumulative count reaches k (+inf if the total is < k)
template <int NR>
__device__ __forceinline__ float radius_of_count(const float (&hr)[NR], const int (&hc)[NR],
                                                 int k) {
    int acc = 0;
    float R = INFINITY;
    bool found = false;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        acc += hc[i];
        if (!found && acc >= k) {
            R = hr[i];
            found = true;
        }
    }
    return R;
}

constexpr int NR_HEAP = 8;
constexpr int FCAP = 128;  // source children staged per batch

// Walk the (r_low-sorted) source list of one receiving parent in batches: the
// children of consecutive sources are copied into one LDS buffer (their node
// records in F, their indices in FI) until FCAP children; a source with more
// children than FCAP is split over several batches. Sources whose r_low
// exceeds rw() end the walk. fn(nF, fi) then processes the nF staged children
// (fi: their indices).
// The walk is pipelined one batch deep: the next batch is chosen, its indices
// written to the other half of FI and its node records loaded into registers
// before fn runs on the current one, and copied into F after it, so that the
// record loads overlap fn instead of stalling every batch. The next batch is
// chosen with rw() as it was before fn; where rw() shrinks during fn (the
// FindRmax pass) that may take sources a later check would have dropped, which
// only adds candidates to an upper bound. The list entries (and children
// ranges) of the batch after that are loaded meanwhile too.
// With separate query and source points (scnt != nullptr), a staged record's
// count is replaced by its number of source points.
template <class RW, class FN>
__device__ __forceinline__ void for_source_batches(bool staged, const uint64_t *L,
                                                   const int2 *gl, int len,
                                                   const int *__restrict__ par_spl,
                                                   const Node *__restrict__ nodes,
                                                   const int *__restrict__ scnt, Node *F, int *FI,
                                                   RW &&rw, FN &&fn) {
    static_assert(FCAP == 128, "two node records per lane");
    const int lane = lane_id();
    int t = 0, skip = 0;
    // entry t + lane of the list: its r_low and the range of its children
    bool valid = false;
    int s0 = 0, cnt = 0;
    float rl = 0.0f;
    auto load = [&](int t0) {
        valid = t0 + lane < len;
        if (valid) {
            int src;
            list_entry(staged, L, gl, t0 + lane, src, rl);
            s0 = par_spl[src];
            cnt = par_spl[src + 1] - s0;
        }
    };
    // the prepared batch: nN children (0: the walk ends), indices in FI half
    // `half`, the records of positions lane and lane + 64 as two halves each
    int nN = 0, half = 0;
    float4 r0a = make_float4(0, 0, 0, 0), r0b = r0a, r1a = r0a, r1b = r0a;
    auto fetch_rec = [&](int x, float4 &ra, float4 &rb) {
        const float4 *rec = reinterpret_cast<const float4 *>(nodes + x);
        ra = rec[0];
        rb = rec[1];
        if (scnt) rb.w = __int_as_float(scnt[x]);  // Node.count is the last word
    };
    auto prepare = [&](float Rw) {
        int *fi = FI + half * FCAP;
        nN = 0;
        if (t >= len) return;
        const int b0 = s0 + (lane == 0 ? skip : 0);
        const int c_all = cnt - (lane == 0 ? skip : 0);
        const bool ok = valid && (!staged || rl <= Rw);
        const uint64_t okm = __ballot(ok);  // sorted by r_low: a prefix of the lanes
        const int nok = ~okm ? __ffsll((unsigned long long)~okm) - 1 : 64;
        if (nok == 0) {
            t = len;
            return;
        }
        const int c = lane < nok ? c_all : 0;
        const int incl = wave_incl_scan(c);
        const int ntake = __popcll(__ballot(lane < nok && incl <= FCAP));
        if (ntake == 0) {
            // the first source alone overflows the buffer: take FCAP of its
            // children (the loaded entries stay those of position t)
            const int f0 = uni(__shfl(b0, 0, 64));
            for (int f = lane; f < FCAP; f += 64) fi[f] = f0 + f;
            nN = FCAP;
            skip += FCAP;
        } else {
            // lane q < ntake lists the indices of its source's children
            if (lane < ntake) {
                const int off = incl - c;
                for (int q = 0; q < c; ++q) fi[off + q] = b0 + q;
            }
            nN = uni(__shfl(incl, ntake - 1, 64));
            t += ntake;
            skip = 0;
        }
        wave_lds_sync();
        // every lane loads records lane and lane + 64 (independent loads
        // instead of one chain per source)
        if (lane < nN) fetch_rec(fi[lane], r0a, r0b);
        if (lane + 64 < nN) fetch_rec(fi[lane + 64], r1a, r1b);
        if (ntake != 0) load(t);
    };
    auto commit = [&]() {
        float4 *f4 = reinterpret_cast<float4 *>(F);
        if (lane < nN) {
            f4[2 * lane] = r0a;
            f4[2 * lane + 1] = r0b;
        }
        if (lane + 64 < nN) {
            f4[2 * lane + 128] = r1a;
            f4[2 * lane + 129] = r1b;
        }
    };
    load(0);
    prepare(uni(rw()));
    commit();
    wave_lds_sync();
    while (nN > 0) {
        const int nF = nN;
        const int *fcur = FI + half * FCAP;
        half ^= 1;
        prepare(uni(rw()));
        fn(nF, fcur);
        wave_lds_sync();
        commit();
        wave_lds_sync();
    }
}

// The walk's work items: a receiving parent with more than cb children is
// split into items of cb children (each a wave of its own, reading the
// parent's list), so that the few parents with many children and long lists
// do not leave one wave running long after the rest of the level, and so
// that the upper levels, with few parents, still fill the device. cb is at
// most WALK_CB.
constexpr int WALK_CB = 8;
constexpr int WALK_CB_UP = 2;
// A parent whose list is longer than WALK_LONG entries takes items of at most
// WALK_CB_LONG children: such items run many times longer than the rest and
// would otherwise be the tail of the level.
constexpr int WALK_LONG = 1024;
constexpr int WALK_CB_LONG = 2;
__device__ __forceinline__ int item_cb(int cb, int len) {
    return len > WALK_LONG ? min(cb, WALK_CB_LONG) : cb;
}

__global__ __launch_bounds__(64) void k_walk_items(const int *__restrict__ par_spl, int n_par,
                                                   int cb, const int2 *__restrict__ seg_in,
                                                   int2 *__restrict__ items,
                                                   unsigned long long *__restrict__ count) {
    const int lane = lane_id();
    const int P = blk_x() * 64 + lane;
    int c0 = 0, nb = 0, cbe = cb;
    if (P < n_par) {
        c0 = par_spl[P];
        cbe = item_cb(cb, seg_in[P].y);
        nb = max(1, (par_spl[P + 1] - c0 + cbe - 1) / cbe);
    }
    const int incl = wave_incl_scan(nb);
    const int tot = uni(__shfl(incl, 63, 64));
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(count, (unsigned long long)tot);
    base = uni((unsigned long long)__shfl(base, 0, 64));
    for (int b = 0; b < nb; ++b)
        items[base + (unsigned long long)(incl - nb + b)] = make_int2(P, c0 + b * cbe);
}

// Level step of the kNN walk: one wave per work item (a receiving parent and
// up to WALK_CB of its children). The children are spread over the lanes with G = 64 / (children, rounded up to a power of 2)
// lanes per child; the G lanes of a child split the staged source children
// between them (slice sl takes f = sl, sl + G, ...).
//   pass 1  FindRmax: a register heap of (d_up^2, count) per lane; the G
//           heaps of a child are then merged exactly in LDS (R = smallest
//           radius whose cumulative count over all entries reaches k)
//   pass 2  count pairs with d_low^2 <= R
//   pass 3  insert them (with r_low = d_low^2) at offsets reserved with one
//           atomic per wave; a child's entries are contiguous.
template <bool PER>
__global__ __launch_bounds__(64 * WPB) void k_knn_step(
    const int2 *__restrict__ items, const unsigned long long *__restrict__ n_items, int cb,
    const int2 *__restrict__ seg_in, int2 *__restrict__ list_in,
    const int *__restrict__ par_spl, const Node *__restrict__ nodes, int k,
    int2 *__restrict__ seg_out, int2 *__restrict__ list_out,
    unsigned long long *__restrict__ ctr, long long cap, unsigned long long *overflow,
    int sort_cap, int presorted, const int *__restrict__ scnt, float Lp,
    float *__restrict__ rout) {
    // one block per wave: the staged list (LCAP entries), then the staged
    // source children (FCAP records, and their indices for two batches); before the walk the
    // whole block is the scratch in which a longer list is sorted
    constexpr int RAW = LCAP + FCAP * (int)(sizeof(Node) / 8) + FCAP;
    __shared__ __align__(16) uint64_t s_raw[WPB][RAW];
    const int w = WPB == 1 ? 0 : uni((int)(tid_x() >> 6)), lane = tid_x() & 63;
    // work item I: receiving parent it.x, its children from it.y (at most
    // item_cb(cb, list length) of them)
    const int I = xcd_block(blk_x(), nblk_x()) * WPB + w;
    if (I >= (int)uni(*n_items)) return;
    const int2 it = items[I];
    const int P = uni(it.x);
    const int2 sg = seg_in[P];
    int2 *gl = list_in + uni(sg.x);
    const int len = uni(sg.y);
    const int c0 = uni(it.y), c1 = uni(min(par_spl[P + 1], it.y + item_cb(cb, len)));
    uint64_t *L = s_raw[w];
    Node *F = reinterpret_cast<Node *>(L + LCAP);
    int *FI = reinterpret_cast<int *>(L + LCAP + FCAP * (int)(sizeof(Node) / 8));
    const bool staged = stage_list(gl, len, L, min(sort_cap, prev_pow2(RAW)), presorted);

    for (int cb = c0; cb < c1; cb += 64) {
        const int nc = min(64, c1 - cb);
        // G = largest power of two with nc * G <= 64
        int lg = 0;
        while ((nc << (lg + 1)) <= 64) ++lg;
        const int G = 1 << lg;
        const int ci = lane >> lg, sl = lane & (G - 1);
        const int c = cb + (ci < nc ? ci : 0);
        const Node me = nodes[c];
        // with separate point types, a child without query points receives
        // nothing
        const bool act = ci < nc && (!scnt || me.count > scnt[c]);
        float hr[NR_HEAP];
        int hc[NR_HEAP];
#pragma unroll
        for (int i = 0; i < NR_HEAP; ++i) {
            hr[i] = INFINITY;
            hc[i] = 0;
        }
        float R = INFINITY;
        // pass 1: FindRmax over this lane's slice
        for_source_batches(
            staged, L, gl, len, par_spl, nodes, scnt, F, FI,
            [&]() { return wave_max_f(act ? R : -INFINITY); },
            [&](int nF, const int *) {
                for (int f = sl; f < nF; f += G) {
                    const Node o = F[f];
                    const float r = box_up2_m<PER>(me, o, Lp);
                    if (act && r < R && o.count > 0) {
                        heap_insert<NR_HEAP>(hr, hc, r, o.count);
                        R = fminf(R, radius_of_count<NR_HEAP>(hr, hc, k));
                    }
                }
                // each lane's radius already bounds its child (k points of its
                // slice lie within it), so the child's lanes share the smallest
                R = group_min_f(R, G);
            });
        if (G > 1) {
            // exact merge of the G heaps of each child (LDS scratch: F's buffer)
            float *mr = reinterpret_cast<float *>(F);
            int *mc = reinterpret_cast<int *>(F) + NR_HEAP * 64;
#pragma unroll
            for (int i = 0; i < NR_HEAP; ++i) {
                mr[i * 64 + lane] = hr[i];
                mc[i * 64 + lane] = hc[i];
            }
            wave_lds_sync();
            float best = INFINITY;
            const int g0 = ci << lg;
            if (act) {
                for (int e = sl; e < G * NR_HEAP; e += G) {
                    const float re = mr[(e % NR_HEAP) * 64 + g0 + e / NR_HEAP];
                    if (!(re < best)) continue;
                    int acc = 0;
                    for (int g = 0; g < G; ++g)
                        for (int i = 0; i < NR_HEAP; ++i)
                            if (mr[i * 64 + g0 + g] <= re) acc += mc[i * 64 + g0 + g];
                    if (acc >= k) best = re;
                }
            }
            best = group_min_f(best, G);
            R = fminf(best, R);
            wave_lds_sync();
        }
        // the leaf level keeps each child's radius for the leaf stage: k
        // points lie within R of every point of the child
        if (rout && act && sl == 0) rout[c] = R;
        const float Rw = uni(wave_max_f(act ? R : -INFINITY));
        // pass 2: count
        int cnt = 0;
        for_source_batches(
            staged, L, gl, len, par_spl, nodes, scnt, F, FI, [&]() { return Rw; },
            [&](int nF, const int *) {
                for (int f = sl; f < nF; f += G) {
                    const Node o = F[f];
                    cnt += (act && o.count > 0 && box_low2_m<PER>(me, o, Lp) <= R) ? 1 : 0;
                }
            });
        // reserve: lanes are child-major, so a wave scan gives contiguous segments
        const int incl = wave_incl_scan(cnt);
        const int total = uni(__shfl(incl, 63, 64));
        // segment in arena I % LIST_ARENAS (cap entries each)
        const int ar = I & (LIST_ARENAS - 1);
        unsigned long long lb = 0;
        if (lane == 0) lb = atomicAdd(ctr + ar, (unsigned long long)total);
        lb = uni((unsigned long long)__shfl(lb, 0, 64));
        const unsigned long long base = (unsigned long long)ar * (unsigned long long)cap + lb;
        const bool ok = (long long)lb + total <= cap;
        // an overflowing level makes every list below it incomplete: flag it,
        // so that the leaf stage of this attempt exits at once
        if (!ok && lane == 0) *overflow = 1;
        const int gfirst = (ci << lg), glast = gfirst + G - 1;
        const int gstart = __shfl(incl - cnt, gfirst & 63, 64);
        const int gend = __shfl(incl, glast & 63, 64);
        if (ci < nc && sl == 0)
            seg_out[c] = ok ? make_int2((int)((long long)base + gstart), gend - gstart)
                            : make_int2(0, 0);
        if (!ok) continue;
        // pass 3: insert
        long long wp = (long long)base + (incl - cnt);
        for_source_batches(
            staged, L, gl, len, par_spl, nodes, scnt, F, FI, [&]() { return Rw; },
            [&](int nF, const int *fi) {
                for (int f = sl; f < nF; f += G) {
                    const Node o = F[f];
                    const float lo = box_low2_m<PER>(me, o, Lp);
                    if (act && o.count > 0 && lo <= R) {
                        list_out[wp] = make_int2(fi[f], __float_as_int(lo));
                        ++wp;
                    }
                }
            });
    }
}

// Top-k keys are (dist2 bits << 32 | index). dist2 >= 0 is never NaN, so the
// key's top 12 bits are never 0x7FF and, read as an IEEE double, every key is
// a non-negative non-NaN number (small keys are subnormal doubles, which this
// file's kernels keep). For such doubles the numeric order is the unsigned
// integer order of the bits, so the lists are kept as doubles and ordered
// with v_min_f64 / v_max_f64 (one instruction each, no 64-bit integer
// compare-and-select pairs).
__device__ __forceinline__ double key_of(float dd, int idx) {
    return __builtin_bit_cast(double, ((uint64_t)__float_as_uint(dd) << 32) | (uint32_t)idx);
}
__device__ __forceinline__ uint64_t bits_of(double k) { return __builtin_bit_cast(uint64_t, k); }
__device__ __forceinline__ float key_dist(double k) {
    return __uint_as_float((uint32_t)(bits_of(k) >> 32));
}

constexpr int next_pow2(int k) {
    int m = 1;
    while (m < k) m <<= 1;
    return m;
}

// An ascending list of K keys held in one or two vector registers tuples of
// at most 16 doubles. As a vector the list is one register tuple that the
// compiler updates in place; as an array of doubles every insertion renames
// the entries and loops pay a copy of the whole list per iteration.
template <int K>
struct TopK {
    static constexpr int W = K <= 16 ? next_pow2(K) : 16;
    static constexpr int NV = (K + W - 1) / W;
    typedef double vec __attribute__((ext_vector_type(W)));
    vec v[NV];
    __device__ __forceinline__ double get(int i) const { return v[i / W][i % W]; }
    __device__ __forceinline__ void set(int i, double x) { v[i / W][i % W] = x; }
};

// Insert key into the ascending list b (the largest entry falls off).
// Inserting the padding key leaves b unchanged, so callers insert
// unconditionally instead of branching. Each slot computes the carried
// maximum first and then the slot's minimum in place; the scheduling fence
// keeps that order, which lets the register allocator update the list in
// place (with the maxima hoisted, it rotates the list through other
// registers and pays a copy of every entry per insertion).
template <int K>
__device__ __forceinline__ void topk_insert(TopK<K> &b, double key) {
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const double e = b.get(i);
        const double hi = __builtin_fmax(key, e);
        b.set(i, __builtin_fmin(e, key));
        key = hi;
        __builtin_amdgcn_sched_barrier(0);
    }
}

constexpr int SB = 16;        // source leaves examined per batch
constexpr int TILE_PTS = 256; // source points staged per batch (positions fit a byte)
constexpr int CQ = 32;        // queued candidate positions per lane
constexpr int CH = 8;         // tile positions a lane scans between queue checks

// LDS slot of tile position j: inside each chunk of 8 positions the slots are
// permuted by the chunk's low 3 bits, so that lanes reading the same position
// of different chunks at once spread over the LDS banks (unpermuted, every
// chunk starts at a multiple of 128 bytes and all of them meet in one bank
// group).
__device__ __forceinline__ int tslot(int j) { return j ^ ((j >> 3) & 7); }


// Keep the K smallest of two ascending key lists a and b in a (ascending).
// With both lists padded to M = next power of two, min(a[i], b[M-1-i]) is a
// bitonic sequence holding the M smallest of the padded union (so the K
// smallest of a and b); a bitonic sorter then orders it.
template <int K>
__device__ __forceinline__ void merge_topk(TopK<K> &a, const TopK<K> &b) {
    constexpr int M = next_pow2(K);
    const double pad = __builtin_bit_cast(double, PAD_KEY);
    double c[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const double x = i < K ? a.get(i) : pad;
        const double y = (M - 1 - i) < K ? b.get(M - 1 - i) : pad;
        c[i] = __builtin_fmin(x, y);
    }
#pragma unroll
    for (int d = M / 2; d > 0; d >>= 1) {
#pragma unroll
        for (int i = 0; i < M; ++i) {
            if ((i & d) == 0) {
                const double x = c[i], y = c[i + d];
                c[i] = __builtin_fmin(x, y);
                c[i + d] = __builtin_fmax(x, y);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < K; ++i) a.set(i, c[i]);
}

// Sort C keys ascending in registers (bitonic sorting network, C a power of 2).
template <int C>
__device__ __forceinline__ void sort_keys(double (&a)[C]) {
#pragma unroll
    for (int k = 2; k <= C; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < C; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    const double x = a[i], y = a[l];
                    const double lo = __builtin_fmin(x, y), hi = __builtin_fmax(x, y);
                    a[i] = (i & k) == 0 ? lo : hi;
                    a[l] = (i & k) == 0 ? hi : lo;
                }
            }
        }
    }
}

// Merge an ascending chunk of C keys into the top-k list (as merge_topk, the
// chunk padded to M with padding keys).
template <int K, int C>
__device__ __forceinline__ void merge_chunk(TopK<K> &a, const double (&ch)[C]) {
    constexpr int M = next_pow2(K);
    if constexpr (M == K) {
        // in place: only the last min(C, M) entries meet a chunk key (a
        // chunk longer than the list contributes its M smallest keys)
#pragma unroll
        for (int i = (M > C ? M - C : 0); i < M; ++i)
            a.set(i, __builtin_fmin(a.get(i), ch[M - 1 - i]));
#pragma unroll
        for (int d = M / 2; d > 0; d >>= 1) {
#pragma unroll
            for (int i = 0; i < M; ++i) {
                if ((i & d) == 0) {
                    const double x = a.get(i), y = a.get(i + d);
                    a.set(i, __builtin_fmin(x, y));
                    a.set(i + d, __builtin_fmax(x, y));
                }
            }
        }
        return;
    }
    const double pad = __builtin_bit_cast(double, PAD_KEY);
    double c[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const double x = i < K ? a.get(i) : pad;
        c[i] = (M - 1 - i) < C ? __builtin_fmin(x, ch[M - 1 - i]) : x;
    }
#pragma unroll
    for (int d = M / 2; d > 0; d >>= 1) {
#pragma unroll
        for (int i = 0; i < M; ++i) {
            if ((i & d) == 0) {
                const double x = c[i], y = c[i + d];
                c[i] = __builtin_fmin(x, y);
                c[i + d] = __builtin_fmax(x, y);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < K; ++i) a.set(i, c[i]);
}

// Leaf stage, one wave per receiving leaf. A leaf of at most 16 (32) points
// gives each query 4 (2) lanes; the lanes of a query scan interleaved slices
// of every staged tile, keep their own top-k, and prune with the smallest
// k-th distance of the group (the merged k-th can only be smaller), and their
// lists are merged at the end.
// Source leaves are taken in r_low order, in batches: the Node records of up
// to SB sources are read together; each lane marks the sources its query can
// still reach (point-to-box bound <= the group's k-th distance); the points of
// the sources some lane needs are staged together in one LDS tile. The walk
// stops at the first source whose r_low exceeds every query's k-th distance.
// Candidates within the k-th distance are queued as tile positions and
// inserted into the register top-k in rounds, so insert time follows the
// busiest lane rather than every accepted candidate of any lane.
//
// k > 32 takes several passes (the paper's LeafToLeaf with at most 32
// neighbours per call, called again for the next ones): a pass with LO finds
// the K smallest keys strictly above the last key of the previous pass (read
// back from column col0 - 1 of the output row), so that equal distances
// continue by index. A pass writes columns [col0, col0 + kw) of rows of
// out_stride entries.
template <int K, bool LO, bool PER>
__global__ __launch_bounds__(64 * WPB) void k_leaf_knn(
    const int2 *__restrict__ seg, int2 *__restrict__ list, const Node *__restrict__ leaves,
    const float4 *__restrict__ pts, int n_leaves, const int *__restrict__ leaf_base,
    int32_t *__restrict__ out_idx, float *__restrict__ out_d2,
    unsigned long long *__restrict__ stats, const unsigned long long *__restrict__ overflow,
    int sort_cap, int presorted, int out_stride, int col0, int kw,
    const int *__restrict__ scnt0, int src_hi, int qry_lo, float Lp,
    const float *__restrict__ rleaf, const int *__restrict__ first,
    const unsigned long long *__restrict__ n_first, int first_len) {
    // Lp: period of the cube (PER), Lh its half
    const float Lh = 0.5f * Lp;
    // one block per wave: the staged list (LCAP entries), the point tile,
    // the (lo, hi) box of every 8 tile positions and the candidate queues;
    // before the walk the whole block is the scratch in which a longer list
    // is sorted
    constexpr int O_TILE = LCAP, O_BOX = O_TILE + TILE_PTS * 2, O_Q = O_BOX + TILE_PTS / 8 * 4;
    constexpr int RAW = O_Q + CQ * 64 / 8;
    __shared__ __align__(16) uint64_t s_raw[WPB][RAW];
    __shared__ Node s_nodes[WPB][SB];
    __shared__ int s_offs[WPB][SB + 1];
    __shared__ int s_sc[WPB][SB];
    const int w = WPB == 1 ? 0 : uni((int)(tid_x() >> 6)), lane = tid_x() & 63;
    // the first waves take the leaves with lists longer than first_len (in
    // `first`), the others every leaf in order except those
    const int wv = xcd_block(blk_x(), nblk_x()) * WPB + w;
    const int nfirst = (int)uni(*n_first);
    int A;
    if (wv < nfirst) {
        A = uni(first[wv]);
    } else {
        A = wv - nfirst;
        if (A >= n_leaves || uni(seg[A].y) > first_len) return;
    }
    // a level of this attempt overflowed (it is rerun): nothing to do
    if (*overflow) return;
    const Node a = leaves[A];
    uint64_t *L = s_raw[w];
    // The leaf's query points: all its points, or, with separate point types
    // (qry_lo > 0), those with index >= qry_lo; query j sits at leaf
    // position sel[j] (selected through the LDS queue area, unused so far).
    int acount = uni(a.count);
    const bool types = qry_lo > 0;
    const uint8_t *sel = reinterpret_cast<const uint8_t *>(L + O_Q);
    if (types) {
        const bool isq = lane < acount && __float_as_int(pts[a.start + lane].w) >= qry_lo;
        const uint64_t qm = __ballot(isq);
        if (isq) reinterpret_cast<uint8_t *>(L + O_Q)[__popcll(qm & lanemask_lt())] = (uint8_t)lane;
        acount = uni((int)__popcll(qm));
        if (acount == 0) return;
        wave_lds_sync();
    }
    const int lgS = acount <= 16 ? 2 : (acount <= 32 ? 1 : 0);  // log2 lanes per query
    const int q = lane & ((64 >> lgS) - 1), h = lane >> (6 - lgS);
    const bool act = q < acount;
    const int qpos = types ? (int)sel[act ? q : 0] : (act ? q : 0);
    const float4 me = pts[a.start + qpos];
    const int64_t row = (int64_t)__float_as_int(me.w) - qry_lo;
    const int base = leaf_base ? leaf_base[A] : 0;
    // keys at or below lo (and distances below lo_d) belong to earlier passes
    double lo = -1.0;
    float lo_d = 0.0f;
    if constexpr (LO) {
        if (act) {
            const int pi = out_idx[row * out_stride + col0 - 1];
            const float pd = out_d2[row * out_stride + col0 - 1];
            lo = pi < 0 ? __builtin_bit_cast(double, PAD_KEY) : key_of(pd, pi + base);
            lo_d = pi < 0 ? INFINITY : pd;
        }
    }
    const int2 sg = seg[A];
    int2 *gl = list + uni(sg.x);
    const int len = uni(sg.y);
    float4 *tile = reinterpret_cast<float4 *>(L + O_TILE);
    float4 *cbox = reinterpret_cast<float4 *>(L + O_BOX);
    Node *nb = s_nodes[w];
    int *offs = s_offs[w];
    int *sc = s_sc[w];  // source points of each batch source
    const bool staged = stage_list(gl, len, L, min(sort_cap, prev_pow2(RAW)), presorted);

    const double pad = __builtin_bit_cast(double, PAD_KEY);
    TopK<K> best;
#pragma unroll
    for (int i = 0; i < K; ++i) best.set(i, pad);
    unsigned evals = 0, visited = 0, rounds = 0, steps = 0;
    // candidate queue of this lane: positions at q0, q0 + 64, ... up to qp
    // (LDS-typed pointers: 32-bit arithmetic instead of 64-bit)
    typedef __attribute__((address_space(3))) uint8_t lds_u8;
    lds_u8 *const q0 = (lds_u8 *)(reinterpret_cast<uint8_t *>(L + O_Q) + lane);
    lds_u8 *qp = q0;
    const lds_u8 *const qlim = q0 + 64 * (CQ - CH);

    // the group's k-th distance: an upper bound of the query's final k-th
    // the walk's radius of this leaf: the k-th distance of each of its
    // points is at most R (k = all passes' neighbours, so it bounds every
    // pass), so nothing farther is ever needed
    const float Rleaf = uni(rleaf[A]);
    auto group_kth = [&]() __attribute__((always_inline)) {
        float v = key_dist(best.get(K - 1));
        if (lgS >= 1) v = fminf(v, swap32_f(v));
        if (lgS >= 2) v = fminf(v, swap16_f(v));
        return fminf(v, Rleaf);
    };
    // insert the queued candidates of every lane into its top-k: 8 at a time,
    // sorted in registers and merged (the busiest lane sets the trip count,
    // so batches of 8 cost far less than one insertion per candidate)
    // (inlined: outlined, the list it updates would live in scratch memory)
    auto drain = [&]() __attribute__((always_inline)) {
        const int qn = (int)(qp - q0) >> 6;
        // a scalar trip count (a loop on a ballot compiles to a divergent
        // loop, whose exit handling copies the list every round)
        const int nr = uni(wave_max_i(qn));
        for (int c = 0; c < nr; c += 8) {
            rounds += 8;
            double ch[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                // slots are read unconditionally (branches around the reads
                // would make the compiler copy the list)
                // (a slot past the lane's count holds a stale byte: still a
                // tile position, and its key is replaced by the padding key)
                const int slot = min(c + u, CQ - 1);
                const int qv = q0[64 * slot];
                const float4 s = tile[qv];
                const float dd = dist2_m<PER>(me.x, me.y, me.z, s.x, s.y, s.z, Lp, Lh);
                const double kk = key_of(dd, __float_as_int(s.w));
                ch[u] = (c + u < qn && (!LO || kk > lo)) ? kk : pad;
            }
            sort_keys<8>(ch);
            merge_chunk<K, 8>(best, ch);
        }
        qp = q0;
    };

    // The list entries of the next batch window and their Node records are
    // fetched one batch ahead (into registers of lanes 0..SB-1), so the Node
    // loads overlap the current batch's work.
    int pf_src = 0, pf_sc = 0;
    float pf_rl = INFINITY;
    bool pf_ok = false;
    float4 pf_lo = make_float4(0, 0, 0, 0), pf_hi = pf_lo;  // the Node record's two halves
    auto fetch = [&](int t0, int cnt) __attribute__((always_inline)) {
        pf_ok = lane < cnt && t0 + lane < len;
        if (pf_ok) {
            list_entry(staged, L, gl, t0 + lane, pf_src, pf_rl);
            const float4 *rec = reinterpret_cast<const float4 *>(leaves + pf_src);
            pf_lo = rec[0];
            pf_hi = rec[1];
            pf_sc = scnt0 ? scnt0[pf_src] : __float_as_int(pf_hi.w);
        }
    };
    // the first batch is one source, so that the top-k fills from the
    // nearest leaf before anything else is filtered against it
    fetch(0, 1);
    int t = 0;
    while (t < len) {
        float kth = group_kth();
        const float Rw = uni(wave_max_f(act ? kth : -INFINITY));
        // sources t .. t + nb_n - 1 of this batch: the window's entries with
        // r_low <= Rw (a prefix, the list being sorted by r_low)
        const bool inb = pf_ok && (!staged || pf_rl <= Rw);
        const uint64_t inmask = __ballot(inb);
        const int nb_n = __ffsll((unsigned long long)(~inmask)) - 1;
        if (nb_n == 0) break;
        if (lane < nb_n) {
            float4 *rec = reinterpret_cast<float4 *>(nb + lane);
            rec[0] = pf_lo;
            rec[1] = pf_hi;
            sc[lane] = pf_sc;
        }
        wave_lds_sync();
        unsigned needbits = 0;
        for (int qq = 0; qq < nb_n; ++qq)
            if (act && point_low2_m<PER>(me.x, me.y, me.z, nb[qq].lo[0], nb[qq].lo[1], nb[qq].lo[2],
                                         nb[qq].hi[0], nb[qq].hi[1], nb[qq].hi[2], Lp) <= kth)
                needbits |= 1u << qq;
        const unsigned any = uni(wave_or(needbits));
        // take needed sources in order while their points fit the tile; each
        // occupies a multiple of 8 positions, one box per 8 (every lane
        // computes the same offsets; lane 0 keeps them in LDS for the scan)
        int take = 0, npts = 0;
        int o_r[SB + 1];
        o_r[0] = 0;
        if (lane == 0) offs[0] = 0;
#pragma unroll
        for (int qq = 0; qq < SB; ++qq) {
            const bool want = qq < nb_n && take == qq;
            const int c = want && ((any >> qq) & 1u) ? (uni(sc[qq]) + 7) & -8 : 0;
            if (want && npts + c <= TILE_PTS) {
                npts += c;
                take = qq + 1;
            }
            o_r[qq + 1] = npts;
            if (lane == 0) offs[qq + 1] = npts;
        }
        // stage the taken sources' points (lane f takes point f of a source:
        // a leaf holds at most 64 points) and the bounding box of every 8
        // positions (reduced over groups of 8 lanes). Filler positions hold a
        // point at +inf with index -1: its key is the padding key, so
        // accepting it changes nothing; it is left out of the boxes.
#pragma unroll
        for (int qq = 0; qq < SB; ++qq) {
            if (qq < take && o_r[qq + 1] > o_r[qq]) {
                const int cnt = uni(nb[qq].count), st = uni(nb[qq].start);
                const int nsc = uni(sc[qq]);
                const int size = o_r[qq + 1] - o_r[qq];
                const float4 filler = make_float4(INFINITY, INFINITY, INFINITY, __int_as_float(-1));
                float4 p = filler;
                bool real = lane < cnt;
                if (real) p = pts[st + lane];
                if (types) {
                    // only the source points, packed at the front
                    real = real && __float_as_int(p.w) < src_hi;
                    const uint64_t rm = __ballot(real);
                    if (real) tile[tslot(o_r[qq] + (int)__popcll(rm & lanemask_lt()))] = p;
                    if (lane >= nsc && lane < size) tile[tslot(o_r[qq] + lane)] = filler;
                    wave_lds_sync();
                    real = lane < nsc;
                    p = real ? tile[tslot(o_r[qq] + lane)] : filler;
                } else if (lane < size) {
                    tile[tslot(o_r[qq] + lane)] = p;
                }
                float lx = real ? p.x : INFINITY, ly = real ? p.y : INFINITY,
                      lz = real ? p.z : INFINITY;
                float hx = real ? p.x : -INFINITY, hy = real ? p.y : -INFINITY,
                      hz = real ? p.z : -INFINITY;
                lx = group8_min(lx);
                ly = group8_min(ly);
                lz = group8_min(lz);
                hx = group8_max(hx);
                hy = group8_max(hy);
                hz = group8_max(hz);
                if ((lane & 7) == 0 && lane < size) {
                    // the chunk's box, and in lo.w its number of real points
                    float4 *bx = cbox + ((o_r[qq] + lane) >> 3) * 2;
                    bx[0] = make_float4(lx, ly, lz, __int_as_float(min(8, max(0, nsc - lane))));
                    bx[1] = make_float4(hx, hy, hz, 0.0f);
                }
            }
        }
        // next window
        fetch(t + take, SB);
        wave_lds_sync();
        // the S lanes of a query take positions jj + h of every S-aligned step
        auto scan = [&](auto s_const) __attribute__((always_inline)) {
            constexpr int SS = decltype(s_const)::value;
            if (t == 0) {
                // the first source (one with r_low = 0) meets an empty top-k:
                // every point is accepted, so its points are merged in sorted
                // chunks instead of being queued and inserted one by one
                constexpr int C = K < 8 ? next_pow2(K) : (K <= 16 ? 8 : 16);
                if (take == 1 && (any & 1u)) {
                    ++visited;
                    const int f0 = uni(offs[0]), f1 = uni(offs[1]);
                    for (int j0 = f0; j0 < f1; j0 += C * SS) {
                        double ch[C];
#pragma unroll
                        for (int u = 0; u < C; ++u) {
                            if (j0 + u * SS < f1) {
                                const float4 p = tile[tslot(j0 + u * SS + h)];
                                const float dd = dist2_m<PER>(me.x, me.y, me.z, p.x, p.y, p.z, Lp, Lh);
                                const double kk = key_of(dd, __float_as_int(p.w));
                                ch[u] = (!LO || kk > lo) ? kk : pad;
                            } else {
                                ch[u] = pad;
                            }
                        }
                        sort_keys<C>(ch);
                        merge_chunk<K, C>(best, ch);
                        steps += (unsigned)((min(f1, j0 + C * SS) - j0) / SS);
                    }
                    const int cnt = uni(sc[0]);
                    if (act) evals += cnt > h ? (unsigned)((cnt - h + SS - 1) / SS) : 0u;
                }
                return;
            }
            // Every lane marks the 8-position chunks of the tile its query can
            // reach (chunk box within the group's k-th distance; a chunk box
            // lies inside its source's box, so this also drops the sources the
            // query does not need), then pops its own chunks, lowest first:
            // the lanes work on different chunks at once, so a pass costs the
            // largest per-lane chunk count instead of the number of chunks any
            // lane needs. The S lanes of a query share kth and so the mask,
            // and split each chunk's positions.
            visited += (unsigned)__popc(any & ((1u << take) - 1u));
            const int nch = uni(npts >> 3);
            // In a periodic box the minimum-image wrap of a difference only
            // triggers beyond half a period: for a chunk with fl(q - lo) <= h
            // and fl(q - hi) >= -h on every axis (the rounded difference is
            // monotone in the point), no point of it wraps for this query, and
            // its distances and bound are the open ones, bit for bit. W marks
            // the chunks that may wrap; the periodic forms run only where some
            // lane has one.
            unsigned M = 0, W = 0;
            for (int c = 0; c < nch; ++c) {
                const float4 *bx = cbox + c * 2;
                const float4 blo = bx[0], bhi = bx[1];
                bool wrap = false;
                if constexpr (PER)
                    wrap = !(me.x - blo.x <= Lh && me.x - bhi.x >= -Lh && me.y - blo.y <= Lh &&
                             me.y - bhi.y >= -Lh && me.z - blo.z <= Lh && me.z - bhi.z >= -Lh);
                const float lo2 =
                    (PER && __ballot(act && wrap))
                        ? point_low2_m<PER>(me.x, me.y, me.z, blo.x, blo.y, blo.z, bhi.x, bhi.y,
                                            bhi.z, Lp)
                        : point_low2_m<false>(me.x, me.y, me.z, blo.x, blo.y, blo.z, bhi.x, bhi.y,
                                              bhi.z, Lp);
                const bool need = act && lo2 <= kth;
                M |= need ? (1u << c) : 0u;
                W |= need && wrap ? (1u << c) : 0u;
            }
            const int nit = uni(wave_max_i(__popc(M)));
            for (int it = 0; it < nit; ++it) {
                const bool has = M != 0u;
                const int c = has ? __ffs((int)M) - 1 : 0;
                M &= M - 1u;
                const float thr = has ? kth : -1.0f;
                // tslot(c * 8 + q) for q < 8 is (c * 8 | (c & 7)) ^ q, and
                // q = u * SS + h = (u * SS) ^ h: one XOR per position
                const int jb = (c * 8 | (c & 7)) ^ h;
                // (the queue pointer is kept as an address, not as an offset
                // from the lane's first slot, so no add is needed per write)
                asm volatile("" : "+v"(qp));
                auto eval = [&](auto per_const) __attribute__((always_inline)) {
                    constexpr bool P = decltype(per_const)::value;
#pragma unroll
                    for (int u = 0; u < 8 / SS; ++u) {
                        const int j = jb ^ (u * SS);
                        const float4 p = tile[j];
                        const float dd = dist2_m<P>(me.x, me.y, me.z, p.x, p.y, p.z, Lp, Lh);
                        // written always, kept only if accepted (at most CH
                        // positions per pop from qn <= CQ - CH: the slot exists)
                        *qp = (uint8_t)j;
                        qp += (dd <= thr && (!LO || dd >= lo_d)) ? 64 : 0;
                    }
                };
                if (PER && __ballot(has && ((W >> c) & 1u)))
                    eval(std::integral_constant<bool, PER>());
                else
                    eval(std::integral_constant<bool, false>());
                steps += (unsigned)(8 / SS);
                if (has) {
                    const int r = __float_as_int(cbox[c * 2].w);
                    evals += r > h ? (unsigned)((r - h + SS - 1) / SS) : 0u;
                }
                if (__ballot(qp > qlim)) {
                    drain();
                    kth = group_kth();
                }
            }
        };
        if (lgS == 2) scan(std::integral_constant<int, 4>());
        else if (lgS == 1) scan(std::integral_constant<int, 2>());
        else scan(std::integral_constant<int, 1>());
        drain();
        wave_lds_sync();
        t += take;
    }
    // merge the partial lists of a query's lanes
    if (lgS >= 1) {
        TopK<K> other;
#pragma unroll
        for (int i = 0; i < K; ++i) other.set(i, swap32_d(best.get(i)));
        merge_topk<K>(best, other);
    }
    if (lgS >= 2) {
        TopK<K> other;
#pragma unroll
        for (int i = 0; i < K; ++i) other.set(i, swap16_d(best.get(i)));
        merge_topk<K>(best, other);
    }
    if (act && h == 0) {
        int32_t *oi = out_idx + row * out_stride + col0;
        float *od = out_d2 + row * out_stride + col0;
#pragma unroll
        for (int r = 0; r < K; ++r) {
            if (r < kw) {
                const uint64_t e = bits_of(best.get(r));
                const bool none = e == PAD_KEY;
                oi[r] = none ? -1 : (int)(uint32_t)e - base;
                od[r] = none ? INFINITY : __uint_as_float((uint32_t)(e >> 32));
            }
        }
    }
    const int ev = wave_sum_i((int)evals);
    if (lane == 0) {
        unsigned long long *st = stats + (A & (STAT_SLOTS - 1));
        atomicAdd(st + 0 * STAT_SLOTS, (unsigned long long)ev);
        atomicAdd(st + 1 * STAT_SLOTS, (unsigned long long)visited);
        atomicAdd(st + 2 * STAT_SLOTS, (unsigned long long)rounds);
        atomicAdd(st + 3 * STAT_SLOTS, (unsigned long long)steps);
        if (len > LCAP) atomicAdd(st + (staged ? 4 : 5) * STAT_SLOTS, 1ull);
    }
}

typedef void (*leaf_fn)(const int2 *, int2 *, const Node *, const float4 *, int, const int *,
                        int32_t *, float *, unsigned long long *, const unsigned long long *, int,
                        int, int, int, int, const int *, int, int, float, const float *,
                        const int *, const unsigned long long *, int);

template <int K, bool LO, bool PER>
leaf_fn leaf_ptr() {
    return k_leaf_knn<K, LO, PER>;
}

template <bool PER>
leaf_fn leaf_kernel_m(int k, bool lo) {
    static const leaf_fn table[34] = {
        nullptr,
        leaf_ptr<1, false, PER>(),  leaf_ptr<2, false, PER>(),  leaf_ptr<3, false, PER>(),
        leaf_ptr<4, false, PER>(),  leaf_ptr<5, false, PER>(),  leaf_ptr<6, false, PER>(),
        leaf_ptr<7, false, PER>(),  leaf_ptr<8, false, PER>(),  leaf_ptr<9, false, PER>(),
        leaf_ptr<10, false, PER>(), leaf_ptr<11, false, PER>(), leaf_ptr<12, false, PER>(),
        leaf_ptr<13, false, PER>(), leaf_ptr<14, false, PER>(), leaf_ptr<15, false, PER>(),
        leaf_ptr<16, false, PER>(), leaf_ptr<17, false, PER>(), leaf_ptr<18, false, PER>(),
        leaf_ptr<19, false, PER>(), leaf_ptr<20, false, PER>(), leaf_ptr<21, false, PER>(),
        leaf_ptr<22, false, PER>(), leaf_ptr<23, false, PER>(), leaf_ptr<24, false, PER>(),
        leaf_ptr<25, false, PER>(), leaf_ptr<26, false, PER>(), leaf_ptr<27, false, PER>(),
        leaf_ptr<28, false, PER>(), leaf_ptr<29, false, PER>(), leaf_ptr<30, false, PER>(),
        leaf_ptr<31, false, PER>(), leaf_ptr<32, false, PER>(), leaf_ptr<32, true, PER>()};
    return table[lo ? 33 : k];
}

// The leaf kernel of one pass: K = k for k <= 32 (one pass); for k > 32 the
// first pass has K = 32 and the later ones continue after the last key of the
// pass before (LO).
leaf_fn leaf_kernel(int k, int col, bool per) {
    const int kk = k <= 32 ? k : 32;
    const bool lo = col > 0;
    return per ? leaf_kernel_m<true>(kk, lo) : leaf_kernel_m<false>(kk, lo);
}

}  // namespace

namespace {
__global__ __launch_bounds__(256) void k_zero_words(unsigned long long *__restrict__ p, size_t n) {
    for (size_t i = (size_t)blk_x() * bdim_x() + tid_x(); i < n;
         i += (size_t)nblk_x() * bdim_x())
        p[i] = 0;
}
}  // namespace

jz_status zero_words(unsigned long long *p, size_t n, hipStream_t s) {
    if (n == 0) return JZ_OK;
    k_zero_words<<<(unsigned)std::min<size_t>((n + 255) / 256, 1024), 256, 0, s>>>(p, n);
    JZ_HIP(hipGetLastError());
    return JZ_OK;
}

jz_status run_knn(jz_tree *t, int k, int32_t *idx, float *dist2, hipStream_t s,
                  const AllocCtx *scratch) {
    const AllocCtx *ac = scratch ? scratch : &t->ac;
    const int P = t->P;
    // a joint tree of source and query points: rows are the query points
    const bool joint = t->n_src >= 0;
    // periodic cube (period 0: open)
    const float period = t->opts.period;
    const bool per = period > 0.0f;
    for (int p = 0; p <= JZ_MAX_PLANES; ++p) t->st.list_entries[p] = 0;
    t->st.leaf_pairs = t->st.leaf_pairs_visited = 0;
    t->st.evaluations = 0;
    t->st.leaf_ms = t->st.total_ms = 0;
    t->st.reruns = 0;
    t->st.insert_rounds = t->st.tile_steps = 0;
    t->st.lists_sorted_long = t->st.lists_unordered = 0;
    for (int p = 0; p <= JZ_MAX_PLANES; ++p) t->st.lists_presorted[p][0] = t->st.lists_presorted[p][1] = 0;
    if (t->n == 0) return JZ_OK;

    // counters: four leaf statistics (evaluations, sources visited, insert
    // rounds, tile steps)
    // then two counters of long lists (up to SORT_MID entries, longer) per
    // walk level and for the leaf stage, and one counter of work items per
    // walk level
    DBuf d_ctr;
    const size_t c_long = ctr_words(6), c_items = c_long + 2 * (JZ_MAX_PLANES + 1);
    const size_t c_first = c_items + JZ_MAX_PLANES;  // leaves with long lists
    const size_t nctr = c_first + 1;
    JZ_TRY(d_ctr.get(ac, nctr * sizeof(unsigned long long), s));
    unsigned long long *ctr = d_ctr.as<unsigned long long>();
    JZ_TRY(zero_words(ctr, nctr, s));
    int64_t cap[JZ_MAX_PLANES];
    DBuf segs[JZ_MAX_PLANES], lists[JZ_MAX_PLANES];
    for (int p = 0; p < P; ++p) {
        cap[p] = initial_cap(t, CAP_KNN, k, p);
        JZ_TRY(segs[p].get(ac, t->L[p] * sizeof(int2), s));
    }
    // Lists longer than a wave sorts in LDS (LCAP entries in the walk, whose
    // items of one parent share its list, 1024 in the leaf stage), up to
    // sort_max, are sorted in HBM before their level.
    const int sort_max = t->opts.sort_max;
    const int walk_cap = LCAP, leaf_cap = std::min(sort_max, 1024);
    // work items of the walk (at most one per parent plus one per cb
    // children, or per WALK_CB_LONG children of a parent with a long list):
    // WALK_CB children per item at the leaf level, WALK_CB_UP
    // above it, where there are few parents
    auto cb_of = [&](int p) {
        const int64_t n_par = p == P - 1 ? t->S : t->L[p + 1];
        return p == 0 || n_par >= 4096 ? WALK_CB : WALK_CB_UP;
    };
    auto item_bound = [&](int p) {
        const int64_t n_par = p == P - 1 ? t->S : t->L[p + 1];
        return n_par + t->L[p] / std::min(cb_of(p), WALK_CB_LONG) + 1;
    };
    int64_t max_items = 0;
    for (int p = 0; p < P; ++p) max_items = std::max(max_items, item_bound(p));
    DBuf d_items;
    JZ_TRY(d_items.get(ac, (size_t)max_items * sizeof(int2), s));
    DBuf d_ids, d_rleaf, d_first;
    JZ_TRY(d_ids.get(ac, 2 * (size_t)t->L[0] * sizeof(int), s));
    JZ_TRY(d_rleaf.get(ac, (size_t)t->L[0] * sizeof(float), s));
    JZ_TRY(d_first.get(ac, (size_t)t->L[0] * sizeof(int), s));
    auto presort = [&](int2 *list, const int2 *seg, int64_t n, int min_len,
                       unsigned long long *count) {
        if (sort_max <= min_len) return;
        int *ids_a = d_ids.as<int>(), *ids_b = ids_a + t->L[0];
        const int mid = std::max(min_len, std::min(sort_max, SORT_MID));
        k_find_long<<<(unsigned)((n + 63) / 64), 64, 0, s>>>(seg, (int)n, min_len, mid, sort_max,
                                                             ids_a, count, ids_b, count + 1);
        if (mid > min_len)
            k_sort_lists<SORT_MID, 1><<<4096, 64, 0, s>>>(list, seg, ids_a, count);
        if (sort_max > mid)
            k_sort_lists<SORT_MAX, SORT_WAVES><<<512, 64 * SORT_WAVES, 0, s>>>(list, seg, ids_b,
                                                                              count + 1);
    };
    EventSet ev(jz_profiling());

    // Level p turns the list of plane p+1 (or of the super nodes) into the
    // list of plane p. On overflow, levels from the highest overflowing one
    // down are rerun with larger lists; the levels above are still valid.
    int start = P - 1;
    for (;;) {
        // the lists of the levels to (re)run: released bottom level first,
        // then acquired top level first (a scratch region handed out in
        // stack order takes them back and reuses the space)
        for (int p = 0; p <= start; ++p)
            if (lists[p].bytes < (size_t)cap[p] * sizeof(int2)) lists[p].release();
        for (int p = start; p >= 0; --p) JZ_TRY(lists[p].ensure(ac, cap[p] * sizeof(int2), s));
        if (ev.on) JZ_HIP(hipEventRecord(ev[0], s));
        for (int p = start; p >= 0; --p) {
            const bool top = p == P - 1;
            const int2 *seg_in = top ? t->knn_top_seg.as<int2>() : segs[p + 1].as<int2>();
            // the super-node list belongs to the tree (shared by every call):
            // it is never written, so long lists there are read unordered
            int2 *list_in = top ? t->knn_top_list.as<int2>() : lists[p + 1].as<int2>();
            const int *par_spl = top ? t->super_spl.as<int>() : t->spl[p + 1].as<int>();
            const int64_t n_par = top ? t->S : t->L[p + 1];
            if (!top) presort(list_in, seg_in, n_par, walk_cap, ctr + c_long + 2 * p);
            unsigned long long *n_items = ctr + c_items + p;
            k_walk_items<<<(unsigned)((n_par + 63) / 64), 64, 0, s>>>(
                par_spl, (int)n_par, cb_of(p), seg_in, d_items.as<int2>(), n_items);
            (per ? k_knn_step<true> : k_knn_step<false>)<<<blocks_for(item_bound(p), WPB),
                                                              64 * WPB, 0, s>>>(
                d_items.as<int2>(), n_items, cb_of(p), seg_in, list_in, par_spl,
                t->nodes[p].as<Node>(), k, segs[p].as<int2>(), lists[p].as<int2>(),
                ctr + (size_t)p * LIST_ARENAS, cap[p] / LIST_ARENAS, ctr + CTR_FLAG,
                top ? LCAP : walk_cap, top ? 0 : sort_max,
                joint ? t->src_cnt[p].as<int>() : nullptr, period,
                p == 0 ? d_rleaf.as<float>() : nullptr);
        }
        presort(lists[0].as<int2>(), segs[0].as<int2>(), t->L[0], leaf_cap,
                ctr + c_long + 2 * JZ_MAX_PLANES);
        k_long_first<<<(unsigned)((t->L[0] + 63) / 64), 64, 0, s>>>(
            segs[0].as<int2>(), (int)t->L[0], leaf_cap, d_first.as<int>(), ctr + c_first);
        JZ_HIP(hipGetLastError());
        // waves for every leaf plus the first ones (at most one per leaf_cap
        // + 1 list entries)
        const int64_t n_waves = t->L[0] + std::min<int64_t>(t->L[0], cap[0] / (leaf_cap + 1) + 1);
        if (ev.on) JZ_HIP(hipEventRecord(ev[1], s));
        // k <= 32: one pass; larger k: passes of 32 neighbours, each after
        // the last key of the one before
        for (int col = 0; col < k; col += 32) {
            const leaf_fn fn = leaf_kernel(k, col, per);
            fn<<<blocks_for(n_waves, WPB), 64 * WPB, 0, s>>>(
                segs[0].as<int2>(), lists[0].as<int2>(), t->nodes[0].as<Node>(),
                t->pts4.as<float4>(), (int)t->L[0], t->nsets > 1 ? t->leaf_base.as<int>() : nullptr,
                idx, dist2, ctr + CTR_STATS, ctr + CTR_FLAG, leaf_cap, sort_max, k, col,
                std::min(32, k - col), joint ? t->src_cnt[0].as<int>() : nullptr,
                joint ? (int)t->n_src : INT_MAX, joint ? (int)t->n_src : 0, period,
                d_rleaf.as<float>(), d_first.as<int>(), ctr + c_first, leaf_cap);
            JZ_HIP(hipGetLastError());
        }
        if (ev.on) JZ_HIP(hipEventRecord(ev[2], s));
        std::vector<unsigned long long> hc(nctr);
        JZ_HIP(hipMemcpyAsync(hc.data(), ctr, nctr * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, s));
        JZ_HIP(hipStreamSynchronize(s));
        int redo = -1;
        double sum[JZ_MAX_PLANES], need[JZ_MAX_PLANES];
        for (int p = P - 1; p >= 0; --p) arena_need(hc.data(), p, sum[p], need[p]);
        for (int p = start; p >= 0; --p) {
            if (need[p] <= (double)(cap[p] / LIST_ARENAS * LIST_ARENAS)) continue;
            if (need[p] > (double)INT32_MAX)
                return jz_fail(JZ_E_CAPACITY, "interaction list at plane %d needs %.0f entries "
                               "(more than 2^31-1)", p, need[p]);
            if (redo < 0) redo = p;
            const double want = need[p] * 1.15 + 1024.0;
            cap[p] = want > (double)INT32_MAX ? (int64_t)INT32_MAX : (int64_t)want;
        }
        if (redo >= 0) {
            if (!t->opts.auto_regrow)
                return jz_fail(JZ_E_CAPACITY,
                               "interaction list overflow at plane %d; list_per_node must be at "
                               "least %.1f", redo, need[redo] / (double)t->L[redo]);
            t->st.reruns++;
            start = redo;
            // clear the counters of the levels to redo, the flag and the leaf
            // statistics
            JZ_TRY(zero_words(ctr, (size_t)(start + 1) * LIST_ARENAS, s));
            JZ_TRY(zero_words(ctr + CTR_FLAG, nctr - CTR_FLAG, s));
            continue;
        }
        for (int p = 0; p < P; ++p) {
            t->st.list_entries[p] = (int64_t)sum[p];
            cap_learn(CAP_KNN, k, p, need[p] / (double)std::max<int64_t>(1, t->L[p]));
        }
        t->st.leaf_pairs = t->st.list_entries[0];
        t->st.evaluations = stat_sum(hc.data(), 0);
        t->st.leaf_pairs_visited = (int64_t)stat_sum(hc.data(), 1);
        t->st.insert_rounds = (int64_t)stat_sum(hc.data(), 2);
        t->st.tile_steps = (int64_t)stat_sum(hc.data(), 3);
        t->st.lists_sorted_long = (int64_t)stat_sum(hc.data(), 4);
        t->st.lists_unordered = (int64_t)stat_sum(hc.data(), 5);
        for (int p = 0; p <= JZ_MAX_PLANES; ++p)
            for (int j = 0; j < 2; ++j)
                t->st.lists_presorted[p][j] = (int64_t)hc[c_long + 2 * p + j];
        if (ev.on) {
            float ms = 0;
            JZ_HIP(hipEventElapsedTime(&ms, ev[1], ev[2]));
            t->st.leaf_ms = ms;
            JZ_HIP(hipEventElapsedTime(&ms, ev[0], ev[2]));
            t->st.total_ms = ms;
        }
        return JZ_OK;
    }
}
