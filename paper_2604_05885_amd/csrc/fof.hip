// Friends-of-friends by the same dual walk (paper: FoF section, Eq. 18-19).
//
// Group state: a point-level union-find `uf` over z-order indices (root =
// smallest z-index of its group, linking higher root to lower root by CAS) plus
// one "whole" flag per node and plane: a whole node's points are known to be
// connected. The paper's ParentToNode advection (Eq. 19) becomes:
//   - a child of a whole parent is whole, and its first point is pointed at
//     the parent's first point (never touched before, so a plain store);
//   - a node whose own diagonal is within the linking length is whole.
// Node pairs (pairs are unordered: the lists hold sources >= receiver):
//   discard if d_low^2 > b^2, or both whole and already one group;
//   link    if d_up^2 <= b^2 (all member pairs linked): union the first
//           points and mark both whole (each is connected through the other);
//   descend otherwise (emit the pair into the next plane's list).
// Leaves: point pairs with dist2 <= b^2 are united; a final pass writes each
// point's group label as the smallest input index of its group.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <vector>

#include "jz_device.h"
#include "jz_internal.h"

namespace {

__global__ void k_iota_n(int *__restrict__ a, int64_t n) {
    const int64_t i = (int64_t)blk_x() * bdim_x() + tid_x();
    if (i < n) a[i] = (int)i;
}

// the smallest input index of every group starts as its root's own (a root is
// a member; a point that stays a root of itself needs no update at all)
__global__ __launch_bounds__(256) void k_init_min(const float4 *__restrict__ pts, int64_t n,
                                                  int *__restrict__ minidx) {
    const int64_t i = (int64_t)blk_x() * bdim_x() + tid_x();
    if (i < n) minidx[i] = __float_as_int(pts[i].w);
}

__global__ void k_node_b2(const int *__restrict__ node_set, int64_t L,
                          const float *__restrict__ b2_set, float *__restrict__ b2n) {
    const int64_t i = (int64_t)blk_x() * bdim_x() + tid_x();
    if (i < L) b2n[i] = b2_set[node_set[i]];
}

// ParentToNode: one wave per parent, lanes over its children.
template <bool PER>
__global__ __launch_bounds__(64 * WPB) void k_fof_p2n(const int *__restrict__ par_spl,
                                                 const Node *__restrict__ nodes, int n_par,
                                                 const int *__restrict__ whole_par,
                                                 int *__restrict__ whole, int *__restrict__ uf,
                                                 float b2, const float *__restrict__ b2n, float L) {
    const int w = WPB == 1 ? 0 : uni((int)(tid_x() >> 6)), lane = tid_x() & 63;
    const int P = xcd_block(blk_x(), nblk_x()) * WPB + w;
    if (P >= n_par) return;
    const int c0 = par_spl[P], c1 = par_spl[P + 1];
    const int wp = whole_par ? whole_par[P] : 0;
    const int first = nodes[c0].start;
    for (int c = c0 + lane; c < c1; c += 64) {
        const Node me = nodes[c];
        const float bb = b2n ? b2n[c] : b2;
        const int wc = (wp || box_up2_m<PER>(me, me, L) <= bb) ? 1 : 0;
        whole[c] = wc;
        if (wp && c != c0) uf[me.start] = first;
    }
}

// whole leaves: every point points at the leaf's first point
__global__ __launch_bounds__(64 * WPB) void k_fof_l2p(const Node *__restrict__ leaves, int n_leaves,
                                                 const int *__restrict__ whole,
                                                 int *__restrict__ uf) {
    const int w = WPB == 1 ? 0 : uni((int)(tid_x() >> 6)), lane = tid_x() & 63;
    const int A = xcd_block(blk_x(), nblk_x()) * WPB + w;
    if (A >= n_leaves || !whole[A]) return;
    const Node a = leaves[A];
    for (int i = a.start + 1 + lane; i < a.start + a.count; i += 64) uf[i] = a.start;
}

// kConnected: within reach but both nodes are whole and already one group
enum PairCase { kDiscard = 0, kLinked = 1, kDescend = 2, kConnected = 3 };

template <bool PER>
__device__ __forceinline__ int fof_case(const Node &me, int c, const Node &o, int s, float bb,
                                        int *whole, int *uf, bool do_link, float &lo, float L) {
    lo = box_low2_m<PER>(me, o, L);
    if (lo > bb) return kDiscard;
    // (flags only ever go from 0 to 1 and groups only merge: values read
    // through the caches may be older, which only costs a redundant union)
    if (ld_cached(whole + c) && ld_cached(whole + s) &&
        uf_find_c(uf, me.start) == uf_find_c(uf, o.start))
        return box_up2_m<PER>(me, o, L) <= bb ? kLinked : kConnected;
    if (box_up2_m<PER>(me, o, L) <= bb) {
        if (do_link) {
            uf_union_c(uf, me.start, o.start);
            st_rel(whole + c, 1);
            st_rel(whole + s, 1);
        }
        return kLinked;
    }
    return kDescend;
}

// Node walk step: one wave per receiving parent; its children are spread over
// the lanes with G = 64 / (children, rounded up to a power of 2) lanes per
// child, the G lanes of a child splitting the staged source children between
// them. Pass A links, and counts the pairs that geometry alone sends down
// (within reach, not wholly within b); pass B re-evaluates them and writes
// those still to be descended into: the group state only merges, so pass B
// writes a subset of what pass A counted, whatever either pass read of it.
// A child's entries are placed through a counter in LDS, so its list is one
// contiguous run whichever of its lanes found them.
template <bool PER>
__global__ __launch_bounds__(64 * WPB) void k_fof_step(
    const int2 *__restrict__ seg_in, const int2 *__restrict__ list_in,
    const int *__restrict__ par_spl, const Node *__restrict__ nodes, int n_par, float b2,
    const float *__restrict__ b2n, int *__restrict__ whole, int *__restrict__ uf,
    int2 *__restrict__ seg_out, int2 *__restrict__ list_out,
    unsigned long long *__restrict__ ctr, long long cap, unsigned long long *overflow, float L) {
    __shared__ Node s_tile[WPB][64];
    __shared__ int s_emit[WPB][64];
    const int w = WPB == 1 ? 0 : uni((int)(tid_x() >> 6)), lane = tid_x() & 63;
    const int P = xcd_block(blk_x(), nblk_x()) * WPB + w;
    if (P >= n_par) return;
    const int2 sg = seg_in[P];
    const int2 *gl = list_in + uni(sg.x);
    const int len = uni(sg.y);
    const int c0 = uni(par_spl[P]), c1 = uni(par_spl[P + 1]);
    Node *tile = s_tile[w];
    int *emit = s_emit[w];
    for (int cb = c0; cb < c1; cb += 64) {
        const int nc = min(64, c1 - cb);
        // G = largest power of two with nc * G <= 64
        int lg = 0;
        while ((nc << (lg + 1)) <= 64) ++lg;
        const int G = 1 << lg;
        const int ci = lane >> lg, sl = lane & (G - 1);
        const bool act = ci < nc;
        const int c = cb + (act ? ci : 0);
        const Node me = nodes[c];
        const float bb = b2n ? b2n[c] : b2;
        int cnt = 0;
        for (int t = 0; t < len; ++t) {
            const int S = gl[t].x;
            const int s0 = par_spl[S], s1 = par_spl[S + 1];
            for (int sb = s0; sb < s1; sb += 64) {
                const int ns = min(64, s1 - sb);
                if (lane < ns) tile[lane] = nodes[sb + lane];
                wave_lds_sync();
                for (int j = sl; j < ns; j += G) {
                    const int s = sb + j;
                    if (!act || s < c) continue;
                    float lo;
                    const int k = fof_case<PER>(me, c, tile[j], s, bb, whole, uf, true, lo, L);
                    cnt += (k == kDescend || k == kConnected) ? 1 : 0;
                }
                wave_lds_sync();
            }
        }
        // reserve: lanes are child-major, so a wave scan gives each child a
        // contiguous segment
        const int incl = wave_incl_scan(cnt);
        const int total = uni(__shfl(incl, 63, 64));
        // segment in arena P % LIST_ARENAS (cap entries each)
        const int ar = P & (LIST_ARENAS - 1);
        unsigned long long lb = 0;
        if (lane == 0) lb = atomicAdd(ctr + ar, (unsigned long long)total);
        lb = uni((unsigned long long)__shfl(lb, 0, 64));
        const unsigned long long base = (unsigned long long)ar * (unsigned long long)cap + lb;
        const bool ok = (long long)lb + total <= cap;
        const int gfirst = ci << lg;
        const int gstart = __shfl(incl - cnt, gfirst & 63, 64);
        const int gend = __shfl(incl, (gfirst + G - 1) & 63, 64);
        if (!ok) {
            // lists below are incomplete: the leaf stage of this attempt exits
            if (lane == 0) *overflow = 1;
            if (act && sl == 0) seg_out[c] = make_int2(0, 0);
            continue;
        }
        const long long cpos = (long long)base + gstart;
        const int room = gend - gstart;
        emit[lane] = 0;
        wave_lds_sync();
        for (int t = 0; t < len; ++t) {
            const int S = gl[t].x;
            const int s0 = par_spl[S], s1 = par_spl[S + 1];
            for (int sb = s0; sb < s1; sb += 64) {
                const int ns = min(64, s1 - sb);
                if (lane < ns) tile[lane] = nodes[sb + lane];
                wave_lds_sync();
                for (int j = sl; j < ns; j += G) {
                    const int s = sb + j;
                    if (!act || s < c) continue;
                    float lo;
                    if (fof_case<PER>(me, c, tile[j], s, bb, whole, uf, false, lo, L) == kDescend) {
                        const int k = atomicAdd(emit + ci, 1);
                        if (k < room) list_out[cpos + k] = make_int2(s, __float_as_int(lo));
                    }
                }
                wave_lds_sync();
            }
        }
        if (act && sl == 0) seg_out[c] = make_int2((int)cpos, min(emit[ci], room));
        wave_lds_sync();
    }
}

constexpr int FSB = 8;          // source leaves per batch
constexpr int FTILE = 128;      // source points staged per batch

// LDS slot of tile position j: permuted inside each chunk of 8 by the chunk's
// low 3 bits (lanes reading the same position of different chunks spread
// over the LDS banks)
__device__ __forceinline__ int fslot(int j) { return j ^ ((j >> 3) & 7); }

// Leaf stage: one wave per receiving leaf A, lanes over its points. Sources
// (leaves B >= A) are read in batches of FSB Node records. A source is
// skipped when A and B are both whole and already one group; a lane skips a
// source its point cannot reach (point-to-box bound > b^2); the points of the
// sources some lane needs are staged together in LDS, each source padded to
// a multiple of 8 positions, with the bounding box of every 8 positions; 8
// positions no lane can reach are skipped. Per source, every lane first
// records which of its points link to its own point (no atomics); only if
// some lane links are the roots of the source's points looked up, in
// parallel, and unions made where the roots differ (a lane's own root is
// cached; groups only ever merge, so equal roots, even looked up at different
// times, mean already connected). Two whole leaves need only one link.
template <bool PER>
__global__ __launch_bounds__(64 * WPB) void k_leaf_fof(
    const int2 *__restrict__ seg, const int2 *__restrict__ list, const Node *__restrict__ leaves,
    const float4 *__restrict__ pts, int n_leaves, float b2, const float *__restrict__ b2n,
    const int *__restrict__ whole, int *__restrict__ uf, unsigned long long *__restrict__ stats,
    const unsigned long long *__restrict__ overflow, float L) {
    const float Lh = 0.5f * L;
    __shared__ float4 s_tile[WPB][FTILE];
    __shared__ float4 s_box[WPB][FTILE / 8 * 2];  // (lo, hi) of every 8 tile positions
    __shared__ Node s_nodes[WPB][FSB];
    __shared__ int s_offs[WPB][FSB + 1];
    __shared__ int s_root[WPB][64];
    const int w = WPB == 1 ? 0 : uni((int)(tid_x() >> 6)), lane = tid_x() & 63;
    const int A = xcd_block(blk_x(), nblk_x()) * WPB + w;
    // a level of this attempt overflowed (it is rerun): nothing to do
    if (A >= n_leaves || *overflow) return;
    const Node a = leaves[A];
    const int astart = uni(a.start);
    const bool act = lane < uni(a.count);
    const int my = astart + (act ? lane : 0);
    const float4 me = pts[my];
    const float bb = b2n ? b2n[A] : b2;
    const int wA = uni(whole[A]);
    const int2 sg = seg[A];
    const int2 *gl = list + uni(sg.x);
    const int len = uni(sg.y);
    float4 *tile = s_tile[w];
    float4 *cbox = s_box[w];
    Node *nb = s_nodes[w];
    int *offs = s_offs[w];
    int *rootT = s_root[w];
    int ra = -1;  // cached root of this lane's point
    unsigned evals = 0;
    for (int t = 0; t < len;) {
        const int nb_n = min(FSB, len - t);
        const int rA = wA ? uni(uf_find_c(uf, astart)) : -1;
        bool skip = false;
        int wB = 0;
        if (lane < nb_n) {
            const int B = gl[t + lane].x;
            const Node b = leaves[B];
            nb[lane] = b;
            wB = whole[B];
            skip = wA && wB && uf_find_c(uf, b.start) == rA;
        }
        const unsigned skipmask = (unsigned)__ballot(skip);
        const unsigned wholemask = (unsigned)__ballot(lane < nb_n && wB);
        wave_lds_sync();
        unsigned needbits = 0;
        for (int q = 0; q < nb_n; ++q)
            if (!((skipmask >> q) & 1u) && act &&
                point_low2_m<PER>(me.x, me.y, me.z, nb[q].lo[0], nb[q].lo[1], nb[q].lo[2],
                                  nb[q].hi[0], nb[q].hi[1], nb[q].hi[2], L) <= bb)
                needbits |= 1u << q;
        const unsigned any = uni(wave_or(needbits));
        // take needed sources in order while their (8-padded) points fit
        int take = 0, npts = 0;
        int o_r[FSB + 1];
        o_r[0] = 0;
        if (lane == 0) offs[0] = 0;
#pragma unroll
        for (int q = 0; q < FSB; ++q) {
            const bool want = q < nb_n && take == q;
            const int c = want && ((any >> q) & 1u) ? (uni(nb[q].count) + 7) & -8 : 0;
            if (want && npts + c <= FTILE) {
                npts += c;
                take = q + 1;
            }
            o_r[q + 1] = npts;
            if (lane == 0) offs[q + 1] = npts;
        }
        // stage points (lane f takes point f of a source) and 8-position
        // boxes; fillers lie at +inf (never within b) and stay out of boxes
#pragma unroll
        for (int q = 0; q < FSB; ++q) {
            if (q < take && o_r[q + 1] > o_r[q]) {
                const int cnt = uni(nb[q].count), st = uni(nb[q].start);
                const int size = o_r[q + 1] - o_r[q];
                const bool real = lane < cnt;
                float4 p = make_float4(INFINITY, INFINITY, INFINITY, 0.0f);
                if (real) p = pts[st + lane];
                if (lane < size) tile[fslot(o_r[q] + lane)] = p;
                const float lx = group8_min(real ? p.x : INFINITY);
                const float ly = group8_min(real ? p.y : INFINITY);
                const float lz = group8_min(real ? p.z : INFINITY);
                const float hx = group8_max(real ? p.x : -INFINITY);
                const float hy = group8_max(real ? p.y : -INFINITY);
                const float hz = group8_max(real ? p.z : -INFINITY);
                if ((lane & 7) == 0 && lane < size) {
                    // the chunk's box; lo.w: its number of real points, hi.w:
                    // the z-index of its first position
                    float4 *bx = cbox + ((o_r[q] + lane) >> 3) * 2;
                    bx[0] = make_float4(lx, ly, lz, __int_as_float(min(8, max(0, cnt - lane))));
                    bx[1] = make_float4(hx, hy, hz, __int_as_float(st + lane));
                }
            }
        }
        wave_lds_sync();
        // 1: which tile positions link to this lane's point (a point links to
        // the later points of a pair only). Every lane marks the chunks its
        // point can reach (chunk box within b; a chunk box lies inside its
        // source's box) and pops its own chunks, so a pass costs the largest
        // per-lane chunk count, not the number of chunks any lane needs.
        const int nch = uni(npts >> 3);
        // periodic box: a chunk whose rounded differences to this point stay
        // within half a period on every axis (fl(q - lo) <= h, fl(q - hi) >=
        // -h; the rounded difference is monotone) never wraps, and its bound
        // and distances are the open ones bit for bit; W marks the others,
        // and the periodic forms run only where some lane has one
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
                    ? point_low2_m<PER>(me.x, me.y, me.z, blo.x, blo.y, blo.z, bhi.x, bhi.y, bhi.z, L)
                    : point_low2_m<false>(me.x, me.y, me.z, blo.x, blo.y, blo.z, bhi.x, bhi.y, bhi.z,
                                          L);
            const bool need = act && lo2 <= bb;
            M |= need ? (1u << c) : 0u;
            W |= need && wrap ? (1u << c) : 0u;
        }
        uint64_t lk[FTILE / 64] = {};
        const int nit = uni(wave_max_i(__popc(M)));
        for (int it = 0; it < nit; ++it) {
            const bool has = M != 0u;
            const int c = has ? __ffs((int)M) - 1 : 0;
            M &= M - 1u;
            const int real = has ? __float_as_int(cbox[c * 2].w) : 0;
            const int cfirst = __float_as_int(cbox[c * 2 + 1].w);
            // the positions u that count, as a mask: u < real (a real point)
            // and cfirst + u > my (a pair is taken from its lower point)
            const unsigned okm = (0xffu >> (8 - real)) &
                                 (0xffu << min(max(my - cfirst + 1, 0), 8));
            // fslot(c * 8 + u) for u < 8 is (c * 8 | (c & 7)) ^ u
            const int jb = c * 8 | (c & 7);
            unsigned m8 = 0;
            auto eval = [&](auto per_const) __attribute__((always_inline)) {
                constexpr bool P = decltype(per_const)::value;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const float4 s = tile[jb ^ u];
                    const float dd = dist2_m<P>(me.x, me.y, me.z, s.x, s.y, s.z, L, Lh);
                    m8 |= dd <= bb ? (1u << u) : 0u;
                }
            };
            if (PER && __ballot(has && ((W >> c) & 1u)))
                eval(std::integral_constant<bool, PER>());
            else
                eval(std::integral_constant<bool, false>());
            m8 &= okm;
#pragma unroll
            for (int h = 0; h < FTILE / 64; ++h)
                lk[h] |= (c >> 3) == h ? (uint64_t)m8 << ((c & 7) * 8) : 0ull;
            evals += (unsigned)real;
        }
        for (int q = 0; q < take; ++q) {
            if (!((any >> q) & 1u)) continue;
            const bool wB = (wholemask >> q) & 1u;
            const int f0 = uni(offs[q]), f1 = uni(offs[q + 1]);
            const int b0 = uni(nb[q].start);
            // this source's positions [f0, f1) of the tile link mask (f0 is a
            // multiple of 8 and a source spans at most 64 positions)
            const int h0 = f0 >> 6, sh = f0 & 63;
            uint64_t lm = 0;
#pragma unroll
            for (int h = 0; h < FTILE / 64; ++h) {
                if (h == h0) lm |= lk[h] >> sh;
                if (h == h0 + 1 && sh) lm |= lk[h] << (64 - sh);
            }
            if (f1 - f0 < 64) lm &= (1ull << (f1 - f0)) - 1ull;
            const uint64_t linking = __ballot(lm != 0);
            if (!linking) continue;
            if (wA && wB) {
                // both leaves are whole: a single link joins them
                const int leader = __ffsll((unsigned long long)linking) - 1;
                if (lane == leader) uf_union_c(uf, my, b0 + __ffsll((unsigned long long)lm) - 1);
                continue;
            }
            // 2: roots of the source's points that some lane links to,
            // looked up in parallel
            int rB = -1;
            if (wB) {
                rB = uf_find_c(uf, b0);
            } else {
                const uint64_t want = ((uint64_t)wave_or((unsigned)(lm >> 32)) << 32) |
                                      wave_or((unsigned)lm);
                if ((want >> lane) & 1ull) rootT[lane] = uf_find_c(uf, b0 + lane);
            }
            wave_lds_sync();
            // 3: unite where the roots differ. Groups only merge, so a point
            // whose looked-up root is one this lane has just united with is
            // connected already.
            if (lm) {
                if (ra < 0) ra = uf_find_c(uf, my);
                int last = -1;
                while (lm) {
                    const int f = __ffsll((unsigned long long)lm) - 1;
                    lm &= lm - 1;
                    const int rj = wB ? rB : rootT[f];
                    if (rj != ra && rj != last) {
                        uf_union_c(uf, my, b0 + f);
                        ra = uf_find_c(uf, my);
                        last = rj;
                    }
                }
            }
            wave_lds_sync();
        }
        wave_lds_sync();
        t += take;
    }
    const int ev = wave_sum_i((int)evals);
    if (lane == 0) atomicAdd(stats + (A & (STAT_SLOTS - 1)), (unsigned long long)ev);
}

// Root of every point (a read-only find: no other thread writes uf[i] now)
// and the smallest input index per root. Points of one group are mostly
// contiguous in z-order: the wave takes the minimum over each run of lanes
// with the same root (a segmented scan, 6 steps whatever the number of runs)
// and the last lane of a run issues one atomic for it, unless the root's
// current minimum is already no larger (values only decrease, so one read
// through the caches, even an older one, never skips a needed update).
__global__ __launch_bounds__(256) void k_flatten_min(int *__restrict__ uf,
                                                     const float4 *__restrict__ pts, int64_t n,
                                                     int *__restrict__ minidx) {
    const int64_t i = (int64_t)blk_x() * bdim_x() + tid_x();
    const bool valid = i < n;
    const int lane = lane_id();
    int root = -1 - lane, v = INT_MAX;  // invalid lanes: a root of their own
    if (valid) {
        // (a parent read through the caches may be an older one: still an
        // ancestor, so the walk still ends at the root)
        int x = (int)i;
        int p = ld_cached(uf + x);
        while (p != x) {
            x = p;
            p = ld_cached(uf + x);
        }
        root = x;
        uf[i] = x;
        v = __float_as_int(pts[i].w);
    }
    // segmented inclusive min-scan over runs of equal roots
    const int prev_root = __shfl_up(root, 1, 64);
    bool head = lane == 0 || prev_root != root;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int vu = __shfl_up(v, o, 64);
        const bool hu = __shfl_up((int)head, o, 64) != 0;
        if (lane >= o && !head) v = min(v, vu);
        if (lane >= o) head = head || hu;
    }
    const int next_root = __shfl_down(root, 1, 64);
    const bool tail = lane == 63 || next_root != root;
    if (valid && tail && v < ld_cached(minidx + root)) atomicMin(minidx + root, v);
}

__global__ void k_labels(const int *__restrict__ uf, const float4 *__restrict__ pts, int64_t n,
                         const int *__restrict__ minidx, const int64_t *__restrict__ set_off,
                         int nsets, int32_t *__restrict__ label) {
    const int64_t i = (int64_t)blk_x() * bdim_x() + tid_x();
    if (i >= n) return;
    const int o = __float_as_int(pts[i].w);
    int base = 0;
    if (nsets > 1) {
        int lo_s = 0, hi_s = nsets - 1;
        while (lo_s < hi_s) {
            const int m = (lo_s + hi_s + 1) >> 1;
            if (set_off[m] <= o) lo_s = m; else hi_s = m - 1;
        }
        base = (int)set_off[lo_s];
    }
    label[o] = minidx[uf[i]] - base;
}

}  // namespace

jz_status run_fof(jz_tree *t, const float *b2_set_host, int32_t *label, hipStream_t s,
                  jz_stats *st_out) {
    jz_stats &st = st_out ? *st_out : t->st;
    const AllocCtx *ac = &t->ac;
    const int P = t->P;
    const int64_t n = t->n;
    for (int p = 0; p <= JZ_MAX_PLANES; ++p) st.list_entries[p] = 0;
    st.leaf_pairs = st.leaf_pairs_visited = 0;
    st.evaluations = 0;
    st.leaf_ms = st.total_ms = 0;
    st.reruns = 0;
    st.insert_rounds = st.tile_steps = 0;
    st.lists_sorted_long = st.lists_unordered = 0;
    for (int p = 0; p <= JZ_MAX_PLANES; ++p) st.lists_presorted[p][0] = st.lists_presorted[p][1] = 0;
    if (n == 0) return JZ_OK;

    const bool sets = t->nsets > 1;
    const float b2 = b2_set_host[0];
    // periodic cube of side L (L = 0: open)
    const float L = t->opts.period;
    const bool per = L > 0.0f;
    DBuf d_ctr, d_uf, d_min, d_b2set;
    // counters: one leaf statistic (evaluations)
    const size_t nctr = ctr_words(1);
    JZ_TRY(d_ctr.get(ac, nctr * sizeof(unsigned long long), s));
    JZ_TRY(d_uf.get(ac, n * sizeof(int), s));
    JZ_TRY(d_min.get(ac, n * sizeof(int), s));
    unsigned long long *ctr = d_ctr.as<unsigned long long>();
    DBuf whole[JZ_MAX_PLANES], b2n[JZ_MAX_PLANES], segs[JZ_MAX_PLANES], lists[JZ_MAX_PLANES];
    int64_t cap[JZ_MAX_PLANES];
    for (int p = 0; p < P; ++p) {
        JZ_TRY(whole[p].get(ac, t->L[p] * sizeof(int), s));
        JZ_TRY(segs[p].get(ac, t->L[p] * sizeof(int2), s));
        cap[p] = initial_cap(t, CAP_FOF, 0, p);
    }
    if (sets) {
        JZ_TRY(d_b2set.get(ac, t->nsets * sizeof(float), s));
        JZ_HIP(hipMemcpyAsync(d_b2set.p, b2_set_host, t->nsets * sizeof(float),
                              hipMemcpyHostToDevice, s));
        for (int p = 0; p < P; ++p) {
            JZ_TRY(b2n[p].get(ac, t->L[p] * sizeof(float), s));
            k_node_b2<<<blocks_for(t->L[p], 256), 256, 0, s>>>(t->node_set[p].as<int>(), t->L[p],
                                                               d_b2set.as<float>(),
                                                               b2n[p].as<float>());
        }
    }
    EventSet ev(jz_profiling());

    // Groups only ever merge, so an overflowing run is simply rerun from the
    // start with larger lists.
    for (;;) {
        for (int p = 0; p < P; ++p) JZ_TRY(lists[p].ensure(ac, cap[p] * sizeof(int2), s));
        JZ_HIP(hipMemsetAsync(ctr, 0, d_ctr.bytes, s));
        if (ev.on) JZ_HIP(hipEventRecord(ev[0], s));
        k_iota_n<<<blocks_for(n, 256), 256, 0, s>>>(d_uf.as<int>(), n);
        k_init_min<<<blocks_for(n, 256), 256, 0, s>>>(t->pts4.as<float4>(), n, d_min.as<int>());
        for (int p = P - 1; p >= 0; --p) {
            const bool top = p == P - 1;
            const int2 *seg_in = top ? t->fof_top_seg.as<int2>() : segs[p + 1].as<int2>();
            const int2 *list_in = top ? t->fof_top_list.as<int2>() : lists[p + 1].as<int2>();
            const int *par_spl = top ? t->super_spl.as<int>() : t->spl[p + 1].as<int>();
            const int *whole_par = top ? nullptr : whole[p + 1].as<int>();
            const int64_t n_par = top ? t->S : t->L[p + 1];
            const float *bn = sets ? b2n[p].as<float>() : nullptr;
            (per ? k_fof_p2n<true> : k_fof_p2n<false>)<<<blocks_for(n_par, WPB), 64 * WPB, 0, s>>>(
                par_spl, t->nodes[p].as<Node>(), (int)n_par, whole_par, whole[p].as<int>(),
                d_uf.as<int>(), b2, bn, L);
            (per ? k_fof_step<true> : k_fof_step<false>)<<<blocks_for(n_par, WPB), 64 * WPB, 0, s>>>(
                seg_in, list_in, par_spl, t->nodes[p].as<Node>(), (int)n_par, b2, bn,
                whole[p].as<int>(), d_uf.as<int>(), segs[p].as<int2>(), lists[p].as<int2>(),
                ctr + (size_t)p * LIST_ARENAS, cap[p] / LIST_ARENAS, ctr + CTR_FLAG, L);
        }
        k_fof_l2p<<<blocks_for(t->L[0], WPB), 64 * WPB, 0, s>>>(t->nodes[0].as<Node>(), (int)t->L[0],
                                                         whole[0].as<int>(), d_uf.as<int>());
        JZ_HIP(hipGetLastError());
        if (ev.on) JZ_HIP(hipEventRecord(ev[1], s));
        (per ? k_leaf_fof<true> : k_leaf_fof<false>)<<<blocks_for(t->L[0], WPB), 64 * WPB, 0, s>>>(
            segs[0].as<int2>(), lists[0].as<int2>(), t->nodes[0].as<Node>(), t->pts4.as<float4>(),
            (int)t->L[0], b2, sets ? b2n[0].as<float>() : nullptr, whole[0].as<int>(),
            d_uf.as<int>(), ctr + CTR_STATS, ctr + CTR_FLAG, L);
        if (ev.on) JZ_HIP(hipEventRecord(ev[2], s));
        k_flatten_min<<<blocks_for(n, 256), 256, 0, s>>>(d_uf.as<int>(), t->pts4.as<float4>(), n,
                                                          d_min.as<int>());
        k_labels<<<blocks_for(n, 256), 256, 0, s>>>(d_uf.as<int>(), t->pts4.as<float4>(), n,
                                                     d_min.as<int>(), t->d_set_off.as<int64_t>(),
                                                     t->nsets, label);
        JZ_HIP(hipGetLastError());
        if (ev.on) JZ_HIP(hipEventRecord(ev[3], s));
        std::vector<unsigned long long> hc(nctr);
        JZ_HIP(hipMemcpyAsync(hc.data(), ctr, nctr * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, s));
        JZ_HIP(hipStreamSynchronize(s));
        bool overflow = false;
        double sum[JZ_MAX_PLANES], need[JZ_MAX_PLANES];
        for (int p = 0; p < P; ++p) {
            arena_need(hc.data(), p, sum[p], need[p]);
            if (need[p] <= (double)(cap[p] / LIST_ARENAS * LIST_ARENAS)) continue;
            overflow = true;
            if (need[p] > (double)INT32_MAX)
                return jz_fail(JZ_E_CAPACITY, "FoF list at plane %d needs %.0f entries "
                               "(more than 2^31-1)", p, need[p]);
            const double want = need[p] * 1.15 + 1024.0;
            cap[p] = want > (double)INT32_MAX ? (int64_t)INT32_MAX : (int64_t)want;
        }
        if (overflow) {
            if (!t->opts.auto_regrow)
                return jz_fail(JZ_E_CAPACITY, "FoF interaction list overflow; raise list_per_node");
            st.reruns++;
            continue;
        }
        for (int p = 0; p < P; ++p) {
            st.list_entries[p] = (int64_t)sum[p];
            cap_learn(CAP_FOF, 0, p, need[p] / (double)std::max<int64_t>(1, t->L[p]));
        }
        st.leaf_pairs = st.list_entries[0];
        st.evaluations = stat_sum(hc.data(), 0);
        if (ev.on) {
            float ms = 0;
            JZ_HIP(hipEventElapsedTime(&ms, ev[1], ev[2]));
            st.leaf_ms = ms;
            JZ_HIP(hipEventElapsedTime(&ms, ev[0], ev[3]));
            st.total_ms = ms;
        }
        return JZ_OK;
    }
}
