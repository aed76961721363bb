// hop_knn.hip -- Morton-sorted particle copy, implicit bounding-volume tree,
// and the exact kNN + SPH density kernel (the paper's section 2, stage 1).
//
// Layout.  Particles are sorted by the 63-bit Morton code of their integer
// coordinates (stable, so coincident particles keep input order).  Every 16
// consecutive sorted particles form a leaf; level h of the tree has node j
// covering leaves [j*2^h, (j+1)*2^h), so the tree needs no pointers.  This
// replaces the paper's kd-tree: buckets of tens of particles, built once,
// searched exactly, but with fixed-size leaves that follow the clustering
// without a per-node split decision.
//
// Search.  One wavefront owns a bucket of 64 consecutive sorted particles,
// one query per lane.  Each lane keeps its n_dens-1 nearest others in a
// 4-ary max-heap keyed by (d^2 << B) | tie_key, which orders candidates by
// (d^2, id) exactly (d^2 is an exact integer held in FP64); the heap's top
// two levels sit in registers, the rest in LDS.  The search runs in three
// passes:
//   1. seed: the bucket's own particles and one Morton-neighbour bucket on
//      each side are offered, which gives every lane a finite bound;
//   2. walk: a breadth-first descent of the tree, 64 child boxes tested per
//      step against the boxes and bounds of 8 groups of 8 lanes; it stops at
//      the level where the surviving frontier would exceed the leaf list,
//      so the list may hold whole subtrees (ranges of leaves) as well as
//      single leaves;
//   3. stream: the listed leaves, in classes of increasing distance from
//      the bucket's box, are loaded 64 particles at a time; each particle is
//      tested by all lanes against their current bounds (exactly, in FP64)
//      and the ones that pass are inserted lane by lane, one batch behind
//      (lanes done with a batch go on with the next one's).  After the near
//      classes, and every 24 batches after that, the entries not streamed
//      yet are tested again against the groups' tightened bounds and the
//      list is compacted.
// Only pruning depends on the bounds; every particle that could belong to
// a lane's list is offered to it, so the result is the exact kNN.
//
// Density.  After the walk the heap is sorted in registers by a bitonic
// network; the spline weights are summed pairwise (a fixed tree over 64
// slots, zero-padded) and the result divided by h^3, all in FP64 with
// correctly rounded division and square root and no contraction.
#include "hop_internal.h"

#include <algorithm>
#include <type_traits>
#include <cstring>
#include <vector>

namespace {

__device__ __forceinline__ uint64_t spread3(uint32_t v)
{
    uint64_t x = v & 0x1fffffu;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}

// inverse of spread3: every third bit of v, from bit 0
__device__ __forceinline__ uint32_t compact3(uint64_t v)
{
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
    v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
    v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
    v = (v ^ (v >> 32)) & 0x1fffffull;
    return (uint32_t)v;
}

__global__ void k_morton(const uint32_t *__restrict__ pos, int64_t n, uint32_t glim,
                         uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
                         uint32_t *__restrict__ dflags)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    if (x >= glim || y >= glim || z >= glim) {
        atomicOr(dflags, DERR_RANGE);
        x = min(x, glim - 1);
        y = min(y, glim - 1);
        z = min(z, glim - 1);
    }
    keys[i] = (spread3(x) << 2) | (spread3(y) << 1) | spread3(z);
    vals[i] = (uint32_t)i;
}

// codes: the sorted full Morton codes, which hold the (clamped) coordinates
// themselves, so that no position is gathered; NULL: gather from pos.
__global__ void k_gather_recs(const uint32_t *__restrict__ pos, const uint64_t *__restrict__ codes,
                              const uint32_t *__restrict__ perm, const int32_t *__restrict__ tk,
                              int64_t n, uint32_t glim, SortedRec *__restrict__ recs)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    int32_t j = (int32_t)perm[t];
    SortedRec r;
    if (codes) {
        const uint64_t c = codes[t];
        r.x = (double)compact3(c >> 2);
        r.y = (double)compact3(c >> 1);
        r.z = (double)compact3(c);
    } else {
        r.x = (double)min(pos[3 * (int64_t)j], glim - 1);
        r.y = (double)min(pos[3 * (int64_t)j + 1], glim - 1);
        r.z = (double)min(pos[3 * (int64_t)j + 2], glim - 1);
    }
    r.j = j;
    r.tk = tk ? tk[j] : j;
    recs[t] = r;
}

__global__ void k_leaf_boxes(const SortedRec *__restrict__ recs, int64_t n, int64_t n_leaves,
                             NodeBox *__restrict__ boxes)
{
    int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (L >= n_leaves) return;
    int64_t b = L * HOP_LEAF, e = min(b + HOP_LEAF, n);
    NodeBox bx;
    bx.lo[0] = bx.lo[1] = bx.lo[2] = 0xffffffffu;
    bx.hi[0] = bx.hi[1] = bx.hi[2] = 0u;
    for (int64_t t = b; t < e; t++) {
        uint32_t c[3] = {(uint32_t)recs[t].x, (uint32_t)recs[t].y, (uint32_t)recs[t].z};
#pragma unroll
        for (int a = 0; a < 3; a++) {
            bx.lo[a] = min(bx.lo[a], c[a]);
            bx.hi[a] = max(bx.hi[a], c[a]);
        }
    }
    bx.count = (uint32_t)(e - b);
    bx.pad = 0;
    boxes[L] = bx;
}

__global__ void k_level_boxes(NodeBox *__restrict__ boxes, int64_t child_off, int32_t child_cnt,
                              int64_t off, int32_t cnt)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cnt) return;
    NodeBox a = boxes[child_off + 2 * j];
    if (2 * j + 1 < child_cnt) {
        NodeBox b = boxes[child_off + 2 * j + 1];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            a.lo[k] = min(a.lo[k], b.lo[k]);
            a.hi[k] = max(a.hi[k], b.hi[k]);
        }
        a.count += b.count;
    }
    boxes[off + j] = a;
}

// ---------------------------------------------------------------------------
// kNN + density
// ---------------------------------------------------------------------------

constexpr int kHeapMax = 63;    // n_dens - 1 <= 63 (the default kernels)
constexpr int kHeapMaxBig = 127; // n_dens - 1 <= 127 (the kernels for n_dens 65..128)
#ifndef HOP_SEED_SIDES
#define HOP_SEED_SIDES 1
#endif
constexpr int kSeedSides = HOP_SEED_SIDES;  // Morton-neighbour buckets seeded on each side
#ifndef HOP_LIST_CLASSES
#define HOP_LIST_CLASSES 7
#endif
constexpr int kListClasses = HOP_LIST_CLASSES;  // distance classes of the leaf list
#ifndef HOP_NEAR_CLASSES
#define HOP_NEAR_CLASSES 5
#endif
constexpr int kNearClasses = HOP_NEAR_CLASSES;  // classes streamed before the list is pruned again
#ifndef HOP_PRUNE_EVERY
#define HOP_PRUNE_EVERY 24
#endif
constexpr int kPruneEvery = HOP_PRUNE_EVERY;  // batches between later prunings
constexpr int kWindow = 32;                    // stream positions per interleave window
constexpr int kHeapSlots = 65;     // 4-ary heap of 63: slots up to 4*15+4 are read
constexpr int kHeapSlotsBig = 130; // 4-ary heap of 127: slots up to 4*31+5 are read
// LDS heap slots of a kernel instance
template <bool BIG> constexpr int heap_slots() { return BIG ? kHeapSlotsBig : kHeapSlots; }
// a sift from slot i reads slots 4i+1 .. 4i+4 while 4i+1 < heap size
static_assert(kHeapSlots >= kHeapMax + 2 && kHeapSlotsBig >= kHeapMaxBig + 3, "heap slots");

struct KnnArgs {
    const SortedRec *recs;
    const NodeBox *boxes;
    TreeLevels lv;
    int64_t n;
    int64_t n_buckets;
    int64_t xcd_chunk;   // buckets per XCD slice of the grid
    int hs;              // heap size = n_dens - 1
    int n_dens;
    int k_store;
    int shift;           // bits of the tie key
    uint64_t tk_mask;
    double maxd2;        // largest d^2 the packed key holds
    double norm;         // 1 / (pi * mean_density)
    double gsize;        // 2^grid_bits
    uint32_t gmask;
    int front_cap;       // frontier entries the walk may use (<= kFront)
    int vec_store;       // nbr rows 16-byte aligned with k_store % 4 == 0
    int fp32;            // density arithmetic in FP32 (neighbour search unchanged)
    float norm32;        // norm rounded to FP32
    int32_t *nbr;
    double *dens;
    // (NULL = off) the first 16 list entries and the density again, at the
    // query's sorted position: rows of 64 B written by consecutive lanes
    int32_t *nbr16s;
    double *dens_s;
    const int32_t *tk2j;
    uint32_t *dflags;
    // (NULL = off) [0] nodes tested, [1] leaves scanned, [2] heap-insertion
    // loop iterations, [3] candidates offered to a heap (those that pass
    // the batch test against the lane's bound)
    unsigned long long *counters;
    // learned radius (NULL = off): search radius per cell of side 2^cell_bits,
    // 2^cell_gb cells per axis; lanes whose list does not fit inside it are
    // recorded in miss[bucket] and write nothing
    const float *cell_r;
    int cell_bits, cell_gb;
    unsigned long long *miss;
};

// Work description of a batched launch (device arrays, see k_knn_batch).
struct BatchArgs {
    const int64_t *sub_off;   // [n_sub + 1] particle ranges (sorted = input ranges)
    const int32_t *order;     // [n_sub] processing order of the subvolumes
    const int64_t *item_off;  // [n_sub + 1] first bucket of order[k]
    const double *norm;       // [n_sub] 1 / (pi * mean density)
    const float *norm32;      // [n_sub] the same rounded to FP32
    uint32_t *queue;          // [8] chunk cursors, zero at launch
    uint32_t *done;           // [n_sub] buckets finished, zero at launch
    int64_t n_items;
    int n_sub;
    int xcd_queues;           // 1: one chunk per XCD; 0: one shared queue
};

// (d^2 << shift) | tk.  d^2 is an exact integer below 2^52 held in a double:
// adding 2^52 places it in the low mantissa bits, so two instructions give
// its integer value.
__device__ __forceinline__ uint64_t make_key(double d2, uint32_t tk, const KnnArgs &a)
{
    double c = fmin(d2, a.maxd2) + 4503599627370496.0;  // + 2^52, exact
    uint64_t m = (uint64_t)__double_as_longlong(c) & 0xfffffffffffffull;
    return (m << a.shift) | (uint64_t)tk;
}

__device__ __forceinline__ double key_d2(uint64_t key, int shift)
{
    // d^2 < 2^52: rebuild the double from its integer value the same way
    uint64_t m = key >> shift;
    return __longlong_as_double((long long)(m | 0x4330000000000000ull)) - 4503599627370496.0;
}

// M4 cubic-spline shape without the 1/(pi h^3) factor, q2 = (r/h)^2.
__device__ __forceinline__ double m4_shape(double q2)
{
    double q = __builtin_sqrt(q2);
    double two_q = 2.0 - q;
    if (q2 < 1.0) return 1.0 - (0.75 * two_q) * q2;
    if (q2 < 4.0) return 0.25 * ((two_q * two_q) * two_q);
    return 0.0;
}

// The same shape in FP32 (the reduced-precision density variant).
__device__ __forceinline__ float m4_shape_f32(float q2)
{
    float q = __builtin_sqrtf(q2);
    float two_q = 2.0f - q;
    if (q2 < 1.0f) return 1.0f - (0.75f * two_q) * q2;
    if (q2 < 4.0f) return 0.25f * ((two_q * two_q) * two_q);
    return 0.0f;
}

template <bool PERIODIC>
__device__ __forceinline__ double axis_gap(uint32_t x, uint32_t lo, uint32_t hi, uint32_t gmask)
{
    if (PERIODIC) {
        bool inside = ((x - lo) & gmask) <= (hi - lo);
        uint32_t up = (lo - x) & gmask, dn = (x - hi) & gmask;
        return inside ? 0.0 : (double)min(up, dn);
    } else {
        int d = max(max((int)lo - (int)x, (int)x - (int)hi), 0);
        return (double)d;
    }
}

template <bool PERIODIC>
__device__ __forceinline__ double box_d2(uint32_t ux, uint32_t uy, uint32_t uz, const NodeBox &b,
                                         uint32_t gmask)
{
    double gx = axis_gap<PERIODIC>(ux, b.lo[0], b.hi[0], gmask);
    double gy = axis_gap<PERIODIC>(uy, b.lo[1], b.hi[1], gmask);
    double gz = axis_gap<PERIODIC>(uz, b.lo[2], b.hi[2], gmask);
    return __builtin_fma(gx, gx, __builtin_fma(gy, gy, gz * gz));
}

// 4-ary max-heap of one lane: slot s at heap[s * 64 + lane]; slots in
// [hs, kHeapSlots) hold 0 so that missing children never win.
__device__ __forceinline__ void heap_sift(uint64_t *heap, int lane, int hs, int i, uint64_t x)
{
    for (;;) {
        const int c = 4 * i + 1;
        if (c >= hs) break;
        uint64_t k0 = heap[c * 64 + lane], k1 = heap[(c + 1) * 64 + lane];
        uint64_t k2 = heap[(c + 2) * 64 + lane], k3 = heap[(c + 3) * 64 + lane];
        int m01 = k1 > k0 ? c + 1 : c;
        uint64_t v01 = k1 > k0 ? k1 : k0;
        int m23 = k3 > k2 ? c + 3 : c + 2;
        uint64_t v23 = k3 > k2 ? k3 : k2;
        int m = v23 > v01 ? m23 : m01;
        uint64_t v = v23 > v01 ? v23 : v01;
        if (v <= x) break;
        heap[i * 64 + lane] = v;
        i = m;
    }
    heap[i * 64 + lane] = x;
}

__device__ __forceinline__ double d2_direct(double qx, double qy, double qz, const SortedRec &p)
{
    double dx = qx - p.x, dy = qy - p.y, dz = qz - p.z;
    return __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
}

__device__ __forceinline__ double d2_wrap(double qx, double qy, double qz, const SortedRec &p,
                                          double gsize)
{
    double dx = fabs(qx - p.x), dy = fabs(qy - p.y), dz = fabs(qz - p.z);
    dx = fmin(dx, gsize - dx);
    dy = fmin(dy, gsize - dy);
    dz = fmin(dz, gsize - dz);
    return __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
}

constexpr int kLeafList = 1024;    // leaves the walk may hand to the streaming passes
constexpr int kFront = kLeafList;  // largest frontier_cap honoured
// Frontier entries per level of the breadth-first walk.  A level that
// would hold more than kLeafList entries is never used (the walk keeps the
// previous level), so entries past kLeafList need not be stored; the
// default kernels have room for more in the heap area they borrow.
constexpr int kFrontLevel = 4096;
constexpr int kFrontLevelBig = kLeafList;

// Squared gap between two boxes (minimum image when periodic).
template <bool PERIODIC>
__device__ __forceinline__ double boxbox_d2(const NodeBox &p, const NodeBox &q, uint32_t gmask)
{
    double g2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const uint32_t a1 = p.lo[k], b1 = p.hi[k], a2 = q.lo[k], b2 = q.hi[k];
        double g = 0.0;
        if (!(a1 <= b2 && a2 <= b1)) {
            if (PERIODIC) g = (double)min((a2 - b1) & gmask, (a1 - b2) & gmask);
            else g = (double)max((int)a2 - (int)b1, (int)a1 - (int)b2);
        }
        g2 = __builtin_fma(g, g, g2);
    }
    return g2;
}

// Per-lane 4-ary max-heap of hs keys.  The root (index 0) and its four
// children (indices 1-4) live in registers, the deeper levels (indices
// 5..hs-1) in LDS at heap[i*64 + lane]; LDS slots hs..64 hold 0 so that
// missing children never win.  Replacing the root therefore costs two
// dependent LDS round trips instead of one per level.
struct RegHeap {
    uint64_t r0;
    uint64_t r1[4];
};

// LDS-only 4-ary sift of x from node i (i >= 1, children at 4i+1..4i+4).
__device__ __forceinline__ void lds_sift(uint64_t *heap, int lane, int hs, int i, uint64_t x)
{
    for (;;) {
        const int c = 4 * i + 1;
        if (c >= hs) break;
        const uint64_t k0 = heap[c * 64 + lane], k1 = heap[(c + 1) * 64 + lane];
        const uint64_t k2 = heap[(c + 2) * 64 + lane], k3 = heap[(c + 3) * 64 + lane];
        const int m01 = k1 > k0 ? c + 1 : c;
        const uint64_t v01 = k1 > k0 ? k1 : k0;
        const int m23 = k3 > k2 ? c + 3 : c + 2;
        const uint64_t v23 = k3 > k2 ? k3 : k2;
        const int m = v23 > v01 ? m23 : m01;
        const uint64_t v = v23 > v01 ? v23 : v01;
        if (v <= x) break;
        heap[i * 64 + lane] = v;
        i = m;
    }
    heap[i * 64 + lane] = x;
}

// LDS-only 4-ary sift of x from node i within the first `size` slots
// (slots from `size` on are ignored: the in-place heapsort keeps its sorted
// tail there).
__device__ __forceinline__ void lds_sift_size(uint64_t *heap, int lane, int size, int i, uint64_t x)
{
    for (;;) {
        const int c = 4 * i + 1;
        if (c >= size) break;
        uint64_t v = heap[c * 64 + lane];
        int m = c;
#pragma unroll
        for (int q = 1; q < 4; q++) {
            if (c + q < size) {
                const uint64_t k = heap[(c + q) * 64 + lane];
                m = k > v ? c + q : m;
                v = k > v ? k : v;
            }
        }
        if (v <= x) break;
        heap[i * 64 + lane] = v;
        i = m;
    }
    heap[i * 64 + lane] = x;
}

// Pairwise (binary-counter) sum over NSLOT slots of the spline weights of
// a sorted list: slot 0 is the particle itself (q = 0), slot t < n_dens the
// list entry whose squared distance d2_at(t - 1) returns, the rest zero.
// T(a, b) = T(a, m) + T(m, b) over halves, so the order is fixed for any
// n_dens and adding the zero slots is exact.
template <int NSLOT, typename F, typename D2At, typename Shape>
__device__ __forceinline__ F pairwise_spline(int n_dens, F R, D2At d2_at, Shape shape)
{
    constexpr int LG = NSLOT == 128 ? 7 : 6;
    F part[LG + 1];
#pragma unroll
    for (int t = 0; t < NSLOT; t++) {
        F w;
        if (t == 0) {
            w = shape((F)0);
        } else if (t < n_dens) {
            const uint64_t d2 = d2_at(t - 1);
            w = shape((F)(4 * d2) / R);
        } else {
            w = (F)0;
        }
        F sum = w;
        int lvl = 0;
#pragma unroll
        for (int b = 0; b < LG; b++) {
            if (((t >> b) & 1) == 0) break;
            sum = part[b] + sum;
            lvl = b + 1;
        }
        part[lvl] = sum;
    }
    return part[LG];
}

// Replace the root by x (x below the root) and restore the heap.  Levels 0
// and 1 are registers (selected without indexing), deeper levels LDS.
// The same for a full heap of 63 keys (n_dens = 64), whose depth is fixed:
// level 2 is slots 5..20, level 3 slots 21..62 (children of slots 5..15;
// slots 63 and 64 hold 0).  Written without branches: x equal to the root
// leaves the heap as it is, both LDS slots on the path are always read and
// written (a slot that does not move gets its own key back), so the two LDS
// round trips are the only dependent steps and no lane masks are juggled.
__device__ __forceinline__ void rh_replace_root63(RegHeap &H, uint64_t *heap, int lane, uint64_t x)
{
    const uint64_t k0 = H.r1[0], k1 = H.r1[1], k2 = H.r1[2], k3 = H.r1[3];
    const int m01 = k1 > k0 ? 1 : 0;
    const uint64_t v01 = k1 > k0 ? k1 : k0;
    const int m23 = k3 > k2 ? 3 : 2;
    const uint64_t v23 = k3 > k2 ? k3 : k2;
    const int m = v23 > v01 ? m23 : m01;  // child 1+m
    const uint64_t v = v23 > v01 ? v23 : v01;
    const bool up = v > x;
    H.r0 = up ? v : x;
    // level 2: the children of slot 1+m
    const int c = 4 * m + 5;
    const uint64_t w0 = heap[c * 64 + lane], w1 = heap[(c + 1) * 64 + lane];
    const uint64_t w2 = heap[(c + 2) * 64 + lane], w3 = heap[(c + 3) * 64 + lane];
    const int n01 = w1 > w0 ? c + 1 : c;
    const uint64_t u01 = w1 > w0 ? w1 : w0;
    const int n23 = w3 > w2 ? c + 3 : c + 2;
    const uint64_t u23 = w3 > w2 ? w3 : w2;
    const int nm = u23 > u01 ? n23 : n01;
    const uint64_t u = u23 > u01 ? u23 : u01;
    const bool down = up && u > x;
    // level 3: the children of slot nm (slots up to 64 are inside the heap
    // area; those of slots 16..20 do not exist)
    const int d = 4 * min(nm, 15) + 1;
    const uint64_t z0 = heap[d * 64 + lane], z1 = heap[(d + 1) * 64 + lane];
    const uint64_t z2 = heap[(d + 2) * 64 + lane], z3 = heap[(d + 3) * 64 + lane];
    const int y01i = z1 > z0 ? d + 1 : d;
    const uint64_t y01 = z1 > z0 ? z1 : z0;
    const int y23i = z3 > z2 ? d + 3 : d + 2;
    const uint64_t y23 = z3 > z2 ? z3 : z2;
    const int ym = y23 > y01 ? y23i : y01i;
    const uint64_t yraw = y23 > y01 ? y23 : y01;
    const uint64_t y = (nm <= 15) ? yraw : 0ull;
    const bool deeper = down && y > x;
    const uint64_t put1 = down ? u : x;  // into register slot 1+m
#pragma unroll
    for (int q = 0; q < 4; q++) H.r1[q] = (up && q == m) ? put1 : H.r1[q];
    heap[nm * 64 + lane] = down ? (deeper ? y : x) : u;
    heap[ym * 64 + lane] = deeper ? x : yraw;
}

__device__ __forceinline__ void rh_replace_root(RegHeap &H, uint64_t *heap, int lane, int hs, uint64_t x)
{
    if (hs == kHeapMax) {
        rh_replace_root63(H, heap, lane, x);
        return;
    }
    if (hs <= 1) {
        H.r0 = x;
        return;
    }
    const uint64_t k0 = H.r1[0], k1 = H.r1[1], k2 = H.r1[2], k3 = H.r1[3];
    const int m01 = k1 > k0 ? 1 : 0;
    const uint64_t v01 = k1 > k0 ? k1 : k0;
    const int m23 = k3 > k2 ? 3 : 2;
    const uint64_t v23 = k3 > k2 ? k3 : k2;
    const int m = v23 > v01 ? m23 : m01;  // child 1+m
    const uint64_t v = v23 > v01 ? v23 : v01;
    if (v <= x) {
        H.r0 = x;
        return;
    }
    H.r0 = v;
    // x moves into child 1+m unless one of that child's children is larger
    const int c = 4 * (1 + m) + 1;
    uint64_t put = x;
    int deeper = -1;
    if (c < hs) {
        const uint64_t w0 = heap[c * 64 + lane], w1 = heap[(c + 1) * 64 + lane];
        const uint64_t w2 = heap[(c + 2) * 64 + lane], w3 = heap[(c + 3) * 64 + lane];
        const int n01 = w1 > w0 ? c + 1 : c;
        const uint64_t u01 = w1 > w0 ? w1 : w0;
        const int n23 = w3 > w2 ? c + 3 : c + 2;
        const uint64_t u23 = w3 > w2 ? w3 : w2;
        const int nm = u23 > u01 ? n23 : n01;
        const uint64_t u = u23 > u01 ? u23 : u01;
        if (u > x) {
            put = u;
            deeper = nm;
        }
    }
#pragma unroll
    for (int q = 0; q < 4; q++) H.r1[q] = (q == m) ? put : H.r1[q];
    if (deeper >= 0) lds_sift(heap, lane, hs, deeper, x);
}

// One bucket: the bcount (<= 64) sorted particles from b0, all inside the
// particle range [plo, phi) of one independent problem (the whole box, or
// one subvolume of a batch).  Candidates outside [plo, phi) are never
// offered, and the walk never enters a subtree whose leaves lie outside it.
// heap, stage and leaves are the wave's LDS buffers.
// Only the lanes set in qmask are queries; the others still serve as
// candidates.
// BIG: n_dens up to 128 (heap of up to 127 keys, all but the top two
// levels in LDS, and the walk's frontier in LDS of its own, `front`);
// otherwise n_dens up to 64 and the frontier borrows the heap's LDS while
// the heap's deeper levels are parked in registers (front is unused).
template <bool PERIODIC, bool IDS, bool BIG, bool COUNT>
__device__ __forceinline__ void knn_bucket(const KnnArgs &a, const int64_t b0, const int bcount,
                                           const int64_t plo, const int64_t phi,
                                           const double norm, const float norm32, uint64_t *heap,
                                           uint32_t *front, SortedRec *stage, double *stage_pp,
                                           uint32_t *leaves, const uint64_t qmask,
                                           const int64_t bucket_id)
{
    constexpr int kSlots = heap_slots<BIG>();
    constexpr int kFL = BIG ? kFrontLevelBig : kFrontLevel;
    uint32_t *front_a = BIG ? front : reinterpret_cast<uint32_t *>(heap);
    uint32_t *front_b = front_a + kFL;

    const int lane = threadIdx.x;
    const bool active = lane < bcount && ((qmask >> lane) & 1ull);
    const int hs = a.hs;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const double G = a.gsize;
    const int64_t n_leaf_total = a.lv.cnt[0];
    // work counters (COUNT instances with a.counters set).  A loop that
    // offers marked candidates one per lane per iteration runs exactly as
    // many iterations as its busiest lane has offers, so both counts come
    // from per-batch popcounts and nothing is added to the loops themselves;
    // they live in instances of their own, because their mere presence
    // slowed the kernel by 1.4% with counting off
    const bool counting = COUNT && a.counters != nullptr;
    unsigned long long n_nodes = 0, n_lv = 0, n_it = 0, n_off = 0;
    auto count_offers = [&](uint64_t pass, uint32_t lane_iters) {
        n_off += (unsigned long long)__popcll(pass);
        uint32_t m = lane_iters;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, d));
        n_it += m;
    };

    if (lane < bcount) stage[lane] = a.recs[b0 + lane];
    __syncthreads();
    const SortedRec me = stage[lane < bcount ? lane : 0];
    const double qx = me.x, qy = me.y, qz = me.z;
    const uint32_t ux = (uint32_t)qx, uy = (uint32_t)qy, uz = (uint32_t)qz;
    const int32_t mytk = me.tk;
    // for the expanded distance test of the streaming pass
    const double m2x = -2.0 * qx, m2y = -2.0 * qy, m2z = -2.0 * qz;
    const double qq = __builtin_fma(qx, qx, __builtin_fma(qy, qy, qz * qz));
    // squared search radius of a bounded (learned-radius) search
    double rcap = 1.0e300;
    if (a.cell_r && active) {
        const int64_t c = ((int64_t)(uz >> a.cell_bits) << (2 * a.cell_gb)) |
                          ((int64_t)(uy >> a.cell_bits) << a.cell_gb) | (int64_t)(ux >> a.cell_bits);
        const double r = (double)a.cell_r[c];
        rcap = r * r;
    }

    // 1. seed the heap with the bucket's other particles (the first hs go
    //    straight into place, then one heapify) ...
    RegHeap H;
    {
        for (int s = 0; s < kSlots; s++) heap[s * 64 + lane] = 0;
        int slot = 0;
        for (int k = 0; k < HOP_BUCKET && slot < hs; k++) {
            if (k == lane) continue;
            uint64_t key = ~0ull;
            if (k < bcount) {
                const double d2 = PERIODIC ? d2_wrap(qx, qy, qz, stage[k], G) : d2_direct(qx, qy, qz, stage[k]);
                key = make_key(d2, (uint32_t)stage[k].tk, a);
            }
            heap[slot * 64 + lane] = key;
            slot++;
        }
        for (int s = slot; s < hs; s++) heap[s * 64 + lane] = ~0ull;  // buckets smaller than hs + 1
        for (int i = (hs - 2) / 4; i >= 0; i--) heap_sift(heap, lane, hs, i, heap[i * 64 + lane]);
        H.r0 = heap[lane];
#pragma unroll
        for (int q = 0; q < 4; q++) H.r1[q] = heap[(q + 1) * 64 + lane];
    }
    double tau = active ? fmin(key_d2(H.r0, a.shift), rcap) : -1.0;
    // offer the particles of the staged batch whose bits are set
    // (the key of the next marked particle is computed before the heap
    // update of the current one, so that its LDS read and arithmetic overlap
    // the heap's dependent LDS round trips)
    auto next_key = [&](uint64_t &pass, bool wrap) -> uint64_t {
        const bool any = pass != 0;
        const int k = __builtin_ctzll(pass | (1ull << 63));  // 63 when none is left
        pass &= pass - 1;
        const SortedRec p = stage[k];
        const double d2 = wrap ? d2_wrap(qx, qy, qz, p, G) : d2_direct(qx, qy, qz, p);
        const uint64_t key = make_key(d2, (uint32_t)p.tk, a);
        return any ? key : ~0ull;
    };
    auto insert_marked = [&](uint64_t pass, bool wrap) {
        if (counting) count_offers(pass, (uint32_t)__popcll(pass));
        bool have = pass != 0;
        uint64_t key = next_key(pass, wrap);
        if (!BIG && hs == kHeapMax) {
            while (__any(have)) {
                const bool have_next = pass != 0;
                const uint64_t key_next = next_key(pass, wrap);
                rh_replace_root63(H, heap, lane, (have && key < H.r0) ? key : H.r0);
                have = have_next;
                key = key_next;
            }
        } else {
            while (__any(have)) {
                const bool have_next = pass != 0;
                const uint64_t key_next = next_key(pass, wrap);
                if (have && key < H.r0) rh_replace_root(H, heap, lane, hs, key);
                have = have_next;
                key = key_next;
            }
        }
        if (active) tau = fmin(key_d2(H.r0, a.shift), rcap);
    };
    // ... and offer the rest of the bucket (hs < 63 only) and kSeedSides
    //    Morton-neighbour buckets on each side (exact minimum image).
    //    Nearest buckets first; the two buckets at distance d go in two
    //    batches that each take one half of both (lanes 0-31 from bucket -d,
    //    lanes 32-63 from bucket +d), so the lanes near either side share
    //    each batch's insertions; the halves next to the bucket go first
    for (int si = 0; si < 2 * kSeedSides + 1; si++) {
        if (si == 0 && hs >= HOP_BUCKET - 1) continue;
        int64_t idx = b0 + lane;
        if (si > 0) {
            const int64_t d = (si + 1) >> 1;
            const int near_first = lane < 32 ? (si & 1) : ((si - 1) & 1);
            idx = (lane < 32 ? b0 - d * HOP_BUCKET : b0 + d * HOP_BUCKET) + 32 * near_first + (lane & 31);
        }
        const bool here = si == 0 ? lane < bcount : (idx >= plo && idx < phi);
        const uint64_t vm = __ballot(here);
        if (vm == 0) continue;
        __syncthreads();
        if (here) stage[lane] = a.recs[idx];
        __syncthreads();
        uint64_t pass = 0;
        for (int k0 = 0; k0 < HOP_BUCKET; k0 += 16) {
            SortedRec pr[16];
#pragma unroll
            for (int k = 0; k < 16; k++) pr[k] = stage[k0 + k];
#pragma unroll
            for (int k = 0; k < 16; k++) {
                const int kk = k0 + k;
                const double d2 = PERIODIC ? d2_wrap(qx, qy, qz, pr[k], G) : d2_direct(qx, qy, qz, pr[k]);
                // own bucket: only the particles the fill did not take
                const bool fresh = si != 0 || (kk != lane && kk - (kk > lane ? 1 : 0) >= hs);
                pass |= (uint64_t)((((vm >> kk) & 1) && fresh && pr[k].tk != mytk && d2 <= tau) ? 1u : 0u) << kk;
            }
        }
        insert_marked(pass, PERIODIC);
    }
    // particles already offered by the seed, and the leaves of [plo, phi)
    const int64_t seed_lo = max(b0 - kSeedSides * HOP_BUCKET, plo);
    const int64_t seed_hi = min(b0 + (kSeedSides + 1) * HOP_BUCKET, phi);
    const int64_t leaf_lo = plo / HOP_LEAF, leaf_hi = (phi - 1) / HOP_LEAF;

    double tmax = tau;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) tmax = fmax(tmax, __shfl_xor(tmax, d));
    {
        // the same in every lane: make that visible to the compiler, so that
        // the decisions taken from it are scalar branches
        const long long tb = __double_as_longlong(tmax);
        const int hi = __builtin_amdgcn_readfirstlane((int)(tb >> 32));
        const int lo = __builtin_amdgcn_readfirstlane((int)(tb & 0xffffffff));
        tmax = __longlong_as_double(((long long)hi << 32) | (uint32_t)lo);
    }

    // groups of 8 consecutive lanes: box of their queries and largest bound,
    // held in scalar registers for the walk
    NodeBox gbox[8];
    double gt[8];
    {
        uint32_t lo[3] = {active ? ux : 0xffffffffu, active ? uy : 0xffffffffu, active ? uz : 0xffffffffu};
        uint32_t hi[3] = {active ? ux : 0u, active ? uy : 0u, active ? uz : 0u};
        double t = tau;
#pragma unroll
        for (int d = 1; d < 8; d <<= 1) {
#pragma unroll
            for (int k = 0; k < 3; k++) {
                lo[k] = min(lo[k], (uint32_t)__shfl_xor((int)lo[k], d));
                hi[k] = max(hi[k], (uint32_t)__shfl_xor((int)hi[k], d));
            }
            t = fmax(t, __shfl_xor(t, d));
        }
#pragma unroll
        for (int g = 0; g < 8; g++) {
#pragma unroll
            for (int k = 0; k < 3; k++) {
                gbox[g].lo[k] = (uint32_t)__builtin_amdgcn_readlane((int)lo[k], 8 * g);
                gbox[g].hi[k] = (uint32_t)__builtin_amdgcn_readlane((int)hi[k], 8 * g);
            }
            const long long tb = __double_as_longlong(t);
            const int tlo = __builtin_amdgcn_readlane((int)(tb & 0xffffffff), 8 * g);
            const int thi = __builtin_amdgcn_readlane((int)(tb >> 32), 8 * g);
            gt[g] = __longlong_as_double(((long long)thi << 32) | (uint32_t)tlo);
        }
    }

    // 2. breadth-first walk: keep the nodes within a group's bound of that
    //    group's box; 64 lanes test 64 children at once.  In the default
    //    kernels the frontier uses the heap's LDS levels, so levels 2-3 of
    //    the heap are parked in registers meanwhile.
    NodeBox bb;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        bb.lo[k] = gbox[0].lo[k];
        bb.hi[k] = gbox[0].hi[k];
#pragma unroll
        for (int g = 1; g < 8; g++) {
            bb.lo[k] = min(bb.lo[k], gbox[g].lo[k]);
            bb.hi[k] = max(bb.hi[k], gbox[g].hi[k]);
        }
    }
    // park heap levels 2..3 (slots 5..hs-1) in registers
    uint64_t park[BIG ? 1 : kHeapMax - 5];
    if constexpr (!BIG) {
#pragma unroll
        for (int s = 5; s < kHeapMax; s++) park[s - 5] = s < hs ? heap[s * 64 + lane] : 0;
    }
    __syncthreads();
    int fcnt = 1, hf = a.lv.top;
    uint32_t *fc = front_a, *fn = front_b;
    fc[0] = 0;
    __syncthreads();
    while (hf > 0) {
        const int h = hf;
        // a small frontier descends several levels in one step: its
        // descendants sl levels down fill the 64 lanes (a descendant's box
        // lies inside its ancestor's, so skipping the levels between prunes
        // nothing that the level-by-level walk would keep)
        int sl = 1;
        while (sl < 6 && sl < h && (fcnt << (sl + 1)) <= 64) sl++;
        const int hc = h - sl;
        int ncnt = 0;
        for (int base = 0; base < fcnt; base += (64 >> sl)) {
            const int ni = base + (lane >> sl);
            bool need = false;
            uint32_t child = 0;
            if (ni < fcnt) {
                child = (fc[ni] << sl) + (uint32_t)(lane & ((1 << sl) - 1));
                const int64_t cfirst = (int64_t)child << hc;
                const int64_t clast = cfirst + ((int64_t)1 << hc) - 1;
                if (child < (uint32_t)a.lv.cnt[hc] && cfirst <= leaf_hi && clast >= leaf_lo) {
                    const NodeBox cb = a.boxes[a.lv.off[hc] + child];
#pragma unroll
                    for (int g = 0; g < 8; g++) need |= boxbox_d2<PERIODIC>(gbox[g], cb, a.gmask) <= gt[g];
                }
            }
            const uint64_t m = __ballot(need);
            const int pos = ncnt + (int)__popcll(m & lt_mask);
            if (need && pos < kFL) fn[pos] = child;
            ncnt += (int)__popcll(m);
            n_nodes += 64;
        }
        __syncthreads();
        if (ncnt > min(a.front_cap, kLeafList)) break;  // keep level h
        uint32_t *t = fc;
        fc = fn;
        fn = t;
        fcnt = ncnt;
        hf = hc;
    }
    // list of ranges (node | level << 27), leaves already offered removed,
    // ordered by distance class: the squared gap to the nearest group box,
    // overlapping first, then in steps of 4 up to the largest bound, so
    // that the heaps tighten early and later candidates are rejected by the
    // bound
    int lcnt = 0;
    int l_near = 0;  // entries of the near classes
    {
        // class thresholds on the squared gap, as fractions of the largest bound
        double cth[kListClasses];
#pragma unroll
        for (int c = 1; c < kListClasses; c++)
            cth[c] = tmax * __builtin_ldexp(1.0, -2 * (kListClasses - 1 - c));
        // every entry's class once (4 bits per chunk of 64; the frontier
        // holds at most kLeafList entries), then one gather per class
        uint64_t cls_pack = 0;
        for (int base = 0, ci = 0; base < fcnt; base += 64, ci++) {
            const int i = base + lane;
            int cls = 15;  // not listed
            if (i < fcnt) {
                const uint32_t node = fc[i];
                const int64_t first = (int64_t)node << hf;
                const int64_t last = min(first + ((int64_t)1 << hf), n_leaf_total);
                const bool done = hf == 0 && first * HOP_LEAF >= seed_lo &&
                                  min(last * HOP_LEAF, a.n) <= seed_hi;
                const NodeBox nb = a.boxes[a.lv.off[hf] + node];
                double bd = boxbox_d2<PERIODIC>(gbox[0], nb, a.gmask);
#pragma unroll
                for (int g = 1; g < 8; g++) bd = fmin(bd, boxbox_d2<PERIODIC>(gbox[g], nb, a.gmask));
                int c0 = 0;
#pragma unroll
                for (int c = 1; c < kListClasses; c++) c0 += bd > (c == 1 ? 0.0 : cth[c - 1]) ? 1 : 0;
                cls = done ? 15 : c0;
            }
            cls_pack |= (uint64_t)cls << (4 * ci);
        }
        for (int pass = 0; pass < kListClasses; pass++) {
            for (int base = 0, ci = 0; base < fcnt; base += 64, ci++) {
                const int i = base + lane;
                const bool keep = i < fcnt && (int)((cls_pack >> (4 * ci)) & 15) == pass;
                const uint32_t e = keep ? (fc[i] | ((uint32_t)hf << 27)) : 0u;
                const uint64_t m = __ballot(keep);
                const int pos = lcnt + (int)__popcll(m & lt_mask);
                if (keep) leaves[pos] = e;
                lcnt += (int)__popcll(m);
            }
            if (pass == kNearClasses - 1) l_near = lcnt;
        }
    }
    __syncthreads();
    // unpark the heap
    if constexpr (!BIG) {
#pragma unroll
        for (int s = 5; s < kHeapMax; s++)
            if (s < hs) heap[s * 64 + lane] = park[s - 5];
        for (int s = hs; s < kSlots; s++) heap[s * 64 + lane] = 0;
    }
    __syncthreads();
    // 3. stream the listed leaves, 4 leaves (64 particles) per batch,
    //    loading batch b+1 while batch b is tested.  When every relevant
    //    separation stays under half the box, the loading lane moves each
    //    particle to its image nearest the bucket centre, so the testing
    //    lanes need no per-pair wrap.
    bool fastB = true;
    double cx = 0, cy = 0, cz = 0;
    if (PERIODIC) {
        const double r = __builtin_sqrt(tmax);
        const double half = 0.5 * G;
#pragma unroll
        for (int k = 0; k < 3; k++)
            if ((double)(bb.hi[k] - bb.lo[k]) + 2.0 * r + 2.0 >= half) fastB = false;
        cx = 0.5 * ((double)bb.lo[0] + (double)bb.hi[0]);
        cy = 0.5 * ((double)bb.lo[1] + (double)bb.hi[1]);
        cz = 0.5 * ((double)bb.lo[2] + (double)bb.hi[2]);
    }
    fastB = __builtin_amdgcn_readfirstlane(fastB ? 1 : 0) != 0;
    // every listed entry spans 2^hf leaves (a subtree cut by the end of the
    // tree yields indices past n, which the loader drops), so slot s of
    // batch b is leaf position 4b + s of the list
    int64_t n_stream = (int64_t)lcnt << hf;
    int nbatch = (int)((n_stream + 3) >> 2);
    // after the near classes, and then every kPruneEvery batches, the
    // entries not streamed yet are tested again against the groups' bounds
    // as they are then (the heaps tighten as the stream goes) and the list
    // is compacted; a cut falls where a batch boundary meets an entry and
    // an interleave-window boundary
    const int align = hf >= 2 ? 1 : (4 >> hf);
    const int bi_cut = (int)(((int64_t)(min(lcnt, ((l_near + align - 1) / align) * align)) << hf) >> 2);
    auto reprune = [&](const int e_cut) {
        double gt2[8];
        {
            double t = tau;
#pragma unroll
            for (int d = 1; d < 8; d <<= 1) t = fmax(t, __shfl_xor(t, d));
#pragma unroll
            for (int g = 0; g < 8; g++) {
                const long long tb = __double_as_longlong(t);
                const int tlo = __builtin_amdgcn_readlane((int)(tb & 0xffffffff), 8 * g);
                const int thi = __builtin_amdgcn_readlane((int)(tb >> 32), 8 * g);
                gt2[g] = __longlong_as_double(((long long)thi << 32) | (uint32_t)tlo);
            }
        }
        int nc = e_cut;
        for (int base = e_cut; base < lcnt; base += 64) {
            const int i = base + lane;
            bool keep = false;
            uint32_t e = 0;
            if (i < lcnt) {
                e = leaves[i];
                const NodeBox nb = a.boxes[a.lv.off[hf] + (e & ((1u << 27) - 1))];
#pragma unroll
                for (int g = 0; g < 8; g++) keep |= boxbox_d2<PERIODIC>(gbox[g], nb, a.gmask) <= gt2[g];
            }
            const uint64_t m = __ballot(keep);
            // entries of this chunk are in registers; writes land at or
            // before the chunk, never on an entry still to be read
            if (keep) leaves[nc + (int)__popcll(m & lt_mask)] = e;
            nc += (int)__popcll(m);
        }
        lcnt = nc;
        n_stream = (int64_t)lcnt << hf;
        nbatch = (int)((n_stream + 3) >> 2);
    };
    const int64_t omask = ((int64_t)1 << hf) - 1;
    auto fetch = [&](int bi, SortedRec &r) -> bool {
        int64_t pos = 4 * (int64_t)bi + (lane >> 4);
        if (pos >= n_stream) return false;
        // a full window of kWindow positions is streamed transposed (batch r
        // of the window takes positions r, r + kWindow/4, ...), so the four
        // leaves of a batch lie apart and favour different lanes: the
        // insertion loop runs as long as its busiest lane
        constexpr int64_t wm = kWindow - 1, q = kWindow / 4;
        if ((pos | wm) < n_stream) pos = (pos & ~wm) | ((pos & 3) * q) | ((pos >> 2) & (q - 1));
        const uint32_t e = leaves[(int)(pos >> hf)];
        const int64_t leaf = ((int64_t)(e & ((1u << 27) - 1)) << hf) + (pos & omask);
        const int64_t idx = leaf * HOP_LEAF + (lane & 15);
        if (idx < plo || idx >= phi) return false;          // another problem, or past n
        if (idx >= seed_lo && idx < seed_hi) return false;  // offered in the seed
        r = a.recs[idx];
        return true;
    };
    // Offers are deferred by one batch: a batch's marked particles (po)
    // wait in s_old while the next batch is staged and tested, and the
    // insertion loop runs until the older batch is done, lanes that finish
    // it early going on with the newer one (the loop runs as long as its
    // busiest lane, so this evens out the lanes' work across batches).
    // s_old alternates between the stage and heap slots 0..3, which are
    // free while levels 0 and 1 are in registers.  The key read one ahead
    // (dkey, dhave) is carried across batches.
    SortedRec *s_cur = stage, *s_old = reinterpret_cast<SortedRec *>(heap);
    uint64_t po = 0, dkey = ~0ull;
    bool dhave = false;
    auto next_key2 = [&](uint64_t &pn, bool wrap) -> uint64_t {
        const bool from_old = po != 0;
        const uint64_t p = from_old ? po : pn;
        const bool any = p != 0;
        const int k = __builtin_ctzll(p | (1ull << 63));
        const uint64_t rest = p & (p - 1);
        po = from_old ? rest : po;
        pn = from_old ? pn : rest;
        const SortedRec r = (from_old ? s_old : s_cur)[k];
        const double d2 = wrap ? d2_wrap(qx, qy, qz, r, G) : d2_direct(qx, qy, qz, r);
        const uint64_t key = make_key(d2, (uint32_t)r.tk, a);
        return any ? key : ~0ull;
    };
    auto offer = [&]() {
        if (!BIG && hs == kHeapMax) rh_replace_root63(H, heap, lane, (dhave && dkey < H.r0) ? dkey : H.r0);
        else if (dhave && dkey < H.r0) rh_replace_root(H, heap, lane, hs, dkey);
    };
    // one copy of the loop per distance form (FAST: images already chosen
    // by the loading lane, or no periodicity), so the tests carry no branch
    auto stream = [&](auto fast_tag) {
        constexpr bool FAST = decltype(fast_tag)::value;
        SortedRec nxt;
        bool nxt_ok = nbatch > 0 ? fetch(0, nxt) : false;
        // wait for the first batch here (vmcnt(0)): left outstanding into the
        // loop, it made the compiler wait for every batch's prefetch before
        // that batch's tests, so the prefetch overlapped nothing
        __builtin_amdgcn_s_waitcnt(0x0F70);
        int next_cut = bi_cut;
        for (int bi = 0; bi < nbatch; bi++) {
            if (bi == next_cut) {
                const int64_t p0 = 4 * (int64_t)bi;
                if ((p0 & (omask | (kWindow - 1))) != 0) {
                    next_cut = bi + 1;  // not an entry and window boundary yet
                } else {
                    next_cut = bi + kPruneEvery;
                    if ((int)(p0 >> hf) < lcnt) {
                        __syncthreads();
                        reprune((int)(p0 >> hf));
                        __syncthreads();
                        if (bi >= nbatch) break;
                        nxt_ok = fetch(bi, nxt);
                    }
                }
            }
            SortedRec r = nxt;
            const bool ok = nxt_ok;
            if (ok) {
                if (PERIODIC && FAST) {
                    const double half = 0.5 * G;
                    const double dx = r.x - cx, dy = r.y - cy, dz = r.z - cz;
                    r.x += dx > half ? -G : (dx < -half ? G : 0.0);
                    r.y += dy > half ? -G : (dy < -half ? G : 0.0);
                    r.z += dz > half ? -G : (dz < -half ? G : 0.0);
                }
            } else {
                r.x = r.y = r.z = 1.0e30;  // never selected
                r.j = -1;
                r.tk = -1;
            }
            __syncthreads();
            s_cur[lane] = r;
            if (FAST) stage_pp[lane] = __builtin_fma(r.x, r.x, __builtin_fma(r.y, r.y, r.z * r.z));
            __syncthreads();
            if (bi + 1 < nbatch) nxt_ok = fetch(bi + 1, nxt);
            if (!__any(ok)) continue;
            n_lv += 4;
            // the query itself never appears here: its own bucket lies in the
            // seeded range, which the loader skips
            uint64_t pass = 0;
            if (FAST) {
                // s = |p|^2 - 2 p.q - (tau - |q|^2) - 1/2 = d^2 - tau - 1/2:
                // every partial sum a multiple of 1/2 below 2^52, so the FMAs
                // are exact, and d^2 <= tau exactly when s < 0.  The sign bit
                // of s's high word is shifted into the mask (v_alignbit),
                // candidate k ending at bit k.  (tau < 0: no candidate.)
                const double tq = tau < 0.0 ? -1.0e300 : tau - qq;
                const double ntq = -(tq + 0.5);
                uint32_t wlo = 0u, whi = 0u;
#pragma unroll
                for (int k0 = 48; k0 >= 0; k0 -= 16) {
                    SortedRec pr[16];
                    double pp[16];
#pragma unroll
                    for (int k = 0; k < 16; k++) {
                        pr[k] = s_cur[k0 + k];
                        pp[k] = stage_pp[k0 + k];
                    }
#pragma unroll
                    for (int k = 15; k >= 0; k--) {
                        const double sv = __builtin_fma(m2x, pr[k].x, __builtin_fma(m2y, pr[k].y,
                                                        __builtin_fma(m2z, pr[k].z, pp[k] + ntq)));
                        const uint32_t sh = (uint32_t)((uint64_t)__double_as_longlong(sv) >> 32);
                        if (k0 + k >= 32) whi = __builtin_amdgcn_alignbit(whi, sh, 31);
                        else wlo = __builtin_amdgcn_alignbit(wlo, sh, 31);
                    }
                }
                pass = ((uint64_t)whi << 32) | wlo;
            }
#pragma unroll
            for (int k0 = 0; k0 < 64 && !FAST; k0 += 16) {
                SortedRec pr[16];
#pragma unroll
                for (int k = 0; k < 16; k++) pr[k] = s_cur[k0 + k];
                // per-pair minimum image (the bits go straight into the 64-bit
                // mask, shifted as 64-bit values)
#pragma unroll
                for (int k = 0; k < 16; k++) {
                    const bool ok_k = d2_wrap(qx, qy, qz, pr[k], G) <= tau;
                    pass |= (uint64_t)(ok_k ? 1u : 0u) << (k0 + k);
                }
            }
            // finish the older batch; lanes done with it take this one's
            if (counting) count_offers(pass, (uint32_t)__popcll(po));
            uint64_t pn = pass;
            while (__any(po != 0)) {
                const bool hn = (po | pn) != 0;
                const uint64_t kn = next_key2(pn, PERIODIC && !FAST);
                offer();
                dhave = hn;
                dkey = kn;
            }
            po = pn;
            SortedRec *t = s_cur;
            s_cur = s_old;
            s_old = t;
            if (active) tau = fmin(key_d2(H.r0, a.shift), rcap);
        }
    };
    const bool wrap_tail = PERIODIC && !fastB;
    if (!PERIODIC || fastB) stream(std::true_type{});
    else stream(std::false_type{});
    {
        // the last batch's deferred offers
        if (counting) count_offers(0, (uint32_t)__popcll(po) + ((dhave || po != 0) ? 1u : 0u));
        uint64_t pn = 0;
        while (__any(dhave || po != 0)) {
            const bool hn = po != 0;
            const uint64_t kn = next_key2(pn, wrap_tail);
            offer();
            dhave = hn;
            dkey = kn;
        }
    }
    __syncthreads();  // every read of s_old done before slots 0..4 are rewritten
    // write the register levels back so the heap is whole in LDS
    heap[lane] = H.r0;
#pragma unroll
    for (int q = 0; q < 4; q++) heap[(q + 1) * 64 + lane] = H.r1[q];

    if (a.counters && lane == 0) {
        atomicAdd(&a.counters[0], n_nodes);
        atomicAdd(&a.counters[1], n_lv);
        atomicAdd(&a.counters[2], n_it);
    }
    if (counting) {
        unsigned long long t = active ? n_off : 0ull;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) t += (unsigned long long)__shfl_xor((long long)t, d);
        if (lane == 0) atomicAdd(&a.counters[3], t);
    }
    // a bounded search is exact for a lane whose whole list lies inside its
    // radius; the other lanes are searched again without it
    bool miss = false;
    if (a.cell_r) {
        miss = active && (H.r0 == ~0ull || key_d2(H.r0, a.shift) > rcap);
        const uint64_t mm = __ballot(miss);
        if (lane == 0 && mm) a.miss[bucket_id] = mm;
    }
    if (!active || miss) return;

    const int32_t jq = me.j;
    if constexpr (BIG) {
        // in-place heapsort in LDS: the keys ascending in slots [0, hs)
        for (int e = hs - 1; e >= 1; e--) {
            const uint64_t top = heap[lane], last = heap[e * 64 + lane];
            heap[e * 64 + lane] = top;
            lds_sift_size(heap, lane, e, 0, last);
        }
        auto d2_at = [&](int t) -> uint64_t { return heap[t * 64 + lane] >> a.shift; };
        const uint64_t R = d2_at(hs - 1);
        if (R == 0) atomicOr(a.dflags, DERR_DEGENERATE);
        if ((double)R >= a.maxd2) atomicOr(a.dflags, DERR_KEYWIDTH);
        const double Rd = (double)(R == 0 ? 1 : R);
        double delta;
        if (!a.fp32) {
            const double wsum = pairwise_spline<128, double>(a.n_dens, Rd, d2_at, m4_shape);
            const double h2 = Rd * 0.25;
            const double hh = __builtin_sqrt(h2);
            const double h3 = h2 * hh;
            delta = (wsum * norm) / h3;
        } else {
            const float Rf = (float)Rd;
            const float wsum = pairwise_spline<128, float>(a.n_dens, Rf, d2_at, m4_shape_f32);
            const float h2 = Rf * 0.25f;
            const float hh = __builtin_sqrtf(h2);
            const float h3 = h2 * hh;
            delta = (double)((wsum * norm32) / h3);
        }
        a.dens[jq] = delta;
        auto col = [&](int t) -> int32_t {
            if (t == 0) return jq;
            const uint32_t tkv = (uint32_t)(heap[(t - 1) * 64 + lane] & a.tk_mask);
            // an unfilled slot (flagged above) must not index the table
            if (tkv >= (uint64_t)a.n) return -1;
            return IDS ? a.tk2j[tkv] : (int32_t)tkv;
        };
        if (a.nbr16s) {
            int4 *dst = reinterpret_cast<int4 *>(a.nbr16s + (b0 + lane) * 16);
#pragma unroll
            for (int q = 0; q < 4; q++)
                dst[q] = make_int4(col(4 * q), col(4 * q + 1), col(4 * q + 2), col(4 * q + 3));
            a.dens_s[b0 + lane] = delta;
        }
        if (a.nbr) {
            int32_t *row = a.nbr + (int64_t)jq * a.k_store;
            if (a.vec_store) {
                for (int t = 0; t < a.k_store; t += 4)
                    *reinterpret_cast<int4 *>(row + t) = make_int4(col(t), col(t + 1), col(t + 2), col(t + 3));
            } else {
                for (int t = 0; t < a.k_store; t++) row[t] = col(t);
            }
        }
        return;
    } else {
    // sort the heap ascending in registers (bitonic network over 64 slots)
    uint64_t v[64];
#pragma unroll
    for (int s = 0; s < 64; s++) v[s] = s < hs ? heap[s * 64 + lane] : ~0ull;
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
#pragma unroll
            for (int i = 0; i < 64; i++) {
                const int l = i ^ jj;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const uint64_t x = v[i], y = v[l];
                    const bool sw = up ? (x > y) : (x < y);
                    v[i] = sw ? y : x;
                    v[l] = sw ? x : y;
                }
            }
        }
    }

    // density: L = [self, v[0..hs)], R = d^2 of the farthest
    uint64_t vfar = 0;  // v[hs-1] without a dynamic register index
#pragma unroll
    for (int t = 0; t < 64; t++)
        if (t == hs - 1) vfar = v[t];
    const uint64_t R = vfar >> a.shift;
    if (R == 0) atomicOr(a.dflags, DERR_DEGENERATE);
    if ((double)R >= a.maxd2) atomicOr(a.dflags, DERR_KEYWIDTH);
    const double Rd = (double)(R == 0 ? 1 : R);
    auto d2_at = [&](int t) -> uint64_t { return v[t] >> a.shift; };
    double delta;
    if (!a.fp32) {
        const double wsum = pairwise_spline<64, double>(a.n_dens, Rd, d2_at, m4_shape);
        const double h2 = Rd * 0.25;
        const double hh = __builtin_sqrt(h2);
        const double h3 = h2 * hh;
        delta = (wsum * norm) / h3;
    } else {
        // same operation sequence in FP32; 4 d^2 and r_max^2 are rounded to
        // FP32 on conversion, everything after runs in FP32
        const float Rf = (float)Rd;
        const float wsum = pairwise_spline<64, float>(a.n_dens, Rf, d2_at, m4_shape_f32);
        const float h2 = Rf * 0.25f;
        const float hh = __builtin_sqrtf(h2);
        const float h3 = h2 * hh;
        delta = (double)((wsum * norm32) / h3);
    }

    a.dens[jq] = delta;
    auto col = [&](int t) -> int32_t {
        if (t == 0) return jq;
        const uint32_t tkv = (uint32_t)(v[t - 1] & a.tk_mask);
        // an unfilled slot (flagged above) must not index the table
        if (tkv >= (uint64_t)a.n) return -1;
        return IDS ? a.tk2j[tkv] : (int32_t)tkv;
    };
    if (a.nbr16s) {
        int4 *dst = reinterpret_cast<int4 *>(a.nbr16s + (b0 + lane) * 16);
#pragma unroll
        for (int q = 0; q < 4; q++)
            dst[q] = make_int4(col(4 * q), col(4 * q + 1), col(4 * q + 2), col(4 * q + 3));
        a.dens_s[b0 + lane] = delta;
    }
    if (a.nbr) {
        int32_t *row = a.nbr + (int64_t)jq * a.k_store;
        if (a.vec_store) {
#pragma unroll
            for (int t = 0; t < 64; t += 4) {
                if (t < a.k_store) {
                    int4 q4 = make_int4(col(t), col(t + 1), col(t + 2), col(t + 3));
                    *reinterpret_cast<int4 *>(row + t) = q4;
                }
            }
        } else {
#pragma unroll
            for (int t = 0; t < 64; t++)
                if (t < a.k_store) row[t] = col(t);
        }
    }
    }
}

// One box, persistent: 4 workgroups of one wave per compute unit (2 for
// n_dens > 64) take buckets of 64 sorted particles from 8 queues, queue x
// holding the contiguous run of buckets of XCD x (consecutive blocks land
// on different XCDs, so neighbouring buckets share candidate leaves in one
// L2); a workgroup whose queue is empty goes on with the next queue, and
// leaves once it has found all 8 empty.  Against one workgroup per bucket
// this saves the workgroup launch and dispatch gaps (about 5% of the time).
template <bool PERIODIC, bool IDS, bool BIG, bool COUNT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_knn_density(
    KnnArgs a, uint32_t *__restrict__ queue)
{
    __shared__ __align__(16) uint64_t heap[heap_slots<BIG>() * 64];
    __shared__ uint32_t front[BIG ? 2 * kFrontLevelBig : 1];
    __shared__ SortedRec stage[64];
    __shared__ double stage_pp[64];
    __shared__ uint32_t leaves[kLeafList];
    const int lane = threadIdx.x;
    int q = (int)(blockIdx.x & 7);
    int dry = 0;
    while (dry < 8) {
        uint32_t t = 0;
        if (lane == 0) t = atomicAdd(&queue[q], 1u);
        t = (uint32_t)__shfl((int)t, 0);
        const int64_t bucket = (int64_t)q * a.xcd_chunk + (int64_t)t;
        if ((int64_t)t >= a.xcd_chunk || bucket >= a.n_buckets) {
            q = (q + 1) & 7;
            dry++;
            continue;
        }
        __syncthreads();
        const int64_t b0 = bucket * HOP_BUCKET;
        knn_bucket<PERIODIC, IDS, BIG, COUNT>(a, b0, (int)min((int64_t)HOP_BUCKET, a.n - b0), 0, a.n,
                                              a.norm, a.norm32, heap, front, stage, stage_pp, leaves,
                                              ~0ull, bucket);
    }
}

// Fallback of a bounded search: the listed buckets again, without a radius,
// for the lanes recorded in miss[bucket] only.
template <bool PERIODIC, bool IDS, bool BIG>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_knn_redo(
    KnnArgs a, const uint32_t *__restrict__ list, const unsigned long long *__restrict__ miss)
{
    __shared__ __align__(16) uint64_t heap[heap_slots<BIG>() * 64];
    __shared__ uint32_t front[BIG ? 2 * kFrontLevelBig : 1];
    __shared__ SortedRec stage[64];
    __shared__ double stage_pp[64];
    __shared__ uint32_t leaves[kLeafList];
    const int64_t bucket = list[blockIdx.x];
    const int64_t b0 = bucket * HOP_BUCKET;
    knn_bucket<PERIODIC, IDS, BIG, false>(a, b0, (int)min((int64_t)HOP_BUCKET, a.n - b0), 0, a.n,
                                          a.norm, a.norm32, heap, front, stage, stage_pp, leaves,
                                          miss[bucket], bucket);
}

// buckets with a recorded miss -> list; count the missed lanes
__global__ void k_miss_list(int64_t n_buckets, const unsigned long long *__restrict__ miss,
                            uint32_t *__restrict__ list, uint32_t *__restrict__ counts)
{
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_buckets) return;
    const unsigned long long m = miss[b];
    if (!m) return;
    list[atomicAdd(&counts[0], 1u)] = (uint32_t)b;
    atomicAdd(&counts[1], (uint32_t)__popcll(m));
}

// A batch of independent subvolumes, one persistent wave per SIMD.  Work
// items are buckets, numbered subvolume by subvolume in the order `order`
// (largest first by default) and cut into one contiguous chunk per XCD;
// a wave takes items from its XCD's chunk and, when that runs dry, from the
// next chunks in turn, and exits when all are dry.
template <bool PERIODIC, bool BIG>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_knn_batch(KnnArgs a,
                                                                                             BatchArgs b)
{
    __shared__ __align__(16) uint64_t heap[heap_slots<BIG>() * 64];
    __shared__ uint32_t front[BIG ? 2 * kFrontLevelBig : 1];
    __shared__ SortedRec stage[64];
    __shared__ double stage_pp[64];
    __shared__ uint32_t leaves[kLeafList];
    const int lane = threadIdx.x;
    const int nq = b.xcd_queues ? 8 : 1;
    const int64_t chunk = (b.n_items + nq - 1) / nq;
    int q = b.xcd_queues ? (int)(blockIdx.x & 7) : 0;
    int dry = 0;
    while (dry < nq) {
        uint32_t t = 0;
        if (lane == 0) t = atomicAdd(&b.queue[q], 1u);
        t = (uint32_t)__shfl((int)t, 0);
        const int64_t item = (int64_t)q * chunk + (int64_t)t;
        if ((int64_t)t >= chunk || item >= b.n_items) {
            q = q + 1 == nq ? 0 : q + 1;
            dry++;
            continue;
        }
        // k: item_off[k] <= item < item_off[k + 1]
        int lo = 0, hi = b.n_sub;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (b.item_off[mid] <= item) lo = mid;
            else hi = mid;
        }
        const int sv = b.order[lo];
        const int64_t plo = b.sub_off[sv], phi = b.sub_off[sv + 1];
        const int64_t b0 = plo + (item - b.item_off[lo]) * HOP_BUCKET;
        __syncthreads();
        knn_bucket<PERIODIC, false, BIG, false>(a, b0, (int)min((int64_t)HOP_BUCKET, phi - b0), plo, phi,
                                         b.norm[sv], b.norm32[sv], heap, front, stage, stage_pp,
                                         leaves, ~0ull, 0);
        if (lane == 0) atomicAdd(&b.done[sv], 1u);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

namespace {

// Morton keys of a batch: the subvolume number in the top sub_bits bits,
// then the Morton code without its lowest sub_bits - 1 bits.  The order
// inside a subvolume only affects locality, never a result.
__global__ void k_morton_batch(const uint32_t *__restrict__ pos, int64_t n, uint32_t glim,
                               const int64_t *__restrict__ sub_off, int n_sub, int sub_bits,
                               uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
                               uint32_t *__restrict__ dflags)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = n_sub;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (sub_off[mid] <= i) lo = mid;
        else hi = mid;
    }
    uint32_t x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    if (x >= glim || y >= glim || z >= glim) {
        atomicOr(dflags, DERR_RANGE);
        x = min(x, glim - 1);
        y = min(y, glim - 1);
        z = min(z, glim - 1);
    }
    const uint64_t m = (spread3(x) << 2) | (spread3(y) << 1) | spread3(z);
    keys[i] = ((uint64_t)lo << (64 - sub_bits)) | (m >> (sub_bits - 1));
    vals[i] = (uint32_t)i;
}

// HIP events that are destroyed on every exit path
struct Events {
    hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
    ~Events()
    {
        for (auto &x : e)
            if (x) (void)hipEventDestroy(x);
    }
    hipError_t create()
    {
        for (auto &x : e) {
            hipError_t r = hipEventCreate(&x);
            if (r != hipSuccess) return r;
        }
        return hipSuccess;
    }
};

// Sorted copy (permutation in ctx->vals_a) and the implicit tree over it.
int build_tree(hop_ctx *ctx, int64_t n, const uint32_t *pos, const uint64_t *codes, const int32_t *tk,
               uint32_t glim, hipStream_t s, TreeLevels &lv, SortedRec *&recs, NodeBox *&boxes)
{
    const uint32_t *perm = (const uint32_t *)ctx->vals_a.ptr;
    HOPTRY(hop_reserve(ctx, ctx->recs, (size_t)n * sizeof(SortedRec)));
    recs = (SortedRec *)ctx->recs.ptr;
    k_gather_recs<<<hop_grid(n, 256), 256, 0, s>>>(pos, codes, perm, tk, n, glim, recs);
    HOPCHK(ctx, hipGetLastError());

    lv = TreeLevels{};
    const int64_t n_leaves = hop_div_up(n, HOP_LEAF);
    int64_t total = 0, cnt = n_leaves;
    int lvl = 0;
    for (;;) {
        if (lvl >= HOP_MAX_LEVELS) return hop_fail(ctx, HOP_ERR_ARG, "tree too deep");
        lv.off[lvl] = total;
        lv.cnt[lvl] = (int32_t)cnt;
        total += cnt;
        if (cnt == 1 && lvl >= 2) break;
        cnt = hop_div_up(cnt, 2);
        lvl++;
    }
    lv.top = lvl;
    HOPTRY(hop_reserve(ctx, ctx->boxes, (size_t)total * sizeof(NodeBox)));
    boxes = (NodeBox *)ctx->boxes.ptr;
    k_leaf_boxes<<<hop_grid(n_leaves, 256), 256, 0, s>>>(recs, n, n_leaves, boxes);
    HOPCHK(ctx, hipGetLastError());
    for (int h = 1; h <= lv.top; h++) {
        k_level_boxes<<<hop_grid(lv.cnt[h], 256), 256, 0, s>>>(boxes, lv.off[h - 1], lv.cnt[h - 1],
                                                               lv.off[h], lv.cnt[h]);
        HOPCHK(ctx, hipGetLastError());
    }
    return HOP_OK;
}

double norm_of(const hop_params *p, double mean_density, int64_t n)
{
    const double md = mean_density > 0 ? mean_density
                                        : (double)n / (double)(1ull << (3 * p->grid_bits));
    return 1.0 / (3.141592653589793 * md);
}

// Fields shared by the single-box and batched launches.
void base_args(hop_ctx *ctx, KnnArgs &a, int64_t n, const hop_params *p, SortedRec *recs,
               NodeBox *boxes, const TreeLevels &lv, double *density, int32_t *nbr,
               const int32_t *tk2j)
{
    const uint32_t glim = 1u << p->grid_bits;
    a = KnnArgs{};
    a.recs = recs;
    a.boxes = boxes;
    a.lv = lv;
    a.n = n;
    a.n_buckets = hop_div_up(n, HOP_BUCKET);
    a.xcd_chunk = hop_div_up(a.n_buckets, 8);
    a.hs = p->n_dens - 1;
    a.n_dens = p->n_dens;
    a.k_store = p->k_store;
    int shift = 1;
    while (shift < 31 && ((int64_t)1 << shift) < n) shift++;
    a.shift = shift;
    a.tk_mask = (1ull << shift) - 1;
    a.maxd2 = (double)((~0ull) >> shift);
    if (a.maxd2 > 9.0e15) a.maxd2 = 9.0e15;  // d^2 < 3*2^42 never reaches this
    a.fp32 = (p->flags & HOP_DENSITY_FP32) ? 1 : 0;
    a.gsize = (double)glim;
    a.gmask = glim - 1;
    a.front_cap = std::min(std::max((int)ctx->tuning.front_cap, 1), kFront);
    a.vec_store = nbr && (p->k_store % 4 == 0) && (((uintptr_t)nbr & 15) == 0);
    a.nbr = nbr;
    a.dens = density;
    a.tk2j = tk2j;
    a.dflags = (uint32_t *)ctx->flags.ptr;
    a.counters = nullptr;
}

int finish_stats(hop_ctx *ctx, Events &ev, const KnnArgs &a, int64_t n)
{
    if (!ctx->profiling) return HOP_OK;
    HOPCHK(ctx, hipEventSynchronize(ev.e[2]));
    // e[0] start, e[1] tree built, e[3] radius model done (learned only),
    // e[2] kNN done
    float t0 = 0, t1 = 0, tr = 0;
    HOPCHK(ctx, hipEventElapsedTime(&t0, ev.e[0], ev.e[1]));
    if (a.cell_r) {
        HOPCHK(ctx, hipEventElapsedTime(&tr, ev.e[1], ev.e[3]));
        HOPCHK(ctx, hipEventElapsedTime(&t1, ev.e[3], ev.e[2]));
    } else {
        HOPCHK(ctx, hipEventElapsedTime(&t1, ev.e[1], ev.e[2]));
    }
    unsigned long long c[4] = {0, 0, 0, 0};
    if (a.counters) HOPCHK(ctx, hipMemcpy(c, a.counters, 32, hipMemcpyDeviceToHost));
    ctx->stats.ms_sort = t0;
    ctx->stats.ms_knn = t1;
    ctx->stats.ms_radius = tr;
    ctx->stats.misses = 0;
    ctx->stats.redo_buckets = 0;
    ctx->stats.n = n;
    ctx->stats.nodes_visited = (int64_t)c[0];
    ctx->stats.leaves_scanned = (int64_t)c[1];
    ctx->stats.insert_iterations = (int64_t)c[2];
    ctx->stats.offered = (int64_t)c[3];
    return HOP_OK;
}

// the counting instance only when counters are on
template <bool PERIODIC, bool IDS, bool BIG>
void launch_density(const KnnArgs &a, uint32_t *queue, int waves, hipStream_t s)
{
    if (a.counters) k_knn_density<PERIODIC, IDS, BIG, true><<<waves, 64, 0, s>>>(a, queue);
    else k_knn_density<PERIODIC, IDS, BIG, false><<<waves, 64, 0, s>>>(a, queue);
}

int start_counters(hop_ctx *ctx, KnnArgs &a, hipStream_t s)
{
    if (ctx->profiling & 2) {
        a.counters = (unsigned long long *)((char *)ctx->flags.ptr + 256);
        HOPCHK(ctx, hipMemsetAsync(a.counters, 0, 32, s));
    }
    return HOP_OK;
}

}  // namespace

int hop_density_impl(hop_ctx *ctx, int64_t n, const uint32_t *pos, const int64_t *id,
                     const hop_params *p, double *density, int32_t *nbr, int32_t *nbr16s,
                     double *dens_s, hipStream_t s)
{
    const uint32_t glim = 1u << p->grid_bits;
    const bool periodic = (p->flags & HOP_PERIODIC) != 0;
    uint32_t *dflags = (uint32_t *)ctx->flags.ptr;

    Events ev;
    if (ctx->profiling) {
        HOPCHK(ctx, ev.create());
        HOPCHK(ctx, hipEventRecord(ev.e[0], s));
    }

    const int32_t *tk = nullptr, *tk2j = nullptr;
    if (id) {
        HOPTRY(hop_build_tiekeys(ctx, n, id, s));
        tk = (const int32_t *)ctx->tk.ptr;
        tk2j = (const int32_t *)ctx->tk2j.ptr;
    }

    // 1. Morton sort
    HOPTRY(hop_reserve(ctx, ctx->keys_a, (size_t)n * 8));
    HOPTRY(hop_reserve(ctx, ctx->keys_b, (size_t)n * 8));
    HOPTRY(hop_reserve(ctx, ctx->vals_a, (size_t)n * 4));
    HOPTRY(hop_reserve(ctx, ctx->vals_b, (size_t)n * 4));
    uint64_t *keys = (uint64_t *)ctx->keys_a.ptr;
    uint32_t *perm = (uint32_t *)ctx->vals_a.ptr;
    k_morton<<<hop_grid(n, 256), 256, 0, s>>>(pos, n, glim, keys, perm, dflags);
    HOPCHK(ctx, hipGetLastError());
    // the top 48 bits of the code order cells of 2^(grid_bits - 16) grid
    // units, far below the mean spacing at any n < 2^31: particles sharing
    // a cell keep their input order, which only the locality of the search
    // depends on (its result does not), and two radix passes are saved
    const int code_bits = 3 * (int)p->grid_bits;
    HOPTRY(hop_radix_sort(ctx, keys, perm, (uint64_t *)ctx->keys_b.ptr, (uint32_t *)ctx->vals_b.ptr,
                          n, code_bits, s, std::max(0, code_bits - 48)));
    ctx->perm_n = n;

    // 2. sorted copy and tree
    TreeLevels lv;
    SortedRec *recs = nullptr;
    NodeBox *boxes = nullptr;
    HOPTRY(build_tree(ctx, n, pos, keys, tk, glim, s, lv, recs, boxes));
    if (ctx->profiling) HOPCHK(ctx, hipEventRecord(ev.e[1], s));

    // 3. kNN + density (bounded by the per-cell search radius if asked for)
    KnnArgs a;
    base_args(ctx, a, n, p, recs, boxes, lv, density, nbr, tk2j);
    a.nbr16s = nbr16s;
    a.dens_s = dens_s;
    a.norm = norm_of(p, p->mean_density, n);
    a.norm32 = (float)a.norm;
    const bool learned = (p->flags & HOP_LEARNED_RADIUS) != 0;
    if (learned) {
        HOPTRY(hop_radius_cells(ctx, n, pos, p, s, &a.cell_r, &a.cell_bits, &a.cell_gb));
        HOPTRY(hop_reserve(ctx, ctx->miss, (size_t)a.n_buckets * 8 + 4 * (size_t)a.n_buckets + 64));
        a.miss = (unsigned long long *)ctx->miss.ptr;
        HOPCHK(ctx, hipMemsetAsync(a.miss, 0, (size_t)a.n_buckets * 8, s));
    }
    if (ctx->profiling) HOPCHK(ctx, hipEventRecord(ev.e[3], s));
    HOPTRY(start_counters(ctx, a, s));
    if (a.xcd_chunk >= ((int64_t)1 << 31)) return hop_fail(ctx, HOP_ERR_ARG, "too many particles");
    const bool big = p->n_dens > kHeapMax + 1;
    // the persistent launch: 8 queue cursors in the context's flag block,
    // zero at launch; as many workgroups as fit at once (one wave per SIMD,
    // or two per compute unit for the larger heap), no more than buckets
    uint32_t *queue = (uint32_t *)((char *)ctx->flags.ptr + 512);
    HOPCHK(ctx, hipMemsetAsync(queue, 0, 8 * sizeof(uint32_t), s));
    int64_t waves = ctx->tuning.persistent_waves > 0 ? ctx->tuning.persistent_waves
                                                     : (int64_t)(big ? 2 : 4) * ctx->n_cu;
    waves = std::max<int64_t>(8, std::min<int64_t>(waves, a.xcd_chunk * 8));
    if (big) {
        if (periodic) {
            if (id) launch_density<true, true, true>(a, queue, (int)waves, s);
            else launch_density<true, false, true>(a, queue, (int)waves, s);
        } else {
            if (id) launch_density<false, true, true>(a, queue, (int)waves, s);
            else launch_density<false, false, true>(a, queue, (int)waves, s);
        }
    } else if (periodic) {
        if (id) launch_density<true, true, false>(a, queue, (int)waves, s);
        else launch_density<true, false, false>(a, queue, (int)waves, s);
    } else {
        if (id) launch_density<false, true, false>(a, queue, (int)waves, s);
        else launch_density<false, false, false>(a, queue, (int)waves, s);
    }
    HOPCHK(ctx, hipGetLastError());
    int64_t misses = 0, redo = 0;
    if (learned) {
        uint32_t *list = (uint32_t *)((char *)ctx->miss.ptr + (size_t)a.n_buckets * 8);
        uint32_t *cnt = (uint32_t *)ctx->flags.ptr + 8;
        HOPCHK(ctx, hipMemsetAsync(cnt, 0, 8, s));
        k_miss_list<<<hop_grid(a.n_buckets, 256), 256, 0, s>>>(a.n_buckets, a.miss, list, cnt);
        HOPCHK(ctx, hipGetLastError());
        HOPCHK(ctx, hipMemcpyAsync(&ctx->hflags[8], cnt, 8, hipMemcpyDeviceToHost, s));
        HOPCHK(ctx, hipStreamSynchronize(s));
        const uint32_t *hc = (const uint32_t *)&ctx->hflags[8];
        redo = hc[0];
        misses = hc[1];
        if (redo > 0) {
            KnnArgs r = a;
            r.cell_r = nullptr;
            if (big) {
                if (periodic) {
                    if (id) k_knn_redo<true, true, true><<<(int)redo, 64, 0, s>>>(r, list, a.miss);
                    else k_knn_redo<true, false, true><<<(int)redo, 64, 0, s>>>(r, list, a.miss);
                } else {
                    if (id) k_knn_redo<false, true, true><<<(int)redo, 64, 0, s>>>(r, list, a.miss);
                    else k_knn_redo<false, false, true><<<(int)redo, 64, 0, s>>>(r, list, a.miss);
                }
            } else if (periodic) {
                if (id) k_knn_redo<true, true, false><<<(int)redo, 64, 0, s>>>(r, list, a.miss);
                else k_knn_redo<true, false, false><<<(int)redo, 64, 0, s>>>(r, list, a.miss);
            } else {
                if (id) k_knn_redo<false, true, false><<<(int)redo, 64, 0, s>>>(r, list, a.miss);
                else k_knn_redo<false, false, false><<<(int)redo, 64, 0, s>>>(r, list, a.miss);
            }
            HOPCHK(ctx, hipGetLastError());
        }
    }
    if (ctx->profiling) HOPCHK(ctx, hipEventRecord(ev.e[2], s));
    HOPTRY(finish_stats(ctx, ev, a, n));
    ctx->stats.misses = misses;
    ctx->stats.redo_buckets = redo;
    return HOP_OK;
}

int hop_density_batch_impl(hop_ctx *ctx, int32_t n_sub, const int64_t *off, const uint32_t *pos,
                           const double *mean_density, const hop_params *p, double *density,
                           int32_t *nbr, int32_t *nbr16s, double *dens_s, int64_t **sub_off_dev,
                           hipStream_t s)
{
    const uint32_t glim = 1u << p->grid_bits;
    const bool periodic = (p->flags & HOP_PERIODIC) != 0;
    uint32_t *dflags = (uint32_t *)ctx->flags.ptr;
    const int64_t n = off[n_sub];
    ctx->perm_n = 0;

    Events ev;
    if (ctx->profiling) {
        HOPCHK(ctx, ev.create());
        HOPCHK(ctx, hipEventRecord(ev.e[0], s));
    }

    // work description: subvolume order, first bucket of each, norms
    std::vector<int32_t> order(n_sub);
    for (int k = 0; k < n_sub; k++) order[k] = k;
    if (ctx->tuning.largest_first)
        std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
            return off[x + 1] - off[x] > off[y + 1] - off[y];
        });
    std::vector<int64_t> item_off(n_sub + 1);
    item_off[0] = 0;
    for (int k = 0; k < n_sub; k++)
        item_off[k + 1] = item_off[k] + hop_div_up(off[order[k] + 1] - off[order[k]], HOP_BUCKET);
    std::vector<double> nrm(n_sub);
    std::vector<float> nrm32(n_sub);
    for (int k = 0; k < n_sub; k++) {
        nrm[k] = norm_of(p, mean_density ? mean_density[k] : 0.0, off[k + 1] - off[k]);
        nrm32[k] = (float)nrm[k];
    }
    const size_t n1 = (size_t)n_sub + 1;
    size_t o_sub = 0, o_ord = o_sub + 8 * n1, o_item = (o_ord + 4 * n1 + 7) & ~(size_t)7;
    size_t o_nrm = o_item + 8 * n1, o_n32 = o_nrm + 8 * n1, o_q = (o_n32 + 4 * n1 + 63) & ~(size_t)63;
    size_t o_done = o_q + 64, bytes = o_done + 4 * n1;
    std::vector<char> host(bytes, 0);
    std::memcpy(host.data() + o_sub, off, 8 * n1);
    std::memcpy(host.data() + o_ord, order.data(), 4 * (size_t)n_sub);
    std::memcpy(host.data() + o_item, item_off.data(), 8 * n1);
    std::memcpy(host.data() + o_nrm, nrm.data(), 8 * (size_t)n_sub);
    std::memcpy(host.data() + o_n32, nrm32.data(), 4 * (size_t)n_sub);
    HOPTRY(hop_reserve(ctx, ctx->batch_tab, bytes));
    char *tab = (char *)ctx->batch_tab.ptr;
    HOPCHK(ctx, hipMemcpyAsync(tab, host.data(), bytes, hipMemcpyHostToDevice, s));
    HOPCHK(ctx, hipStreamSynchronize(s));  // `host` goes out of scope
    const int64_t *sub_off = (const int64_t *)(tab + o_sub);
    *sub_off_dev = (int64_t *)(tab + o_sub);

    // 1. keys (subvolume, Morton) and sort
    int sub_bits = 1;
    while (((int64_t)1 << sub_bits) < n_sub) sub_bits++;
    HOPTRY(hop_reserve(ctx, ctx->keys_a, (size_t)n * 8));
    HOPTRY(hop_reserve(ctx, ctx->keys_b, (size_t)n * 8));
    HOPTRY(hop_reserve(ctx, ctx->vals_a, (size_t)n * 4));
    HOPTRY(hop_reserve(ctx, ctx->vals_b, (size_t)n * 4));
    uint64_t *keys = (uint64_t *)ctx->keys_a.ptr;
    uint32_t *perm = (uint32_t *)ctx->vals_a.ptr;
    k_morton_batch<<<hop_grid(n, 256), 256, 0, s>>>(pos, n, glim, sub_off, n_sub, sub_bits, keys,
                                                    perm, dflags);
    HOPCHK(ctx, hipGetLastError());
    HOPTRY(hop_radix_sort(ctx, keys, perm, (uint64_t *)ctx->keys_b.ptr, (uint32_t *)ctx->vals_b.ptr,
                          n, 64, s));

    // 2. one tree over the whole batch; the walk stays inside a subvolume
    TreeLevels lv;
    SortedRec *recs = nullptr;
    NodeBox *boxes = nullptr;
    // (the batch keys drop low code bits: positions are gathered)
    HOPTRY(build_tree(ctx, n, pos, nullptr, nullptr, glim, s, lv, recs, boxes));
    if (ctx->profiling) HOPCHK(ctx, hipEventRecord(ev.e[1], s));

    // 3. persistent kNN + density over all buckets of all subvolumes
    KnnArgs a;
    base_args(ctx, a, n, p, recs, boxes, lv, density, nbr, nullptr);
    a.nbr16s = nbr16s;
    a.dens_s = dens_s;
    HOPTRY(start_counters(ctx, a, s));
    BatchArgs b{};
    b.sub_off = sub_off;
    b.order = (const int32_t *)(tab + o_ord);
    b.item_off = (const int64_t *)(tab + o_item);
    b.norm = (const double *)(tab + o_nrm);
    b.norm32 = (const float *)(tab + o_n32);
    b.queue = (uint32_t *)(tab + o_q);
    b.done = (uint32_t *)(tab + o_done);
    b.n_items = item_off[n_sub];
    b.n_sub = n_sub;
    b.xcd_queues = ctx->tuning.xcd_queues ? 1 : 0;
    // one wave per SIMD fits the default kernel's LDS; the n_dens > 64
    // kernel's larger heap leaves room for two waves per compute unit
    const bool big = p->n_dens > kHeapMax + 1;
    int waves = ctx->tuning.persistent_waves > 0 ? ctx->tuning.persistent_waves
                                                 : (big ? 2 : 4) * ctx->n_cu;
    if (waves < 8) waves = 8;
    if (big) {
        if (periodic) k_knn_batch<true, true><<<waves, 64, 0, s>>>(a, b);
        else k_knn_batch<false, true><<<waves, 64, 0, s>>>(a, b);
    } else if (periodic) {
        k_knn_batch<true, false><<<waves, 64, 0, s>>>(a, b);
    } else {
        k_knn_batch<false, false><<<waves, 64, 0, s>>>(a, b);
    }
    HOPCHK(ctx, hipGetLastError());
    if (ctx->profiling) HOPCHK(ctx, hipEventRecord(ev.e[2], s));

    // every bucket of every subvolume must have been processed once
    std::vector<uint32_t> done(n_sub);
    HOPCHK(ctx, hipMemcpyAsync(done.data(), b.done, 4 * (size_t)n_sub, hipMemcpyDeviceToHost, s));
    HOPCHK(ctx, hipStreamSynchronize(s));
    for (int k = 0; k < n_sub; k++)
        if ((int64_t)done[k] != hop_div_up(off[k + 1] - off[k], HOP_BUCKET))
            return hop_fail(ctx, HOP_ERR_ARG, "batched kNN left work undone");
    return finish_stats(ctx, ev, a, n);
}
