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
// max-heap in LDS, keyed by (d^2 << B) | tie_key, which orders candidates by
// (d^2, id) exactly (d^2 is an exact integer held in FP64).  The heap starts
// from the bucket's own particles, then the wave walks the tree nearest
// child first; a node is visited when ANY lane's heap could still take a
// particle from it, a leaf's 16 particles are staged in LDS and tested
// against every lane's current bound, and candidates that pass are inserted
// lane by lane.  The walk is wave-uniform, so lanes never diverge on the
// tree, only on heap insertions.
//
// Density.  After the walk the heap is sorted in registers by a bitonic
// network; the spline weights are summed pairwise (a fixed tree over 64
// slots, zero-padded) and the result divided by h^3, all in FP64 with
// correctly rounded division and square root and no contraction.
#include "hop_internal.h"

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

__global__ void k_gather_recs(const uint32_t *__restrict__ pos, const uint32_t *__restrict__ perm,
                              const int32_t *__restrict__ tk, int64_t n, uint32_t glim,
                              SortedRec *__restrict__ recs)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    int32_t j = (int32_t)perm[t];
    SortedRec r;
    r.x = (double)min(pos[3 * (int64_t)j], glim - 1);
    r.y = (double)min(pos[3 * (int64_t)j + 1], glim - 1);
    r.z = (double)min(pos[3 * (int64_t)j + 2], glim - 1);
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

constexpr int kHeapMax = 63;  // n_dens - 1 <= 63

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
    int vec_store;       // nbr rows 16-byte aligned with k_store % 4 == 0
    int32_t *nbr;
    double *dens;
    const int32_t *tk2j;
    uint32_t *dflags;
    unsigned long long *counters;  // [0] nodes tested, [1] leaves scanned (NULL = off)
};

__device__ __forceinline__ uint64_t make_key(double d2, uint32_t tk, const KnnArgs &a)
{
    double c = d2 < a.maxd2 ? d2 : a.maxd2;
    return ((uint64_t)c << a.shift) | (uint64_t)tk;
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

// Heap of one lane: slot s at heap[s * 64 + lane].
__device__ __forceinline__ void heap_sift(uint64_t *heap, int lane, int hs, int i, uint64_t x)
{
    for (;;) {
        int l = 2 * i + 1;
        if (l >= hs) break;
        uint64_t kc = heap[l * 64 + lane];
        int c = l;
        if (l + 1 < hs) {
            uint64_t kr = heap[(l + 1) * 64 + lane];
            if (kr > kc) {
                kc = kr;
                c = l + 1;
            }
        }
        if (kc <= x) break;
        heap[i * 64 + lane] = kc;
        i = c;
    }
    heap[i * 64 + lane] = x;
}

// Exact squared distance of this lane's query to a staged particle.
template <bool PERIODIC>
__device__ __forceinline__ double pair_d2(double qx, double qy, double qz, const SortedRec &p,
                                          bool fast, double gsize)
{
    double dx = qx - p.x, dy = qy - p.y, dz = qz - p.z;
    if (PERIODIC && !fast) {
        dx = fabs(dx);
        dy = fabs(dy);
        dz = fabs(dz);
        dx = fmin(dx, gsize - dx);
        dy = fmin(dy, gsize - dy);
        dz = fmin(dz, gsize - dz);
    }
    return __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
}

template <bool PERIODIC, bool IDS>
__global__ __launch_bounds__(64) void k_knn_density(KnnArgs a)
{
    __shared__ uint64_t heap[kHeapMax * 64];
    __shared__ SortedRec stage[64];
    __shared__ uint32_t stk[64];

    const int lane = threadIdx.x;
    // XCD-aware bucket order: consecutive blocks land on different XCDs, so
    // give each XCD a contiguous run of buckets (neighbouring buckets share
    // candidate leaves in that XCD's L2).
    const int64_t bid = blockIdx.x;
    const int64_t bucket = (bid & 7) * a.xcd_chunk + (bid >> 3);
    if (bucket >= a.n_buckets) return;
    const int64_t b0 = bucket * HOP_BUCKET;
    const int bcount = (int)min((int64_t)HOP_BUCKET, a.n - b0);
    const bool active = lane < bcount;
    const int hs = a.hs;

    // stage the bucket's own particles
    if (active) stage[lane] = a.recs[b0 + lane];
    __syncthreads();
    const SortedRec me = stage[active ? lane : 0];
    const double qx = me.x, qy = me.y, qz = me.z;
    const uint32_t ux = (uint32_t)qx, uy = (uint32_t)qy, uz = (uint32_t)qz;

    // initial heap: the bucket's other particles (first hs of them heapified,
    // the rest offered)
    {
        int filled = 0;
        for (int k = 0; k < HOP_BUCKET; k++) {
            if (k == lane) continue;  // divergent only for this lane's own slot
            uint64_t key = ~0ull;
            if (k < bcount) {
                double d2 = pair_d2<PERIODIC>(qx, qy, qz, stage[k], false, a.gsize);
                key = make_key(d2, (uint32_t)stage[k].tk, a);
            }
            if (filled < hs) {
                heap[filled * 64 + lane] = key;
                filled++;
                if (filled == hs) {
                    for (int i = hs / 2 - 1; i >= 0; i--) heap_sift(heap, lane, hs, i, heap[i * 64 + lane]);
                }
            } else if (key < heap[lane]) {
                heap_sift(heap, lane, hs, 0, key);
            }
        }
        if (filled < hs) {  // only when the bucket is smaller than hs + 1
            for (int s = filled; s < hs; s++) heap[s * 64 + lane] = ~0ull;
            for (int i = hs / 2 - 1; i >= 0; i--) heap_sift(heap, lane, hs, i, heap[i * 64 + lane]);
        }
    }
    uint64_t tau_key = heap[lane];
    double tau = active ? (double)(tau_key >> a.shift) : -1.0;

    // bucket box (level-2 node = the bucket's 4 leaves) for near-first order
    // and for the periodic fast path
    const NodeBox bb = a.boxes[a.lv.off[2] + bucket];
    const int64_t bcx = ((int64_t)bb.lo[0] + bb.hi[0]) >> 1;
    const int64_t bcy = ((int64_t)bb.lo[1] + bb.hi[1]) >> 1;
    const int64_t bcz = ((int64_t)bb.lo[2] + bb.hi[2]) >> 1;
    const int64_t G = (int64_t)a.gmask + 1;

    unsigned long long n_nodes = 0, n_leaves = 0;
    int sp = 0;
    stk[sp++] = ((uint32_t)a.lv.top << 27) | 0u;
    while (sp > 0) {
        const uint32_t code = __builtin_amdgcn_readfirstlane(stk[--sp]);
        const int h = (int)(code >> 27);
        const int64_t j = code & ((1u << 27) - 1);
        const NodeBox bx = a.boxes[a.lv.off[h] + j];
        n_nodes++;
        double gx = axis_gap<PERIODIC>(ux, bx.lo[0], bx.hi[0], a.gmask);
        double gy = axis_gap<PERIODIC>(uy, bx.lo[1], bx.hi[1], a.gmask);
        double gz = axis_gap<PERIODIC>(uz, bx.lo[2], bx.hi[2], a.gmask);
        double md2 = __builtin_fma(gx, gx, __builtin_fma(gy, gy, gz * gz));
        if (!__any(md2 <= tau)) continue;
        if (h > 0) {
            const int64_t c0 = 2 * j, c1 = 2 * j + 1;
            if (c1 >= a.lv.cnt[h - 1]) {
                stk[sp++] = ((uint32_t)(h - 1) << 27) | (uint32_t)c0;
                continue;
            }
            // near-first: Chebyshev distance from the bucket centre to each
            // child's centre (minimum image when periodic)
            const NodeBox b0x = a.boxes[a.lv.off[h - 1] + c0];
            const NodeBox b1x = a.boxes[a.lv.off[h - 1] + c1];
            int64_t d0 = 0, d1 = 0;
            const int64_t bc[3] = {bcx, bcy, bcz};
#pragma unroll
            for (int k = 0; k < 3; k++) {
                int64_t e0 = ((((int64_t)b0x.lo[k] + b0x.hi[k]) >> 1) - bc[k]);
                int64_t e1 = ((((int64_t)b1x.lo[k] + b1x.hi[k]) >> 1) - bc[k]);
                e0 = e0 < 0 ? -e0 : e0;
                e1 = e1 < 0 ? -e1 : e1;
                if (PERIODIC) {
                    e0 = min(e0, G - e0);
                    e1 = min(e1, G - e1);
                }
                d0 = max(d0, e0);
                d1 = max(d1, e1);
            }
            const uint32_t k0 = ((uint32_t)(h - 1) << 27) | (uint32_t)c0;
            const uint32_t k1 = ((uint32_t)(h - 1) << 27) | (uint32_t)c1;
            if (d0 <= d1) {
                stk[sp++] = k1;
                stk[sp++] = k0;
            } else {
                stk[sp++] = k0;
                stk[sp++] = k1;
            }
            continue;
        }
        // a leaf
        if ((j >> 2) == bucket) continue;  // the bucket's own leaves are in the heap
        n_leaves++;
        const int cnt = (int)bx.count;
        const int64_t p0 = j * HOP_LEAF;
        __syncthreads();
        if (lane < cnt * 4) {
            const uint64_t *src = reinterpret_cast<const uint64_t *>(a.recs + p0);
            reinterpret_cast<uint64_t *>(stage)[lane] = src[lane];
        }
        __syncthreads();
        // periodic fast path: one image shift per axis for the whole leaf when
        // every query-particle separation stays within half the box
        bool fast = true;
        double sx = 0, sy = 0, sz = 0;
        if (PERIODIC) {
            const int64_t half = G >> 1;
            double sh[3];
#pragma unroll
            for (int k = 0; k < 3; k++) {
                int64_t lc = ((int64_t)bx.lo[k] + bx.hi[k]) >> 1;
                int64_t s = 0;
                if (lc - ((k == 0) ? bcx : (k == 1) ? bcy : bcz) > half) s = G;
                if (lc - ((k == 0) ? bcx : (k == 1) ? bcy : bcz) < -half) s = -G;
                // particle p is used as p - s; the largest separation
                int64_t m1 = (int64_t)bb.hi[k] - ((int64_t)bx.lo[k] - s);
                int64_t m2 = ((int64_t)bx.hi[k] - s) - (int64_t)bb.lo[k];
                if (max(m1, m2) > half) fast = false;
                sh[k] = (double)s;
            }
            sx = sh[0];
            sy = sh[1];
            sz = sh[2];
        }
        const double fx = qx + sx, fy = qy + sy, fz = qz + sz;
        uint32_t pass = 0;
        for (int k = 0; k < cnt; k++) {
            const SortedRec p = stage[k];
            double d2 = fast ? pair_d2<false>(fx, fy, fz, p, true, a.gsize)
                             : pair_d2<PERIODIC>(qx, qy, qz, p, false, a.gsize);
            pass |= (d2 <= tau ? 1u : 0u) << k;
        }
        // insert the passing particles, lane by lane
        while (__any(pass != 0)) {
            if (pass != 0) {
                const int k = __builtin_ctz(pass);
                pass &= pass - 1;
                const SortedRec p = stage[k];
                double d2 = fast ? pair_d2<false>(fx, fy, fz, p, true, a.gsize)
                                 : pair_d2<PERIODIC>(qx, qy, qz, p, false, a.gsize);
                uint64_t key = make_key(d2, (uint32_t)p.tk, a);
                if (key < tau_key) {
                    heap_sift(heap, lane, hs, 0, key);
                    tau_key = heap[lane];
                    tau = (double)(tau_key >> a.shift);
                }
            }
        }
    }

    if (a.counters && lane == 0) {
        atomicAdd(&a.counters[0], n_nodes);
        atomicAdd(&a.counters[1], n_leaves);
    }
    if (!active) return;

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
    double part[7];
#pragma unroll
    for (int t = 0; t < 64; t++) {
        double w;
        if (t == 0) {
            w = m4_shape(0.0);
        } else if (t < a.n_dens) {
            const uint64_t d2 = v[t - 1] >> a.shift;
            w = m4_shape((double)(4 * d2) / Rd);
        } else {
            w = 0.0;
        }
        // pairwise (binary-counter) accumulation: T(a,b) = T(a,m) + T(m,b)
        double s = w;
        int lvl = 0;
#pragma unroll
        for (int b = 0; b < 6; b++) {
            if (((t >> b) & 1) == 0) break;
            s = part[b] + s;
            lvl = b + 1;
        }
        part[lvl] = s;
    }
    const double S = part[6];
    const double h2 = Rd * 0.25;
    const double hh = __builtin_sqrt(h2);
    const double h3 = h2 * hh;
    const double delta = (S * a.norm) / h3;

    const int32_t jq = me.j;
    a.dens[jq] = delta;
    if (a.nbr) {
        int32_t *row = a.nbr + (int64_t)jq * a.k_store;
        auto col = [&](int t) -> int32_t {
            if (t == 0) return jq;
            const uint32_t tkv = (uint32_t)(v[t - 1] & a.tk_mask);
            // an unfilled slot (flagged above) must not index the table
            if (IDS) return tkv < (uint64_t)a.n ? a.tk2j[tkv] : -1;
            return (int32_t)tkv;
        };
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

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

int hop_density_impl(hop_ctx *ctx, int64_t n, const uint32_t *pos, const int64_t *id,
                     const hop_params *p, double *density, int32_t *nbr, hipStream_t s)
{
    const uint32_t glim = 1u << p->grid_bits;
    const bool periodic = (p->flags & HOP_PERIODIC) != 0;
    uint32_t *dflags = (uint32_t *)ctx->flags.ptr;

    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    if (ctx->profiling) {
        for (auto &e : ev) HOPCHK(ctx, hipEventCreate(&e));
        HOPCHK(ctx, hipEventRecord(ev[0], s));
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
    HOPTRY(hop_radix_sort(ctx, keys, perm, (uint64_t *)ctx->keys_b.ptr, (uint32_t *)ctx->vals_b.ptr,
                          n, 3 * (int)p->grid_bits, s));
    ctx->perm_n = n;

    // 2. sorted copy and tree
    HOPTRY(hop_reserve(ctx, ctx->recs, (size_t)n * sizeof(SortedRec)));
    SortedRec *recs = (SortedRec *)ctx->recs.ptr;
    k_gather_recs<<<hop_grid(n, 256), 256, 0, s>>>(pos, perm, tk, n, glim, recs);
    HOPCHK(ctx, hipGetLastError());

    TreeLevels lv{};
    int64_t n_leaves = hop_div_up(n, HOP_LEAF);
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
    NodeBox *boxes = (NodeBox *)ctx->boxes.ptr;
    k_leaf_boxes<<<hop_grid(n_leaves, 256), 256, 0, s>>>(recs, n, n_leaves, boxes);
    HOPCHK(ctx, hipGetLastError());
    for (int h = 1; h <= lv.top; h++) {
        k_level_boxes<<<hop_grid(lv.cnt[h], 256), 256, 0, s>>>(boxes, lv.off[h - 1], lv.cnt[h - 1],
                                                               lv.off[h], lv.cnt[h]);
        HOPCHK(ctx, hipGetLastError());
    }
    if (ctx->profiling) HOPCHK(ctx, hipEventRecord(ev[1], s));

    // 3. kNN + density
    KnnArgs a{};
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
    const double md = p->mean_density > 0 ? p->mean_density
                                          : (double)n / (double)(1ull << (3 * p->grid_bits));
    a.norm = 1.0 / (3.141592653589793 * md);
    a.gsize = (double)glim;
    a.gmask = glim - 1;
    a.vec_store = nbr && (p->k_store % 4 == 0) && (((uintptr_t)nbr & 15) == 0);
    a.nbr = nbr;
    a.dens = density;
    a.tk2j = tk2j;
    a.dflags = dflags;
    a.counters = nullptr;
    unsigned long long *counters = (unsigned long long *)((char *)ctx->flags.ptr + 256);
    if (ctx->profiling & 2) {
        a.counters = counters;
        HOPCHK(ctx, hipMemsetAsync(a.counters, 0, 16, s));
    }
    const int64_t grid = a.xcd_chunk * 8;
    if (grid >= ((int64_t)1 << 31)) return hop_fail(ctx, HOP_ERR_ARG, "too many particles");
    if (periodic) {
        if (id) k_knn_density<true, true><<<(int)grid, 64, 0, s>>>(a);
        else k_knn_density<true, false><<<(int)grid, 64, 0, s>>>(a);
    } else {
        if (id) k_knn_density<false, true><<<(int)grid, 64, 0, s>>>(a);
        else k_knn_density<false, false><<<(int)grid, 64, 0, s>>>(a);
    }
    HOPCHK(ctx, hipGetLastError());

    if (ctx->profiling) {
        HOPCHK(ctx, hipEventRecord(ev[2], s));
        HOPCHK(ctx, hipEventSynchronize(ev[2]));
        float t0 = 0, t1 = 0;
        HOPCHK(ctx, hipEventElapsedTime(&t0, ev[0], ev[1]));
        HOPCHK(ctx, hipEventElapsedTime(&t1, ev[1], ev[2]));
        unsigned long long c[2] = {0, 0};
        if (a.counters) HOPCHK(ctx, hipMemcpy(c, a.counters, 16, hipMemcpyDeviceToHost));
        ctx->stats.ms_sort = t0;
        ctx->stats.ms_knn = t1;
        ctx->stats.n = n;
        ctx->stats.nodes_visited = (int64_t)c[0];
        ctx->stats.leaves_scanned = (int64_t)c[1];
        for (auto &e : ev) hipEventDestroy(e);
    }
    return HOP_OK;
}
