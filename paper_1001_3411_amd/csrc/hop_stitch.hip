// hop_stitch.hip -- whole-box chains, boundaries and halos from padded
// subvolumes (the paper's section 3.1, the steps after each task's own
// densities and links, and its premerge step).
//
// Input: the rows of a batched run (hop_run_batch) over padded subvolumes
// cut from one box -- every row's box index, padding flag, density, list
// and link, all local to its subvolume.  Padded rows link to themselves
// (the section 3.1 rule), so a chain of a subvolume may end on a padded
// particle; the paper reconnects such a chain through the particle's owner
// (the subvolume where it is local).  Here each padded row gets a virtual
// link to its owner's row, and pointer jumping over rows, links and virtual
// links together reaches each chain's true peak: a local, self-linked row.
// Chains are the alive true peaks, numbered by box index (the whole-box
// order).  Every row, padded or not, then takes its owner's chain (the
// annulus exchange of the paper), and the boundary table is built from all
// rows at once -- one table for every subvolume's pairs, a padded-padded
// pair skipped -- before the merge and the labels, which count local rows
// only.  The optional premerge joins, inside each subvolume, the chains of
// that subvolume whose own peaks reach delta_peak and that share a boundary
// at or above delta_saddle, before any reconnection; those joins are kept in
// the final halos.
#include <algorithm>

#include "hop_internal.h"

namespace {

__device__ __forceinline__ int sub_of_row(const int64_t *__restrict__ off, int n_sub, int64_t r)
{
    int lo = 0, hi = n_sub;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= r) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void k_fill32(int32_t *__restrict__ p, int64_t n, int32_t v)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

// owner[g] = the local (unpadded) row of box index g; a second local row of
// the same index sets DERR_OWNER, an index outside [0, n) DERR_INDEX
__global__ void k_owner(int64_t rows, const int64_t *__restrict__ index,
                        const uint8_t *__restrict__ padded, int64_t n, int32_t *__restrict__ owner,
                        uint32_t *__restrict__ dflags)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const int64_t g = index[r];
    if (g < 0 || g >= n) {
        atomicOr(dflags, DERR_INDEX);
        return;
    }
    if (padded && padded[r]) return;
    if (atomicCAS(&owner[g], -1, (int32_t)r) != -1) atomicOr(dflags, DERR_OWNER);
}

__global__ void k_owner_missing(int64_t n, const int32_t *__restrict__ owner,
                                uint32_t *__restrict__ dflags)
{
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n && owner[g] < 0) atomicOr(dflags, DERR_OWNER);
}

// Density of every row: its own (as its subvolume computed it), or its
// owner's (the annulus exchange carrying densities as well as chains).
// tk = box index of the row, the tie key of links and of the group order.
__global__ void k_row_dens(int64_t rows, const int64_t *__restrict__ index, int64_t n,
                           const int32_t *__restrict__ owner, const double *__restrict__ density_b,
                           int own_density, double *__restrict__ dens, int32_t *__restrict__ tk)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const int64_t g = index[r];
    const bool ok = g >= 0 && g < n;
    tk[r] = ok ? (int32_t)g : 0;
    dens[r] = (own_density && ok) ? density_b[owner[g]] : density_b[r];
}

// Links over rows: a local row to its link (a row of its subvolume), a
// padded row to its owner's row (the virtual link).  lroot gets the links
// without virtual links (padded rows stay self-linked), for the premerge.
// The link of a local row is hop_b's, or (hop_b NULL) formed again from
// its first n_hop list entries with the row densities dens: the densest,
// equal densities to the smaller box index (as in the whole box).
__global__ void k_row_links(int64_t rows, const int64_t *__restrict__ off, int n_sub,
                            const int64_t *__restrict__ index, const uint8_t *__restrict__ padded,
                            const int32_t *__restrict__ hop_b, const int32_t *__restrict__ nbr_b,
                            int k_store, int n_hop, const double *__restrict__ dens,
                            const int32_t *__restrict__ tk, int64_t n,
                            const int32_t *__restrict__ owner, int32_t *__restrict__ vroot,
                            int32_t *__restrict__ lroot, uint32_t *__restrict__ dflags)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const int64_t g = index[r];
    const bool pad = padded && padded[r];
    int32_t own = (int32_t)r;
    if (g >= 0 && g < n && owner[g] >= 0) own = owner[g];
    if (pad) {
        vroot[r] = own;
        lroot[r] = (int32_t)r;
        return;
    }
    const int sv = sub_of_row(off, n_sub, r);
    const int64_t base = off[sv], cnt = off[sv + 1] - base;
    int32_t to = (int32_t)r;
    if (hop_b) {
        const int32_t h = hop_b[r];
        if (h >= 0 && h < cnt) to = (int32_t)(base + h);
        else atomicOr(dflags, DERR_INDEX);
    } else {
        double bd = dens[r];
        int32_t bt = tk[r];
        for (int t = 0; t < n_hop; t++) {
            const int32_t j = nbr_b[r * k_store + t];
            if (j < 0 || j >= cnt) {
                atomicOr(dflags, DERR_INDEX);
                continue;
            }
            const int32_t J = (int32_t)(base + j);
            const double dj = dens[J];
            const int32_t tj = tk[J];
            if (dj > bd || (dj == bd && tj < bt)) {
                to = J;
                bd = dj;
                bt = tj;
            }
        }
    }
    vroot[r] = to;
    lroot[r] = to;
}

// a true peak must be a local row (padded rows always link on)
__global__ void k_true_roots(int64_t rows, const int32_t *__restrict__ vroot,
                             const int64_t *__restrict__ index, const double *__restrict__ dens,
                             double delta_outer, int64_t n, uint32_t *__restrict__ flag)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    if (vroot[r] != (int32_t)r || !(dens[r] >= delta_outer)) return;
    const int64_t g = index[r];
    if (g >= 0 && g < n) flag[g] = 1u;
}

// chain of every row from its owner (the annulus exchange), box outputs of
// the local rows
__global__ void k_row_chains(int64_t rows, const int64_t *__restrict__ index,
                             const uint8_t *__restrict__ padded, const double *__restrict__ dens,
                             const int32_t *__restrict__ lnk, int64_t n,
                             const int32_t *__restrict__ owner,
                             const int32_t *__restrict__ vroot, const uint32_t *__restrict__ num,
                             double delta_outer, int32_t *__restrict__ label,
                             double *__restrict__ density, int32_t *__restrict__ hop,
                             int32_t *__restrict__ root, int32_t *__restrict__ chain_of)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const int64_t g = index[r];
    if (g < 0 || g >= n) {
        label[r] = -1;
        return;
    }
    const int32_t u = owner[g];
    int32_t c = -1;
    int64_t groot = g;
    if (u >= 0) {
        groot = index[vroot[u]];
        if (dens[u] >= delta_outer && groot >= 0 && groot < n) c = (int32_t)num[groot];
    }
    label[r] = c;
    if (padded && padded[r]) return;
    density[g] = dens[r];
    if (hop) hop[g] = (int32_t)index[lnk[r]];
    root[g] = (int32_t)groot;
    chain_of[g] = c;
}

// batch-wide copy of the first n_merge list columns
__global__ void k_row_lists(int64_t rows, const int64_t *__restrict__ off, int n_sub,
                            const int32_t *__restrict__ nbr_b, int k_store, int n_merge,
                            int32_t *__restrict__ nbrm, uint32_t *__restrict__ dflags)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const int sv = sub_of_row(off, n_sub, r);
    const int64_t base = off[sv], cnt = off[sv + 1] - base;
    for (int t = 0; t < n_merge; t++) {
        const int32_t j = nbr_b[r * k_store + t];
        int32_t J = (int32_t)r;
        if (j >= 0 && j < cnt) J = (int32_t)(base + j);
        else atomicOr(dflags, DERR_INDEX);
        nbrm[r * n_merge + t] = J;
    }
}

// Premerge inside each subvolume (before reconnection): the subvolume's own
// chains (roots lroot, peaks their own densities); a pair of rows within
// n_merge - 1 ranks, not both padded, in two such chains whose peaks reach
// delta_peak, with 0.5 (d_i + d_j) >= delta_saddle, joins the two chains --
// recorded as the pair of global chains they belong to.
__global__ void k_premerge(int64_t rows, const int32_t *__restrict__ nbrm, int n_merge,
                           const double *__restrict__ dens, const uint8_t *__restrict__ padded,
                           const int32_t *__restrict__ lroot, const int32_t *__restrict__ label,
                           double delta_outer, double delta_saddle, double delta_peak,
                           int32_t *__restrict__ pre_lo, int32_t *__restrict__ pre_hi,
                           uint32_t *__restrict__ count, int64_t cap)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    if (!(dens[i] >= delta_outer)) return;
    const int32_t ri = lroot[i];
    if (!(dens[ri] >= delta_peak)) return;
    const bool pi = padded && padded[i];
    for (int t = 1; t < n_merge; t++) {
        const int32_t j = nbrm[i * n_merge + t];
        if (!(dens[j] >= delta_outer)) continue;
        if (pi && padded[j]) continue;
        const int32_t rj = lroot[j];
        if (rj == ri || !(dens[rj] >= delta_peak)) continue;
        if (!((dens[i] + dens[j]) * 0.5 >= delta_saddle)) continue;
        const int32_t a = label[ri], b = label[rj];
        if (a < 0 || b < 0 || a == b) continue;
        const uint32_t at = atomicAdd(count, 1u);
        if (at < cap) {
            pre_lo[at] = min(a, b);
            pre_hi[at] = max(a, b);
        }
    }
}

// group of every box particle from its local row
__global__ void k_box_groups(int64_t rows, const int64_t *__restrict__ index,
                             const uint8_t *__restrict__ padded, int64_t n,
                             const int32_t *__restrict__ group_r, int32_t *__restrict__ group)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    if (padded && padded[r]) return;
    const int64_t g = index[r];
    if (g >= 0 && g < n) group[g] = group_r[r];
}

struct Carve {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(int64_t count)
    {
        off = (off + 255) & ~(size_t)255;
        T *p = (T *)(base + off);
        off += (size_t)count * sizeof(T);
        return p;
    }
};

}  // namespace

extern "C" int hop_stitch(hop_ctx *ctx, int32_t n_sub, const int64_t *offsets, const int64_t *index,
                          const uint8_t *padded, const double *density_b, const int32_t *nbr_b,
                          const int32_t *hop_b, const hop_params *p, int32_t mode, int64_t n,
                          double *density, int32_t *hop, int32_t *root, int32_t *chain_of,
                          int32_t *group, int32_t *n_chains, int32_t *n_groups,
                          hop_group_info *groups, void *stream)
{
    if (!ctx) return HOP_ERR_ARG;
    ctx->err.clear();
    if (n_sub < 1 || n_sub > 65536 || !offsets || offsets[0] != 0)
        return hop_fail(ctx, HOP_ERR_ARG, "need 1 <= n_sub <= 65536 and offsets from 0");
    for (int k = 0; k < n_sub; k++)
        if (offsets[k + 1] < offsets[k]) return hop_fail(ctx, HOP_ERR_ARG, "offsets must not decrease");
    const int64_t rows = offsets[n_sub];
    HOPTRY(hop_check_params(ctx, n, p));
    if (rows < n || rows >= ((int64_t)1 << 31) - 64)
        return hop_fail(ctx, HOP_ERR_ARG, "need n <= rows < 2^31");
    if (!(p->flags & HOP_PADDED_RULES) || !padded)
        return hop_fail(ctx, HOP_ERR_ARG, "stitching needs the padded rules and the padding flags");
    if (!index || !density_b || !nbr_b || !density || !root || !chain_of || !group || !n_chains ||
        !n_groups)
        return hop_fail(ctx, HOP_ERR_ARG, "index, batch outputs and box outputs must be non-NULL");
    if (mode & ~(HOP_STITCH_PREMERGE | HOP_STITCH_TASK_DENSITIES))
        return hop_fail(ctx, HOP_ERR_ARG, "unknown stitch mode bit");
    const bool task_dens = (mode & HOP_STITCH_TASK_DENSITIES) != 0;
    const bool premerge = (mode & HOP_STITCH_PREMERGE) != 0;
    if (task_dens && !hop_b) return hop_fail(ctx, HOP_ERR_ARG, "HOP_STITCH_TASK_DENSITIES needs hop_b");
    HOPTRY(hop_set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    uint32_t *dflags = (uint32_t *)ctx->flags.ptr;
    const int nm = p->n_merge;

    // scratch: offsets, owner rows, links, labels, tie keys, lists, premerge pairs
    const int64_t pre_cap = rows * (int64_t)(nm > 1 ? nm - 1 : 1);
    const size_t need = (size_t)(n_sub + 1) * 8 + (size_t)n * 8 + (size_t)rows * (8 + 4 * 6 + 4 * nm) +
                        (size_t)pre_cap * 8 + 16 * 256;
    HOPTRY(hop_reserve(ctx, ctx->stitch, need));
    Carve cv{(char *)ctx->stitch.ptr};
    int64_t *off = cv.take<int64_t>(n_sub + 1);
    int32_t *owner = cv.take<int32_t>(n);
    uint32_t *flag = cv.take<uint32_t>(n);
    double *dens = cv.take<double>(rows);
    int32_t *lnk = cv.take<int32_t>(rows);
    int32_t *vroot = cv.take<int32_t>(rows);
    int32_t *lroot = cv.take<int32_t>(rows);
    int32_t *label = cv.take<int32_t>(rows);
    int32_t *tk = cv.take<int32_t>(rows);
    int32_t *group_r = cv.take<int32_t>(rows);
    int32_t *nbrm = cv.take<int32_t>(rows * nm);
    int32_t *pre_lo = cv.take<int32_t>(pre_cap);
    int32_t *pre_hi = cv.take<int32_t>(pre_cap);
    HOPCHK(ctx, hipMemcpyAsync(off, offsets, (size_t)(n_sub + 1) * 8, hipMemcpyHostToDevice, s));

    // 1. owners: every box index is the local row of exactly one subvolume
    k_fill32<<<hop_grid(n, 256), 256, 0, s>>>(owner, n, -1);
    k_owner<<<hop_grid(rows, 256), 256, 0, s>>>(rows, index, padded, n, owner, dflags);
    k_owner_missing<<<hop_grid(n, 256), 256, 0, s>>>(n, owner, dflags);
    HOPCHK(ctx, hipGetLastError());
    HOPTRY(hop_check_device(ctx, s, "hop_stitch"));  // also keeps `offsets` until the copy ran

    // 2. row densities; links and virtual links over rows, resolved to the
    //    true peaks
    k_row_dens<<<hop_grid(rows, 256), 256, 0, s>>>(rows, index, n, owner, density_b, task_dens ? 0 : 1,
                                                   dens, tk);
    k_row_links<<<hop_grid(rows, 256), 256, 0, s>>>(rows, off, n_sub, index, padded,
                                                    task_dens ? hop_b : nullptr, nbr_b, p->k_store,
                                                    p->n_hop, dens, tk, n, owner, vroot, lroot,
                                                    dflags);
    HOPCHK(ctx, hipGetLastError());
    HOPCHK(ctx, hipMemcpyAsync(lnk, vroot, (size_t)rows * 4, hipMemcpyDeviceToDevice, s));
    HOPTRY(hop_jump_impl(ctx, rows, vroot, s));
    if (premerge) HOPTRY(hop_jump_impl(ctx, rows, lroot, s));

    // 3. chains: alive true peaks numbered by box index
    HOPCHK(ctx, hipMemsetAsync(flag, 0, (size_t)n * 4, s));
    k_true_roots<<<hop_grid(rows, 256), 256, 0, s>>>(rows, vroot, index, dens, p->delta_outer, n,
                                                     flag);
    HOPCHK(ctx, hipGetLastError());
    uint32_t *total = dflags + 2;
    HOPTRY(hop_scan_u32(ctx, flag, n, total, s));
    HOPCHK(ctx, hipMemcpyAsync(ctx->hflags, total, 4, hipMemcpyDeviceToHost, s));

    // 4. every row's chain from its owner; box outputs of the local rows
    k_row_chains<<<hop_grid(rows, 256), 256, 0, s>>>(rows, index, padded, dens, lnk, n, owner, vroot,
                                                     flag, p->delta_outer, label, density, hop, root,
                                                     chain_of);
    k_row_lists<<<hop_grid(rows, 256), 256, 0, s>>>(rows, off, n_sub, nbr_b, p->k_store, nm, nbrm,
                                                    dflags);
    HOPCHK(ctx, hipGetLastError());
    HOPTRY(hop_check_device(ctx, s, "hop_stitch"));
    const int32_t C = (int32_t)((uint32_t *)ctx->hflags)[0];

    // 5. optional premerge inside each subvolume
    MergeExtra mx;
    mx.tk_is_index = true;
    if (premerge && C > 0) {
        uint32_t *cnt = dflags + 12;
        HOPCHK(ctx, hipMemsetAsync(cnt, 0, 4, s));
        k_premerge<<<hop_grid(rows, 256), 256, 0, s>>>(rows, nbrm, nm, dens, padded, lroot, label,
                                                       p->delta_outer, p->delta_saddle, p->delta_peak,
                                                       pre_lo, pre_hi, cnt, pre_cap);
        HOPCHK(ctx, hipGetLastError());
        HOPCHK(ctx, hipMemcpyAsync(ctx->hflags + 12, cnt, 4, hipMemcpyDeviceToHost, s));
        HOPCHK(ctx, hipStreamSynchronize(s));
        mx.pre_lo = pre_lo;
        mx.pre_hi = pre_hi;
        mx.n_pre = std::min<int64_t>((int64_t)((uint32_t *)(ctx->hflags + 12))[0], pre_cap);
    }
    ctx->stats.premerged = mx.n_pre;

    // 6. one boundary table over every row's pairs, the merge and the labels
    hop_params q = *p;
    q.k_store = nm;
    int32_t ng = 0;
    HOPTRY(hop_merge_impl(ctx, rows, nbrm, dens, vroot, label, C, tk, padded, &q, group_r, &ng,
                          groups, mx, s));
    k_box_groups<<<hop_grid(rows, 256), 256, 0, s>>>(rows, index, padded, n, group_r, group);
    HOPCHK(ctx, hipGetLastError());
    HOPTRY(hop_check_device(ctx, s, "hop_stitch"));
    *n_chains = C;
    *n_groups = ng;
    return HOP_OK;
}
