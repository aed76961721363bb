// hop_batch.hip -- the whole path for a batch of independent subvolumes
// (the per-task shape of the paper's section 3.1) in one call.
//
// The subvolumes are concatenated, so every per-particle stage runs once
// over the batch: the kNN is one persistent launch (hop_knn.hip), and the
// links, chains, boundaries and merge run on batch-wide indices.  None of
// them crosses a subvolume: neighbours come from the own subvolume only, so
// links, chains and boundaries stay inside it, and the merge's forest never
// joins two subvolumes (no boundary connects them; proto-halos of different
// subvolumes meeting at the virtual root changes no decision, because a
// boundary is skipped exactly when both its ends already reach a
// proto-halo).  Chains are numbered by root index, so each subvolume owns a
// contiguous block of chain numbers; halos are sorted by subvolume first,
// so each owns a contiguous block of group numbers.  A last pass turns every
// index and number into the subvolume's own.
#include <cstring>
#include <vector>

#include "hop_internal.h"

namespace {

__device__ __forceinline__ int sub_of(const int64_t *__restrict__ off, int n_sub, int64_t i)
{
    int lo = 0, hi = n_sub;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

// chain_base[s] = chains whose root lies before subvolume s (the scan of
// the root flags at the subvolume's first particle)
__global__ void k_chain_base(const uint32_t *__restrict__ scan, const int64_t *__restrict__ off,
                             int n_sub, int32_t total, int32_t *__restrict__ cbase)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t > n_sub) return;
    cbase[t] = t < n_sub ? (int32_t)scan[off[t]] : total;
}

// batch-wide indices and numbers -> the subvolume's own
__global__ void k_localise(int64_t n, const int64_t *__restrict__ off, int n_sub,
                           const int32_t *__restrict__ cbase, const int32_t *__restrict__ gbase,
                           int32_t *__restrict__ nbr, int k_store, int vec, int32_t *__restrict__ hop,
                           int32_t *__restrict__ root, int32_t *__restrict__ chain_of,
                           int32_t *__restrict__ group)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int sv = sub_of(off, n_sub, i);
    const int32_t base = (int32_t)off[sv];
    int32_t *row = nbr + i * k_store;
    if (vec) {
        for (int t = 0; t < k_store; t += 4) {
            int4 q = *reinterpret_cast<int4 *>(row + t);
            q.x -= base;
            q.y -= base;
            q.z -= base;
            q.w -= base;
            *reinterpret_cast<int4 *>(row + t) = q;
        }
    } else {
        for (int t = 0; t < k_store; t++) row[t] -= base;
    }
    hop[i] -= base;
    root[i] -= base;
    const int32_t c = chain_of[i];
    if (c >= 0) chain_of[i] = c - cbase[sv];
    const int32_t g = group[i];
    if (g >= 0) group[i] = g - gbase[sv];
}

__global__ void k_localise_groups(int64_t G, const int64_t *__restrict__ off,
                                  const int32_t *__restrict__ gbase, int n_sub,
                                  hop_group_info *__restrict__ groups)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= G) return;
    int lo = 0, hi = n_sub;  // largest s with gbase[s] <= t
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (gbase[mid] <= t) lo = mid;
        else hi = mid;
    }
    groups[t].peak -= (int32_t)off[lo];
}

}  // namespace

extern "C" int hop_run_batch(hop_ctx *ctx, int32_t n_sub, const int64_t *offsets,
                             const uint32_t *pos, const uint8_t *padded,
                             const double *mean_density, const hop_params *p, double *density,
                             int32_t *nbr, int32_t *hop, int32_t *root, int32_t *chain_of,
                             int32_t *group, int32_t *n_chains, int32_t *n_groups,
                             hop_group_info *groups, int64_t *group_off, void *stream)
{
    if (!ctx) return HOP_ERR_ARG;
    ctx->err.clear();
    if (n_sub < 1 || n_sub > 65536 || !offsets)
        return hop_fail(ctx, HOP_ERR_ARG, "need 1 <= n_sub <= 65536 and offsets");
    if (!pos || !density || !nbr || !hop || !root || !chain_of || !group || !n_chains || !n_groups)
        return hop_fail(ctx, HOP_ERR_ARG, "pos and every per-particle output must be non-NULL");
    if (offsets[0] != 0) return hop_fail(ctx, HOP_ERR_ARG, "offsets[0] must be 0");
    if (!p) return hop_fail(ctx, HOP_ERR_ARG, "params is NULL");
    if (p->flags & HOP_LEARNED_RADIUS)
        return hop_fail(ctx, HOP_ERR_ARG, "HOP_LEARNED_RADIUS is not available for batches");
    for (int k = 0; k < n_sub; k++) {
        if (offsets[k + 1] - offsets[k] < p->n_dens)
            return hop_fail(ctx, HOP_ERR_ARG, "subvolume " + std::to_string(k) + " has fewer than n_dens particles");
        if (mean_density && !(mean_density[k] == mean_density[k] && mean_density[k] < 1e300))
            return hop_fail(ctx, HOP_ERR_ARG, "mean_density must be finite");
    }
    const int64_t n = offsets[n_sub];
    HOPTRY(hop_check_params(ctx, n, p));
    HOPTRY(hop_set_device(ctx));
    hipStream_t s = (hipStream_t)stream;

    // 1. kNN + density, one persistent launch (with the Morton-order copy of
    //    list heads and densities that the links read, when n_hop <= 16)
    int64_t *sub_off = nullptr;
    int32_t *nbr16s = nullptr;
    double *dens_s = nullptr;
    if (p->n_hop <= 16) {
        const size_t rows = (size_t)hop_div_up(n, HOP_BUCKET) * HOP_BUCKET;
        HOPTRY(hop_reserve(ctx, ctx->srt_nbr, rows * 16 * 4));
        HOPTRY(hop_reserve(ctx, ctx->srt_dens, rows * 8));
        nbr16s = (int32_t *)ctx->srt_nbr.ptr;
        dens_s = (double *)ctx->srt_dens.ptr;
    }
    HOPTRY(hop_density_batch_impl(ctx, n_sub, offsets, pos, mean_density, p, density, nbr, nbr16s,
                                  dens_s, &sub_off, s));

    // 2.-3. links and chains on batch-wide indices
    if (nbr16s) HOPTRY(hop_link_sorted_impl(ctx, n, nbr16s, dens_s, density, nullptr, padded, p, hop, s));
    else HOPTRY(hop_link_impl(ctx, n, nbr, density, nullptr, padded, p, hop, s));
    int32_t nc = 0;
    HOPTRY(hop_groups_impl(ctx, n, hop, density, nullptr, p, root, chain_of, &nc, s));
    HOPTRY(hop_reserve(ctx, ctx->batch_aux, (size_t)(3 * n_sub + 3) * 4));
    int32_t *cbase = (int32_t *)ctx->batch_aux.ptr;
    int32_t *gfirst = cbase + (n_sub + 1);
    int32_t *gbase = gfirst + (n_sub + 1);
    k_chain_base<<<hop_grid(n_sub + 1, 256), 256, 0, s>>>((const uint32_t *)ctx->work_a.ptr, sub_off,
                                                          n_sub, nc, cbase);
    HOPCHK(ctx, hipGetLastError());

    // 4. boundaries, merge and labels, halos ordered by subvolume first
    std::vector<int32_t> gf(n_sub + 1, 0);
    HOPCHK(ctx, hipMemsetAsync(gfirst, 0xff, (size_t)(n_sub + 1) * 4, s));
    int32_t ng = 0;
    MergeExtra mx;
    mx.chain_base = nc > 0 ? cbase : nullptr;
    mx.n_sub = n_sub;
    mx.group_first = gfirst;
    HOPTRY(hop_merge_impl(ctx, n, nbr, density, root, chain_of, nc, nullptr, padded, p, group, &ng,
                          groups, mx, s));
    std::vector<int32_t> cb(n_sub + 1, 0);
    if (nc > 0) {
        HOPCHK(ctx, hipMemcpyAsync(cb.data(), cbase, (size_t)(n_sub + 1) * 4, hipMemcpyDeviceToHost, s));
        HOPCHK(ctx, hipMemcpyAsync(gf.data(), gfirst, (size_t)(n_sub + 1) * 4, hipMemcpyDeviceToHost, s));
        HOPCHK(ctx, hipStreamSynchronize(s));
    }
    // first group of each subvolume: its own first, or the next one's
    std::vector<int32_t> gb(n_sub + 1);
    gb[n_sub] = ng;
    for (int k = n_sub - 1; k >= 0; k--) gb[k] = (nc > 0 && gf[k] >= 0) ? gf[k] : gb[k + 1];
    for (int k = 0; k < n_sub; k++) {
        n_chains[k] = nc > 0 ? cb[k + 1] - cb[k] : 0;
        n_groups[k] = gb[k + 1] - gb[k];
        if (group_off) group_off[k] = gb[k];
    }
    if (group_off) group_off[n_sub] = ng;

    // 5. every index and number local to its subvolume
    HOPCHK(ctx, hipMemcpyAsync(gbase, gb.data(), (size_t)(n_sub + 1) * 4, hipMemcpyHostToDevice, s));
    if (nc == 0) HOPCHK(ctx, hipMemsetAsync(cbase, 0, (size_t)(n_sub + 1) * 4, s));
    const int vec = (p->k_store % 4 == 0) && (((uintptr_t)nbr & 15) == 0);
    k_localise<<<hop_grid(n, 256), 256, 0, s>>>(n, sub_off, n_sub, cbase, gbase, nbr, p->k_store, vec,
                                                hop, root, chain_of, group);
    HOPCHK(ctx, hipGetLastError());
    if (groups && ng > 0) {
        k_localise_groups<<<hop_grid(ng, 256), 256, 0, s>>>(ng, sub_off, gbase, n_sub, groups);
        HOPCHK(ctx, hipGetLastError());
    }
    HOPTRY(hop_check_device(ctx, s, "hop_run_batch"));  // also keeps gb alive until the copy ran
    return HOP_OK;
}

