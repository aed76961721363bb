// hop_link.hip -- tie keys, densest-neighbour links and chain resolution
// (the paper's section 2, stages 2 and 3, and merge step 1).
//
// Links: one lane per particle reads its first n_hop neighbours and their
// densities; the densest wins, equal densities go to the smaller tie key.
// k_hop takes particles in input order (any neighbour lists); k_hop_sorted
// takes them in Morton order from the copy the kNN kernel writes for the
// fused density + link call, so that a wave's gathers fall in cache.
// Chains: pointer jumping (root <- root[root]) until no root changes; every
// step at least halves the remaining distance to the self-linked particle,
// so a chain of depth D resolves in ceil(log2 D) rounds.  Chains are then
// numbered by an exclusive scan over the tie-key order of their roots.
#include "hop_internal.h"

namespace {

__global__ void k_id_keys(const int64_t *__restrict__ id, int64_t n, uint64_t *__restrict__ keys,
                          uint32_t *__restrict__ vals)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = (uint64_t)id[i] ^ 0x8000000000000000ull;  // signed order as unsigned
    vals[i] = (uint32_t)i;
}

__global__ void k_id_ranks(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals,
                           int64_t n, int32_t *__restrict__ tk, int32_t *__restrict__ tk2j,
                           uint32_t *__restrict__ dflags)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    uint32_t j = vals[t];
    tk[j] = (int32_t)t;
    tk2j[t] = (int32_t)j;
    if (t > 0 && keys[t] == keys[t - 1]) atomicOr(dflags, DERR_IDS);
}

__global__ void k_hop(int64_t n, const int32_t *__restrict__ nbr, int k_store, int n_hop,
                      const double *__restrict__ dens, const int32_t *__restrict__ tk,
                      const uint8_t *__restrict__ padded, int padded_rules,
                      int32_t *__restrict__ hop, uint32_t *__restrict__ dflags)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (padded_rules && padded && padded[i]) {
        hop[i] = (int32_t)i;
        return;
    }
    int32_t best = (int32_t)i;
    double bd = dens[i];
    int32_t bt = tk ? tk[i] : (int32_t)i;
    const int32_t *row = nbr + i * k_store;
    bool bad = false;
    for (int s = 0; s < n_hop; s++) {
        int32_t j = row[s];
        if (j < 0 || j >= n) {
            bad = true;
            continue;
        }
        double dj = dens[j];
        int32_t tj = tk ? tk[j] : j;
        if (dj > bd || (dj == bd && tj < bt)) {
            best = j;
            bd = dj;
            bt = tj;
        }
    }
    if (bad) atomicOr(dflags, DERR_INDEX);
    hop[i] = best;
}

// The same links in Morton order: thread t takes the particle at sorted
// position t, its first 16 list entries from the sorted copy (one 64-byte
// row, consecutive threads on consecutive rows; entry 0 is the particle
// itself) and its density from the sorted copy; the neighbours' densities
// are gathered from the input-order array, where the 64 threads of a wave,
// being neighbours in space, mostly gather the same entries.  Same
// comparisons in the same order as k_hop.
__device__ __forceinline__ void hop_sorted_one(int64_t t, int64_t n, const int32_t *__restrict__ nbr16s,
                                               int n_hop, const double *__restrict__ dens_s,
                                               const double *__restrict__ dens,
                                               const int32_t *__restrict__ tk,
                                               const uint8_t *__restrict__ padded, int padded_rules,
                                               int32_t *__restrict__ hop, uint32_t *__restrict__ dflags)
{
    const int4 *row = reinterpret_cast<const int4 *>(nbr16s + t * 16);
    int32_t js[16];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int4 v = row[q];
        js[4 * q] = v.x;
        js[4 * q + 1] = v.y;
        js[4 * q + 2] = v.z;
        js[4 * q + 3] = v.w;
    }
    const int32_t i = js[0];  // every list starts with the particle itself
    if (i < 0 || i >= n) {
        atomicOr(dflags, DERR_INDEX);
        return;
    }
    if (padded_rules && padded && padded[i]) {
        hop[i] = i;
        return;
    }
    int32_t best = i;
    double bd = dens_s[t];
    int32_t bt = tk ? tk[i] : i;
    bool bad = false;
#pragma unroll
    for (int s = 0; s < 16; s++) {
        if (s >= n_hop) break;
        const int32_t j = js[s];
        if (j < 0 || j >= n) {
            bad = true;
            continue;
        }
        const double dj = dens[j];
        const int32_t tj = tk ? tk[j] : j;
        if (dj > bd || (dj == bd && tj < bt)) {
            best = j;
            bd = dj;
            bt = tj;
        }
    }
    if (bad) atomicOr(dflags, DERR_INDEX);
    hop[i] = best;
}

// The sorted positions in blocks of 256, each XCD taking a contiguous run
// of xcd_chunk blocks (consecutive workgroup numbers go to different XCDs),
// so that neighbouring blocks, which gather many of the same densities,
// share one L2.  per_xcd workgroups per XCD walk its run in order, a few
// per compute unit: the densities being gathered then stay within the L2
// (with one workgroup per block, the blocks in flight gathered from more
// lines than the L2 holds; 2 per compute unit measured fastest, 18.7 ->
// 16.3 ms at 134M particles).
__global__ void k_hop_sorted(int64_t n, const int32_t *__restrict__ nbr16s, int n_hop,
                             const double *__restrict__ dens_s, const double *__restrict__ dens,
                             const int32_t *__restrict__ tk, const uint8_t *__restrict__ padded,
                             int padded_rules, int32_t *__restrict__ hop,
                             uint32_t *__restrict__ dflags, int64_t xcd_chunk, int64_t per_xcd)
{
    const int64_t x = blockIdx.x & 7;
    for (int64_t r = blockIdx.x >> 3; r < xcd_chunk; r += per_xcd) {
        const int64_t t = (x * xcd_chunk + r) * blockDim.x + threadIdx.x;
        if (t < n) hop_sorted_one(t, n, nbr16s, n_hop, dens_s, dens, tk, padded, padded_rules, hop, dflags);
    }
}

__global__ void k_root_init(int64_t n, const int32_t *__restrict__ hop, int32_t *__restrict__ root,
                            uint32_t *__restrict__ dflags)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t h = hop[i];
    if (h < 0 || h >= n) {
        atomicOr(dflags, DERR_INDEX);
        h = (int32_t)i;
    }
    root[i] = h;
}

// Up to 4 jumps per launch; *changed is set when a root moved.  A particle
// whose root is found self-linked is marked done, and later launches skip
// it with a one-byte read instead of a random gather (most chains resolve
// in the first launch).
__global__ void k_jump(int64_t n, int32_t *__restrict__ root, uint8_t *__restrict__ done,
                       uint32_t *__restrict__ changed)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (done[i]) return;
    int32_t r = root[i];
    int32_t r0 = r;
    bool fin = false;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        int32_t rr = root[r];
        if (rr == r) {
            fin = true;
            break;
        }
        r = rr;
    }
    if (r != r0) {
        root[i] = r;
        *changed = 1u;
    }
    if (fin) done[i] = 1;
}

// Chain roots, flagged by tie key.  After the jumps every root must be a
// self-linked particle; links that close a cycle (which uphill links never
// do) leave roots that are not, and raise DERR_CYCLE.
__global__ void k_chain_flags(int64_t n, const int32_t *__restrict__ hop,
                              const int32_t *__restrict__ root, const double *__restrict__ dens,
                              const int32_t *__restrict__ tk, double delta_outer,
                              uint32_t *__restrict__ flag, uint32_t *__restrict__ dflags)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t r = root[i];
    if (hop[r] != r) atomicOr(dflags, DERR_CYCLE);
    uint32_t f = (r == (int32_t)i && hop[i] == (int32_t)i && dens[i] >= delta_outer) ? 1u : 0u;
    flag[tk ? tk[i] : i] = f;
}

__global__ void k_chain_of(int64_t n, const int32_t *__restrict__ root,
                           const double *__restrict__ dens, const int32_t *__restrict__ tk,
                           double delta_outer, const uint32_t *__restrict__ cidx,
                           int32_t *__restrict__ chain_of)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t r = root[i];
    chain_of[i] = dens[i] >= delta_outer ? (int32_t)cidx[tk ? tk[r] : r] : -1;
}

}  // namespace

int hop_build_tiekeys(hop_ctx *ctx, int64_t n, const int64_t *id, hipStream_t s)
{
    HOPTRY(hop_reserve(ctx, ctx->keys_a, (size_t)n * 8));
    HOPTRY(hop_reserve(ctx, ctx->keys_b, (size_t)n * 8));
    HOPTRY(hop_reserve(ctx, ctx->vals_a, (size_t)n * 4));
    HOPTRY(hop_reserve(ctx, ctx->vals_b, (size_t)n * 4));
    HOPTRY(hop_reserve(ctx, ctx->tk, (size_t)n * 4));
    HOPTRY(hop_reserve(ctx, ctx->tk2j, (size_t)n * 4));
    uint64_t *keys = (uint64_t *)ctx->keys_a.ptr;
    uint32_t *vals = (uint32_t *)ctx->vals_a.ptr;
    k_id_keys<<<hop_grid(n, 256), 256, 0, s>>>(id, n, keys, vals);
    HOPCHK(ctx, hipGetLastError());
    HOPTRY(hop_radix_sort(ctx, keys, vals, (uint64_t *)ctx->keys_b.ptr, (uint32_t *)ctx->vals_b.ptr,
                          n, 64, s));
    k_id_ranks<<<hop_grid(n, 256), 256, 0, s>>>(keys, vals, n, (int32_t *)ctx->tk.ptr,
                                                (int32_t *)ctx->tk2j.ptr, (uint32_t *)ctx->flags.ptr);
    HOPCHK(ctx, hipGetLastError());
    return HOP_OK;
}

int hop_link_impl(hop_ctx *ctx, int64_t n, const int32_t *nbr, const double *density,
                  const int32_t *tk, const uint8_t *padded, const hop_params *p, int32_t *hop,
                  hipStream_t s)
{
    k_hop<<<hop_grid(n, 256), 256, 0, s>>>(n, nbr, p->k_store, p->n_hop, density, tk, padded,
                                           (p->flags & HOP_PADDED_RULES) ? 1 : 0, hop,
                                           (uint32_t *)ctx->flags.ptr);
    HOPCHK(ctx, hipGetLastError());
    return HOP_OK;
}

int hop_link_sorted_impl(hop_ctx *ctx, int64_t n, const int32_t *nbr16s, const double *dens_s,
                         const double *density, const int32_t *tk, const uint8_t *padded,
                         const hop_params *p, int32_t *hop, hipStream_t s)
{
    if (p->n_hop > 16) return hop_fail(ctx, HOP_ERR_ARG, "the sorted link path needs n_hop <= 16");
    // blocks of 256 sorted positions, xcd_chunk consecutive ones per XCD,
    // walked by 2 workgroups per compute unit
    const int64_t chunk = hop_div_up(hop_div_up(n, 256), 8);
    if (chunk * 8 >= ((int64_t)1 << 31)) return hop_fail(ctx, HOP_ERR_ARG, "too many particles");
    const int64_t per_xcd = std::max<int64_t>(1, std::min<int64_t>(chunk, (int64_t)2 * ctx->n_cu / 8));
    k_hop_sorted<<<(int)(per_xcd * 8), 256, 0, s>>>(n, nbr16s, p->n_hop, dens_s, density, tk, padded,
                                                 (p->flags & HOP_PADDED_RULES) ? 1 : 0, hop,
                                                 (uint32_t *)ctx->flags.ptr, chunk, per_xcd);
    HOPCHK(ctx, hipGetLastError());
    return HOP_OK;
}

int hop_jump_impl(hop_ctx *ctx, int64_t n, int32_t *root, hipStream_t s)
{
    uint32_t *changed = (uint32_t *)ctx->flags.ptr + 1;
    HOPTRY(hop_reserve(ctx, ctx->jump_done, (size_t)n));
    uint8_t *done = (uint8_t *)ctx->jump_done.ptr;
    HOPCHK(ctx, hipMemsetAsync(done, 0, (size_t)n, s));
    for (int rounds = 0;; rounds++) {
        HOPCHK(ctx, hipMemsetAsync(changed, 0, 4, s));
        k_jump<<<hop_grid(n, 256), 256, 0, s>>>(n, root, done, changed);
        HOPCHK(ctx, hipGetLastError());
        HOPCHK(ctx, hipMemcpyAsync(ctx->hflags, changed, 4, hipMemcpyDeviceToHost, s));
        HOPCHK(ctx, hipStreamSynchronize(s));
        if (((uint32_t *)ctx->hflags)[0] == 0u) return HOP_OK;
        // 4 jumps per round: 40 rounds resolve any chain shorter than 2^80
        if (rounds >= 40) return hop_fail(ctx, HOP_ERR_ARG, "links do not reach a self-linked particle");
    }
}

int hop_groups_impl(hop_ctx *ctx, int64_t n, const int32_t *hop, const double *density,
                    const int32_t *tk, const hop_params *p, int32_t *root, int32_t *chain_of,
                    int32_t *n_chains, hipStream_t s)
{
    uint32_t *dflags = (uint32_t *)ctx->flags.ptr;
    uint32_t *total = dflags + 2;
    k_root_init<<<hop_grid(n, 256), 256, 0, s>>>(n, hop, root, dflags);
    HOPCHK(ctx, hipGetLastError());
    HOPTRY(hop_jump_impl(ctx, n, root, s));
    HOPTRY(hop_reserve(ctx, ctx->work_a, (size_t)n * 4));
    uint32_t *flag = (uint32_t *)ctx->work_a.ptr;
    k_chain_flags<<<hop_grid(n, 256), 256, 0, s>>>(n, hop, root, density, tk, p->delta_outer, flag,
                                                   dflags);
    HOPCHK(ctx, hipGetLastError());
    HOPTRY(hop_scan_u32(ctx, flag, n, total, s));
    k_chain_of<<<hop_grid(n, 256), 256, 0, s>>>(n, root, density, tk, p->delta_outer, flag,
                                                chain_of);
    HOPCHK(ctx, hipGetLastError());
    HOPCHK(ctx, hipMemcpyAsync(ctx->hflags, total, 4, hipMemcpyDeviceToHost, s));
    HOPTRY(hop_check_device(ctx, s, "hop_groups"));
    *n_chains = (int32_t)((uint32_t *)ctx->hflags)[0];
    return HOP_OK;
}
