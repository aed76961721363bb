// hop_api.hip -- the C ABI: context, validation, error reporting and the four
// stage entry points declared in include/hop.h.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

#include "hop_internal.h"

int hop_fail(hop_ctx *ctx, int code, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return code;
}

int hop_hip_fail(hop_ctx *ctx, hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return hop_fail(ctx, HOP_ERR_NOMEM, m);
    return hop_fail(ctx, HOP_ERR_HIP, m);
}

int hop_reserve(hop_ctx *ctx, DevBuf &b, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    if (b.bytes >= bytes) return HOP_OK;
    if (b.ptr) {
        // the old contents are not kept; make sure no queued work still uses them
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hop_hip_fail(ctx, e, "hipDeviceSynchronize");
        hipFree(b.ptr);
        b.ptr = nullptr;
        b.bytes = 0;
    }
    size_t want = bytes + bytes / 8;  // headroom against small regrowth
    hipError_t e = hipMalloc(&b.ptr, want);
    if (e != hipSuccess) {
        b.ptr = nullptr;
        (void)hipGetLastError();
        e = hipMalloc(&b.ptr, bytes);
        if (e != hipSuccess) {
            b.ptr = nullptr;
            (void)hipGetLastError();
            return hop_fail(ctx, HOP_ERR_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
        }
        want = bytes;
    }
    b.bytes = want;
    return HOP_OK;
}

int hop_check_device(hop_ctx *ctx, hipStream_t s, const char *stage)
{
    uint32_t *dflags = (uint32_t *)ctx->flags.ptr;
    HOPCHK(ctx, hipMemcpyAsync(&ctx->hflags[1], dflags, 4, hipMemcpyDeviceToHost, s));
    HOPCHK(ctx, hipStreamSynchronize(s));
    uint32_t f = (uint32_t)(ctx->hflags[1] & 0xffffffffu);
    if (f == 0) return HOP_OK;
    // clear so the error is reported once
    HOPCHK(ctx, hipMemsetAsync(dflags, 0, 4, s));
    HOPCHK(ctx, hipStreamSynchronize(s));
    std::string where = std::string(stage) + ": ";
    // causes first: a list the search could not fill (degenerate or beyond
    // the key range) also leaves indices that later stages flag
    if (f & DERR_RANGE) return hop_fail(ctx, HOP_ERR_RANGE, where + "a coordinate is >= 2^grid_bits");
    if (f & DERR_DEGENERATE)
        return hop_fail(ctx, HOP_ERR_DEGENERATE, where + "r_max = 0: n_dens or more coincident particles");
    if (f & DERR_KEYWIDTH)
        return hop_fail(ctx, HOP_ERR_CAPACITY, where + "a neighbour distance exceeds the packed key range");
    if (f & DERR_INDEX) return hop_fail(ctx, HOP_ERR_RANGE, where + "an input index is outside [0, n)");
    if (f & DERR_CAPACITY) return hop_fail(ctx, HOP_ERR_CAPACITY, where + "an internal table overflowed");
    if (f & DERR_CYCLE) return hop_fail(ctx, HOP_ERR_ARG, where + "links do not reach a self-linked particle");
    if (f & DERR_IDS) return hop_fail(ctx, HOP_ERR_ARG, where + "ids are not distinct");
    if (f & DERR_OWNER)
        return hop_fail(ctx, HOP_ERR_ARG, where + "a box index is not the core row of exactly one subvolume");
    return hop_fail(ctx, HOP_ERR_HIP, where + "unknown device error");
}

int hop_check_params(hop_ctx *ctx, int64_t n, const hop_params *p)
{
    if (!p) return hop_fail(ctx, HOP_ERR_ARG, "params is NULL");
    if (!(1 <= p->n_merge && p->n_merge <= p->n_hop && p->n_hop <= p->k_store &&
          p->k_store <= p->n_dens && p->n_dens <= 128 && p->n_dens >= 2))
        return hop_fail(ctx, HOP_ERR_ARG, "need 1 <= n_merge <= n_hop <= k_store <= n_dens <= 128, n_dens >= 2");
    if (p->grid_bits < 1 || p->grid_bits > 21) return hop_fail(ctx, HOP_ERR_ARG, "grid_bits must be in [1, 21]");
    const double d[3] = {p->delta_outer, p->delta_saddle, p->delta_peak};
    for (double v : d)
        if (!std::isfinite(v) || v < 0) return hop_fail(ctx, HOP_ERR_ARG, "thresholds must be finite and >= 0");
    if (!std::isfinite(p->mean_density) || p->mean_density < 0)
        return hop_fail(ctx, HOP_ERR_ARG, "mean_density must be finite and >= 0");
    if (p->flags & ~(HOP_PERIODIC | HOP_DENSITY_FP32 | HOP_PADDED_RULES | HOP_LEARNED_RADIUS))
        return hop_fail(ctx, HOP_ERR_ARG, "unknown flag");
    if (n < p->n_dens) return hop_fail(ctx, HOP_ERR_ARG, "need n >= n_dens");
    if (n >= ((int64_t)1 << 31) - 64) return hop_fail(ctx, HOP_ERR_ARG, "need n < 2^31");
    return HOP_OK;
}

int hop_set_device(hop_ctx *ctx)
{
    HOPCHK(ctx, hipSetDevice(ctx->device));
    return HOP_OK;
}

extern "C" {

void hop_params_default(hop_params *p)
{
    if (!p) return;
    p->n_dens = 64;
    p->n_hop = 16;
    p->n_merge = 4;
    p->k_store = 64;
    p->delta_outer = 80.0;
    p->delta_saddle = 200.0;
    p->delta_peak = 240.0;
    p->mean_density = 0.0;
    p->grid_bits = 21;
    p->flags = HOP_PERIODIC;
}

int hop_ctx_create(int device, hop_ctx **out)
{
    if (!out) return HOP_ERR_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return HOP_ERR_ARG;
    }
    hop_ctx *ctx = new (std::nothrow) hop_ctx();
    if (!ctx) return HOP_ERR_NOMEM;
    ctx->device = device;
    int rc = hop_set_device(ctx);
    if (rc == HOP_OK) {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cu > 0)
            ctx->n_cu = cu;
        else
            (void)hipGetLastError();
    }
    if (rc == HOP_OK) rc = hop_noalloc_init(ctx);
    if (rc == HOP_OK) rc = hop_reserve(ctx, ctx->flags, 4096);
    if (rc == HOP_OK && hipMemset(ctx->flags.ptr, 0, 4096) != hipSuccess) rc = HOP_ERR_HIP;
    if (rc == HOP_OK && hipHostMalloc((void **)&ctx->hflags, 4096, 0) != hipSuccess) rc = HOP_ERR_NOMEM;
    if (rc != HOP_OK) {
        hop_ctx_destroy(ctx);
        return rc;
    }
    std::memset(ctx->hflags, 0, 4096);
    *out = ctx;
    return HOP_OK;
}

void hop_ctx_destroy(hop_ctx *ctx)
{
    if (!ctx) return;
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    DevBuf *bufs[] = {&ctx->keys_a, &ctx->keys_b, &ctx->vals_a, &ctx->vals_b, &ctx->scan_tmp,
                      &ctx->recs, &ctx->boxes, &ctx->tk, &ctx->tk2j, &ctx->flags,
                      &ctx->work_a, &ctx->work_b, &ctx->work_c, &ctx->work_d, &ctx->work_e,
                      &ctx->work_f, &ctx->hash_keys, &ctx->hash_vals, &ctx->edges_lo,
                      &ctx->edges_hi, &ctx->edges_s, &ctx->batch_tab, &ctx->batch_aux,
                      &ctx->cell_counts, &ctx->cell_r, &ctx->radius_w, &ctx->mlp_part, &ctx->miss,
                      &ctx->srt_nbr, &ctx->srt_dens, &ctx->jump_done, &ctx->stitch};
    for (DevBuf *b : bufs)
        if (b->ptr) hipFree(b->ptr);
    if (ctx->hflags) hipHostFree(ctx->hflags);
    delete ctx;
}

const char *hop_last_error(const hop_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : "no context";
}

int hop_set_profiling(hop_ctx *ctx, int on)
{
    if (!ctx) return HOP_ERR_ARG;
    ctx->profiling = on & 3;
    return HOP_OK;
}

int hop_set_tuning(hop_ctx *ctx, const hop_tuning *t)
{
    if (!ctx || !t) return HOP_ERR_ARG;
    ctx->err.clear();
    if (t->front_cap < 1 || t->front_cap > 1024)
        return hop_fail(ctx, HOP_ERR_ARG, "front_cap must be in [1, 1024]");
    if (t->persistent_waves < 0 || t->persistent_waves > (1 << 20))
        return hop_fail(ctx, HOP_ERR_ARG, "persistent_waves must be in [0, 2^20]");
    if ((t->xcd_queues != 0 && t->xcd_queues != 1) || (t->largest_first != 0 && t->largest_first != 1))
        return hop_fail(ctx, HOP_ERR_ARG, "xcd_queues and largest_first must be 0 or 1");
    if (t->hash_slots < 0 || t->hash_slots > (1 << 30))
        return hop_fail(ctx, HOP_ERR_ARG, "hash_slots must be in [0, 2^30]");
    ctx->tuning = *t;
    return HOP_OK;
}

int hop_get_tuning(const hop_ctx *ctx, hop_tuning *t)
{
    if (!ctx || !t) return HOP_ERR_ARG;
    *t = ctx->tuning;
    return HOP_OK;
}

int hop_get_stats(const hop_ctx *ctx, hop_stats *out)
{
    if (!ctx || !out) return HOP_ERR_ARG;
    *out = ctx->stats;
    return HOP_OK;
}

int hop_sync(hop_ctx *ctx, void *stream)
{
    if (!ctx) return HOP_ERR_ARG;
    ctx->err.clear();
    HOPTRY(hop_set_device(ctx));
    return hop_check_device(ctx, (hipStream_t)stream, "hop_sync");
}

// The kNN call; a failed one may leave the sorted copy incomplete, so its
// order is then not offered to later stages (ctx->perm_n = 0).
static int density_call(hop_ctx *ctx, int64_t n, const uint32_t *pos, const int64_t *id,
                        const hop_params *p, double *density, int32_t *nbr, int32_t *nbr16s,
                        double *dens_s, hipStream_t s)
{
    const int rc = hop_density_impl(ctx, n, pos, id, p, density, nbr, nbr16s, dens_s, s);
    if (rc != HOP_OK) ctx->perm_n = 0;
    return rc;
}

int hop_density(hop_ctx *ctx, int64_t n, const uint32_t *pos, const int64_t *id,
                const hop_params *p, double *density, int32_t *nbr, void *stream)
{
    if (!ctx) return HOP_ERR_ARG;
    ctx->err.clear();
    HOPTRY(hop_check_params(ctx, n, p));
    if (!pos || !density) return hop_fail(ctx, HOP_ERR_ARG, "pos and density must be non-NULL");
    HOPTRY(hop_set_device(ctx));
    return density_call(ctx, n, pos, id, p, density, nbr, nullptr, nullptr, (hipStream_t)stream);
}

int hop_density_link(hop_ctx *ctx, int64_t n, const uint32_t *pos, const int64_t *id,
                     const uint8_t *padded, const hop_params *p, double *density, int32_t *nbr,
                     int32_t *hop, void *stream)
{
    if (!ctx) return HOP_ERR_ARG;
    ctx->err.clear();
    HOPTRY(hop_check_params(ctx, n, p));
    if (!pos || !density || !hop) return hop_fail(ctx, HOP_ERR_ARG, "pos, density and hop must be non-NULL");
    HOPTRY(hop_set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    if (p->n_hop > 16) {
        // no sorted copy for longer link lists: the two calls as they are
        if (!nbr) return hop_fail(ctx, HOP_ERR_ARG, "nbr must be non-NULL when n_hop > 16");
        HOPTRY(density_call(ctx, n, pos, id, p, density, nbr, nullptr, nullptr, s));
        const int32_t *tk = id ? (const int32_t *)ctx->tk.ptr : nullptr;
        return hop_link_impl(ctx, n, nbr, density, tk, padded, p, hop, s);
    }
    const size_t rows = (size_t)hop_div_up(n, HOP_BUCKET) * HOP_BUCKET;
    HOPTRY(hop_reserve(ctx, ctx->srt_nbr, rows * 16 * 4));
    HOPTRY(hop_reserve(ctx, ctx->srt_dens, rows * 8));
    int32_t *nbr16s = (int32_t *)ctx->srt_nbr.ptr;
    double *dens_s = (double *)ctx->srt_dens.ptr;
    HOPTRY(density_call(ctx, n, pos, id, p, density, nbr, nbr16s, dens_s, s));
    const int32_t *tk = id ? (const int32_t *)ctx->tk.ptr : nullptr;
    return hop_link_sorted_impl(ctx, n, nbr16s, dens_s, density, tk, padded, p, hop, s);
}

int hop_link(hop_ctx *ctx, int64_t n, const int32_t *nbr, const double *density,
             const int64_t *id, const uint8_t *padded, const hop_params *p, int32_t *hop,
             void *stream)
{
    if (!ctx) return HOP_ERR_ARG;
    ctx->err.clear();
    HOPTRY(hop_check_params(ctx, n, p));
    if (!nbr || !density || !hop) return hop_fail(ctx, HOP_ERR_ARG, "nbr, density and hop must be non-NULL");
    HOPTRY(hop_set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    const int32_t *tk = nullptr;
    if (id) {
        HOPTRY(hop_build_tiekeys(ctx, n, id, s));
        tk = (const int32_t *)ctx->tk.ptr;
    }
    return hop_link_impl(ctx, n, nbr, density, tk, padded, p, hop, s);
}

int hop_groups(hop_ctx *ctx, int64_t n, const int32_t *hop, const double *density,
               const int64_t *id, const hop_params *p, int32_t *root, int32_t *chain_of,
               int32_t *n_chains, void *stream)
{
    if (!ctx) return HOP_ERR_ARG;
    ctx->err.clear();
    HOPTRY(hop_check_params(ctx, n, p));
    if (!hop || !density || !root || !chain_of || !n_chains)
        return hop_fail(ctx, HOP_ERR_ARG, "hop, density, root, chain_of and n_chains must be non-NULL");
    HOPTRY(hop_set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    const int32_t *tk = nullptr;
    if (id) {
        HOPTRY(hop_build_tiekeys(ctx, n, id, s));
        tk = (const int32_t *)ctx->tk.ptr;
    }
    return hop_groups_impl(ctx, n, hop, density, tk, p, root, chain_of, n_chains, s);
}

int hop_merge(hop_ctx *ctx, int64_t n, const int32_t *nbr, const double *density,
              const int32_t *root, const int32_t *chain_of, int32_t n_chains, const int64_t *id,
              const uint8_t *padded, const hop_params *p, int32_t *group, int32_t *n_groups,
              hop_group_info *groups, void *stream)
{
    if (!ctx) return HOP_ERR_ARG;
    ctx->err.clear();
    HOPTRY(hop_check_params(ctx, n, p));
    if (!nbr || !density || !root || !chain_of || !group || !n_groups)
        return hop_fail(ctx, HOP_ERR_ARG, "nbr, density, root, chain_of, group and n_groups must be non-NULL");
    if (n_chains < 0 || n_chains > n) return hop_fail(ctx, HOP_ERR_ARG, "n_chains outside [0, n]");
    HOPTRY(hop_set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    const int32_t *tk = nullptr;
    if (id) {
        HOPTRY(hop_build_tiekeys(ctx, n, id, s));
        tk = (const int32_t *)ctx->tk.ptr;
    }
    return hop_merge_impl(ctx, n, nbr, density, root, chain_of, n_chains, tk, padded, p, group,
                          n_groups, groups, MergeExtra{}, s);
}

}  // extern "C"
