// hop_internal.h -- declarations shared by the HIP translation units of the
// HOP library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/hop.h"

// Device-side error bits, accumulated in ctx->dflags[0] with atomicOr.
enum : uint32_t {
    DERR_RANGE = 1u,       // coordinate >= 2^grid_bits
    DERR_DEGENERATE = 2u,  // r_max == 0
    DERR_KEYWIDTH = 4u,    // a neighbour distance did not fit the packed key
    DERR_INDEX = 8u,       // an input index outside [0, n)
    DERR_CAPACITY = 16u,   // a hash table or queue overflowed
    DERR_CYCLE = 32u,      // links that do not reach a self-linked particle
    DERR_IDS = 64u,        // duplicate ids
    DERR_OWNER = 128u,     // stitching: a box index is not the core row of exactly one subvolume
};

// One particle of the Morton-sorted copy: FP64 coordinates (exact copies of
// the integer grid coordinates), its input index and its tie key.
struct __align__(16) SortedRec {
    double x, y, z;
    int32_t j;   // input index
    int32_t tk;  // tie key: rank of (id, index), = j when no ids are given
};

// Axis-aligned box of a tree node, integer grid coordinates.
struct __align__(16) NodeBox {
    uint32_t lo[3];
    uint32_t count;  // particles below the node
    uint32_t hi[3];
    uint32_t pad;
};

#define HOP_LEAF 16        // particles per tree leaf
#define HOP_BUCKET 64      // particles per query bucket (one wavefront)
#define HOP_MAX_LEVELS 32

struct TreeLevels {
    int64_t off[HOP_MAX_LEVELS];  // first node of each level (level 0 = leaves)
    int32_t cnt[HOP_MAX_LEVELS];  // nodes in each level
    int32_t top;                  // root level
};

// A growable device buffer owned by the context.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct hop_ctx {
    int device = 0;
    std::string err;
    int profiling = 0;
    int n_cu = 256;  // compute units of the device
    hop_tuning tuning{1024, 0, 1, 1, 0};
    hop_stats stats{};

    // device scratch
    DevBuf keys_a, keys_b, vals_a, vals_b;  // radix sort double buffers
    DevBuf scan_tmp;                         // scan partial sums
    DevBuf recs;                             // SortedRec[n]
    DevBuf boxes;                            // NodeBox[nodes]
    DevBuf tk, tk2j;                         // tie keys (when ids are given)
    DevBuf flags;                            // device counters / error bits
    DevBuf work_a, work_b, work_c, work_d, work_e, work_f;  // stage scratch
    DevBuf hash_keys, hash_vals;
    DevBuf edges_lo, edges_hi, edges_s;
    DevBuf batch_tab, batch_aux;  // batched launch: work description, per-subvolume bases
    DevBuf cell_counts, cell_r;   // learned radius: particles and search radius per cell
    DevBuf radius_w, mlp_part;    // BF16 model weights; training partial sums
    DevBuf miss;                  // learned radius: per-bucket lanes to search again
    DevBuf srt_nbr, srt_dens;     // density + links: sorted copies of list heads and densities
    DevBuf jump_done;             // chains: particles whose root is final
    DevBuf stitch;                // stitching: owner rows, virtual-link roots, labels
    // hop_halo_stats_noalloc: this device's address of the static scratch
    // (set at context creation by hop_noalloc_init)
    void *noalloc_scratch = nullptr;
    int radius_kind = 0;          // HOP_RADIUS_* of the loaded model, 0 = none
    float radius_margin = 0.0f;
    float radius_occupancy = 8.0f;
    // pinned host mirror of the device counters
    int64_t *hflags = nullptr;

    // Morton order of the last hop_density (sorted position -> input index),
    // valid for perm_n particles.  Other stages may use it as a processing
    // order; their results do not depend on it.
    int64_t perm_n = 0;
};

// ---------------------------------------------------------------------------
// host helpers (hop_api.hip)
// ---------------------------------------------------------------------------
int hop_fail(hop_ctx *ctx, int code, const std::string &msg);
int hop_hip_fail(hop_ctx *ctx, hipError_t e, const char *what);
int hop_reserve(hop_ctx *ctx, DevBuf &b, size_t bytes);
int hop_check_params(hop_ctx *ctx, int64_t n, const hop_params *p);
int hop_set_device(hop_ctx *ctx);
// Looks up this device's address of the static scratch of
// hop_halo_stats_noalloc (hop_stats.hip); the context's device is current.
int hop_noalloc_init(hop_ctx *ctx);
// Reads the device error bits (synchronising the stream) and turns them into
// a return code.
int hop_check_device(hop_ctx *ctx, hipStream_t s, const char *stage);

#define HOPCHK(ctx, call)                                              \
    do {                                                               \
        hipError_t _e = (call);                                        \
        if (_e != hipSuccess) return hop_hip_fail((ctx), _e, #call);   \
    } while (0)

#define HOPTRY(call)                  \
    do {                              \
        int _rc = (call);             \
        if (_rc != HOP_OK) return _rc; \
    } while (0)

// ---------------------------------------------------------------------------
// primitives (hop_sort.hip)
// ---------------------------------------------------------------------------
// Exclusive scan of n uint32 values, in place; the total is written to
// *total_dev (device pointer) when non-null.  Totals must stay below 2^32.
int hop_scan_u32(hop_ctx *ctx, uint32_t *data, int64_t n, uint32_t *total_dev, hipStream_t s);
// Stable LSD radix sort of (key, value) pairs on key bits [lo_bit, bits)
// (pairs equal on those bits keep their input order).  keys/vals hold the
// input and receive the output; tk/tv are scratch of the same sizes.
int hop_radix_sort(hop_ctx *ctx, uint64_t *keys, uint32_t *vals, uint64_t *tk, uint32_t *tv,
                   int64_t n, int bits, hipStream_t s, int lo_bit = 0);

// ---------------------------------------------------------------------------
// stages
// ---------------------------------------------------------------------------
// Builds the tie keys for ids (tk[i] = rank of (id_i, i)) into ctx->tk and
// the inverse into ctx->tk2j.
int hop_build_tiekeys(hop_ctx *ctx, int64_t n, const int64_t *id, hipStream_t s);
// nbr16s / dens_s (both NULL or both set, n rounded up to whole buckets):
// a copy of the first 16 list entries and of the densities in Morton
// (sorted) order, for hop_link_sorted_impl.
int hop_density_impl(hop_ctx *ctx, int64_t n, const uint32_t *pos, const int64_t *id,
                     const hop_params *p, double *density, int32_t *nbr, int32_t *nbr16s,
                     double *dens_s, hipStream_t s);
int hop_link_impl(hop_ctx *ctx, int64_t n, const int32_t *nbr, const double *density,
                  const int32_t *tk, const uint8_t *padded, const hop_params *p, int32_t *hop,
                  hipStream_t s);
// The same links from the sorted copies of the last hop_density_impl on
// this context (entry 0 of each copied row is the particle itself); needs
// n_hop <= 16.
int hop_link_sorted_impl(hop_ctx *ctx, int64_t n, const int32_t *nbr16s, const double *dens_s,
                         const double *density, const int32_t *tk, const uint8_t *padded,
                         const hop_params *p, int32_t *hop, hipStream_t s);
// Leaves the exclusive scan of the chain-root flags (indexed by tie key)
// in ctx->work_a: entry k = number of chains whose root has tie key < k.
int hop_groups_impl(hop_ctx *ctx, int64_t n, const int32_t *hop, const double *density,
                    const int32_t *tk, const hop_params *p, int32_t *root, int32_t *chain_of,
                    int32_t *n_chains, hipStream_t s);
// Optional inputs of hop_merge_impl beyond the plain call.
struct MergeExtra {
    // chain_base (device, [n_sub+1]): for a batch, the first chain of each
    // subvolume; the halos are then ordered by subvolume first, and
    // group_first (device, [n_sub]) receives the first group of each
    // subvolume that has one (entries of the others are left alone)
    const int32_t *chain_base = nullptr;
    int32_t n_sub = 0;
    int32_t *group_first = nullptr;
    // tk holds the output indices themselves (group peaks are tk values);
    // otherwise tk is a rank of ids and ctx->tk2j maps it back
    bool tk_is_index = false;
    // chain pairs (device, lo[n_pre], hi[n_pre]) joined into one halo before
    // the labels, besides the proto-halo pairs of the boundary table
    const int32_t *pre_lo = nullptr, *pre_hi = nullptr;
    int64_t n_pre = 0;
};
int hop_merge_impl(hop_ctx *ctx, int64_t n, const int32_t *nbr, const double *density,
                   const int32_t *root, const int32_t *chain_of, int32_t n_chains,
                   const int32_t *tk, const uint8_t *padded, const hop_params *p, int32_t *group,
                   int32_t *n_groups, hop_group_info *groups, const MergeExtra &x, hipStream_t s);
// Pointer jumping root[i] <- root[root[i]] until no root changes (root
// holds links on entry, roots on return); HOP_ERR_ARG if it does not end.
int hop_jump_impl(hop_ctx *ctx, int64_t n, int32_t *root, hipStream_t s);
// kNN + density for a batch of subvolumes (offsets on the host); neighbour
// lists hold batch-wide input indices.  *sub_off_dev receives a device copy
// of the offsets, valid until the next batched call.
int hop_density_batch_impl(hop_ctx *ctx, int32_t n_sub, const int64_t *off, const uint32_t *pos,
                           const double *mean_density, const hop_params *p, double *density,
                           int32_t *nbr, int32_t *nbr16s, double *dens_s, int64_t **sub_off_dev,
                           hipStream_t s);

// Learned radius: cell side bits for n particles, and the per-cell search
// radii of pos (cell counts, then the loaded model per cell).
int hop_cell_bits(const hop_ctx *ctx, int64_t n, const hop_params *p);
int hop_radius_cells(hop_ctx *ctx, int64_t n, const uint32_t *pos, const hop_params *p, hipStream_t s,
                     const float **cell_r, int *cb, int *gb);

static inline int64_t hop_div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }
static inline int hop_grid(int64_t items, int per_block)
{
    int64_t g = hop_div_up(items, per_block);
    return (int)(g < 1 ? 1 : g);
}
