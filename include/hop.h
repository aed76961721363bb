/*
 * hop.h -- C ABI of the MI355X HOP hot path.
 *
 * HOP (Eisenstein & Hut 1998) as described in Skory et al., "Parallel HOP",
 * section 2, run on one GPU for either a whole periodic box or one task's
 * padded subvolume (section 3.1).  The stages are:
 *
 *   hop_density  kNN (N_dens nearest, self included) + SPH density  (sec. 2, stage 1)
 *   hop_link     link to the densest of the N_hop nearest            (sec. 2, stage 2)
 *   hop_density_link  the two above in one call (links formed in Morton order)
 *   hop_groups   chains to self-linked peaks, delta_outer cut        (sec. 2, stage 3; merge step 1)
 *   hop_merge    boundary table, proto-halo and sub-peak merge,
 *                group labels                                        (sec. 2, merge steps 2-5;
 *                                                                     sec. 3.1 last step)
 *   hop_stitch   whole-box chains and halos from padded subvolumes   (sec. 3.1)
 *   hop_halo_stats  per-halo count, centre, maximum radius, bulk velocity
 *                (sec. 3.1 output step)
 *   hop_subhalos substructure at density levels from symmetric chain
 *                boundaries (the paper's subhalo subsection)
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * - All array arguments are DEVICE pointers allocated and owned by the
 *   caller; the library never frees them.  Arrays are indexed by the
 *   caller's particle order ("input order"); neighbour, link, root and peak
 *   values are input-order indices.  The library's internal particle order
 *   never appears in an output.
 * - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *   work and return without waiting, except where a host-side count is
 *   returned (hop_groups, hop_merge): those synchronise `stream` first.
 * - Returns HOP_OK (0) or a negative HOP_ERR_* code; hop_last_error()
 *   gives a message.  Nothing is thrown across the ABI.  On error the
 *   outputs are unspecified but nothing is written out of bounds.
 * - Errors found on the device (coordinate out of range, degenerate
 *   neighbourhood, bad index in an input array) are reported by the next
 *   call that synchronises, at the latest.
 * - A context is not thread-safe; use one context per host thread.
 *   Calls made through one context use its scratch memory, so two calls
 *   on one context must not overlap on different streams.
 * - Particle counts: n_dens <= n < 2^31.
 */
#ifndef HOP_H
#define HOP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define HOP_OK              0
#define HOP_ERR_ARG        (-1) /* bad argument (NULL, size, parameter range)            */
#define HOP_ERR_RANGE      (-2) /* coordinate >= 2^grid_bits, or index out of [0,n)       */
#define HOP_ERR_DEGENERATE (-3) /* r_max = 0: at least n_dens coincident particles        */
#define HOP_ERR_CAPACITY   (-4) /* an internal table could not hold the input             */
#define HOP_ERR_NOMEM      (-5) /* device allocation failed                               */
#define HOP_ERR_HIP        (-6) /* a HIP runtime call failed                              */

/* hop_params.flags */
#define HOP_PERIODIC       0x1u /* whole periodic box: minimum-image distances            */
#define HOP_DENSITY_FP32   0x2u /* FP32 density arithmetic (the FP64 path is the default) */
#define HOP_PADDED_RULES   0x4u /* section 3.1 rules for padded particles                 */
#define HOP_LEARNED_RADIUS 0x8u /* hop_density: search radius from the loaded model,       */
                                /* exact fallback (results unchanged)                      */

/*
 * Parameters (section 4.1 and Table 2 of the paper).  Constraints:
 *   1 <= n_merge <= n_hop <= k_store <= n_dens <= 128,
 *   delta_* finite and >= 0, mean_density > 0 (or 0 for the default),
 *   1 <= grid_bits <= 21.
 * n_dens     particles in the smoothing kernel, self included
 * n_hop      neighbours searched for the densest link, self included
 * n_merge    neighbours searched for chain boundaries, self included
 * k_store    neighbour-list columns written by hop_density
 * delta_outer / delta_saddle / delta_peak   thresholds in units of the mean
 *            density (paper defaults 80 / 2.5*80 / 3*80)
 * mean_density  particles per grid-unit^3 used to normalise the density;
 *            0 selects n / 2^(3*grid_bits), the whole-box value.  For a
 *            subvolume pass the global value (section 2: normalised to the
 *            mean density of the simulation volume).
 * grid_bits  coordinates are integers in [0, 2^grid_bits)
 */
typedef struct hop_params {
    int32_t n_dens;
    int32_t n_hop;
    int32_t n_merge;
    int32_t k_store;
    double delta_outer;
    double delta_saddle;
    double delta_peak;
    double mean_density;
    uint32_t grid_bits;
    uint32_t flags;
} hop_params;

/* one output group (halo); groups are numbered by count descending, then
   peak density descending, then peak index ascending */
typedef struct hop_group_info {
    int64_t count;        /* particles carrying this label                   */
    int32_t peak;         /* input index of the densest particle              */
    int32_t reserved;
    double peak_density;  /* its density                                      */
} hop_group_info;

typedef struct hop_ctx hop_ctx;

/* Fills the defaults: 64/16/4/64, 80/200/240, mean_density 0, 21 bits,
   HOP_PERIODIC. */
void hop_params_default(hop_params *p);

/* Creates a context on HIP device `device`.  The context owns the scratch
   memory (sorted particle copy, search tree, hash tables); it grows on
   demand and is released by hop_ctx_destroy. */
int hop_ctx_create(int device, hop_ctx **out);
void hop_ctx_destroy(hop_ctx *ctx);

/* Message describing the last error on this context ("" if none).  The
   pointer stays valid until the next call on the context. */
const char *hop_last_error(const hop_ctx *ctx);

/*
 * hop_density -- neighbour lists and SPH densities (section 2, stage 1).
 *
 * For every particle i: L_i = [i, then the n_dens-1 nearest others ordered
 * by (squared distance, id)], with minimum-image distances under
 * HOP_PERIODIC, plain differences otherwise.  Distances are exact integers.
 * r_max^2 = d^2 to L_i[n_dens-1], h = r_max/2, and
 *   density[i] = sum_t W(|x_i - x_{L_i[t]}|, h) / mean_density
 * with the M4 cubic spline W (unit masses), summed pairwise over a
 * zero-padded array of 64 slots (128 when n_dens > 64).  The arithmetic
 * is FP64 (round to nearest, no contraction, correctly rounded division
 * and square root).  Under
 * HOP_DENSITY_FP32 the same operation sequence runs in FP32 after rounding
 * 4 d^2 and r_max^2 to FP32; the neighbour lists are unchanged (the search
 * is exact either way) and the densities are returned widened to FP64.
 *
 * n        particle count
 * pos      [n][3] uint32 coordinates, each < 2^grid_bits (else HOP_ERR_RANGE)
 * id       [n] int64 tie-break ids, or NULL to break ties by index.  Must be
 *          distinct when given.
 * density  [n] output, FP64
 * nbr      [n][k_store] output: the first k_store entries of L_i, or NULL
 * Errors: HOP_ERR_DEGENERATE when some r_max is 0.
 */
int hop_density(hop_ctx *ctx, int64_t n, const uint32_t *pos, const int64_t *id,
                const hop_params *p, double *density, int32_t *nbr, void *stream);

/*
 * hop_link -- densest-neighbour links (section 2, stage 2).
 *
 * hop[i] = the particle j among nbr[i][0 .. n_hop) (self included) with the
 * largest density; equal densities go to the smaller id (index when id is
 * NULL).  Under HOP_PADDED_RULES a padded particle links to itself
 * (section 3.1: no chain link from a padded particle).
 *
 * nbr      [n][k_store] as written by hop_density (k_store from p)
 * density  [n]
 * id       [n] or NULL, as given to hop_density
 * padded   [n] uint8 (nonzero = padded) or NULL
 * hop      [n] output
 */
int hop_link(hop_ctx *ctx, int64_t n, const int32_t *nbr, const double *density,
             const int64_t *id, const uint8_t *padded, const hop_params *p, int32_t *hop,
             void *stream);

/*
 * hop_density_link -- hop_density followed by hop_link on its outputs, in
 * one call (section 2, stages 1 and 2).
 *
 * Same results as the two calls: density and nbr as hop_density writes
 * them, hop as hop_link computes it from them.  With n_hop <= 16 the
 * search also keeps, in the context, a copy of each particle's first 16
 * list entries and its density at its position in Morton order, and the
 * links are formed in that order: the neighbours' densities are then
 * gathered by threads that are neighbours in space, mostly from cache,
 * instead of at random.  The copy costs 72 bytes per particle of context
 * memory (held until the context is destroyed).
 *
 * pos, id  as for hop_density
 * padded   [n] uint8 (nonzero = padded) or NULL, as for hop_link
 * density  [n] output
 * nbr      [n][k_store] output, or NULL when n_hop <= 16
 * hop      [n] output
 * Errors: those of hop_density and hop_link; HOP_ERR_ARG when nbr is NULL
 * and n_hop > 16.
 */
int hop_density_link(hop_ctx *ctx, int64_t n, const uint32_t *pos, const int64_t *id,
                     const uint8_t *padded, const hop_params *p, double *density, int32_t *nbr,
                     int32_t *hop, void *stream);

/*
 * hop_groups -- chains (section 2, stage 3 and merge step 1).
 *
 * root[i] = the self-linked particle reached by following hop from i.
 * Particles with density < delta_outer are excluded.  Chains are the roots
 * of the remaining particles, numbered 0..n_chains-1 by the root's id
 * (index when id is NULL); chain_of[i] is that number, -1 when excluded.
 *
 * hop       [n] from hop_link
 * density   [n]
 * id        [n] or NULL
 * root      [n] output
 * chain_of  [n] output
 * n_chains  HOST pointer, output.  Synchronises `stream`.
 * Errors: HOP_ERR_RANGE when a link is outside [0, n); HOP_ERR_ARG when
 * the links close a cycle, so that some particle reaches no self-linked
 * particle (links from hop_link always go uphill and never do).
 */
int hop_groups(hop_ctx *ctx, int64_t n, const int32_t *hop, const double *density,
               const int64_t *id, const hop_params *p, int32_t *root, int32_t *chain_of,
               int32_t *n_chains, void *stream);

/*
 * hop_merge -- chain boundaries, merge and labels (section 2, merge steps
 * 2-5; section 3.1, boundary and output rules).
 *
 * Boundaries: for every chained particle i and j among nbr[i][1 .. n_merge)
 * in a different chain (and, under HOP_PADDED_RULES, not both padded),
 * delta_link = 0.5*(density[i] + density[j]); each chain pair keeps its
 * maximum.  Chains whose peak density >= delta_peak are proto-halos;
 * proto-halos sharing a boundary >= delta_saddle merge; every other chain
 * joins the halo reached through its densest chain of boundaries (the
 * maximum spanning forest of the chain graph with the proto-halos tied to
 * one virtual root; boundaries ordered by delta_link, then chain numbers).
 * Chains that reach no proto-halo are dropped.
 *
 * group[i] = the halo number of particle i, or -1 (excluded, dropped, or
 * padded under HOP_PADDED_RULES).  Halos are numbered by particle count
 * descending, then peak density descending, then peak id ascending; a halo
 * with no labelled particle gets no number.
 *
 * nbr, density, id, padded   as for hop_link
 * root, chain_of, n_chains   from hop_groups
 * group     [n] output
 * n_groups  HOST pointer, output.  Synchronises `stream`.
 * groups    [n_chains] device output table, or NULL; entries 0..n_groups-1
 *           are written
 */
int hop_merge(hop_ctx *ctx, int64_t n, const int32_t *nbr, const double *density,
              const int32_t *root, const int32_t *chain_of, int32_t n_chains, const int64_t *id,
              const uint8_t *padded, const hop_params *p, int32_t *group, int32_t *n_groups,
              hop_group_info *groups, void *stream);

/*
 * hop_stitch -- whole-box chains and halos from padded subvolumes (section
 * 3.1: after each task's own densities and links, chains broken at a
 * subvolume's edge are rebuilt through the padded particles they end on,
 * padded particles take their owners' chains, one boundary table gathers
 * every task's chain pairs, and the merge and labels run once for the box;
 * optionally, each task first premerges its own proto-halos).
 *
 * Input: the rows of hop_run_batch over padded subvolumes cut from one box
 * (with HOP_PADDED_RULES: padded rows link to themselves), each row's box
 * index, and its padding flag.  A chain of a subvolume that ends on a padded
 * row continues at that particle's row in the subvolume where it is local
 * (its owner): following links and these owner steps reaches a local,
 * self-linked row, the chain's peak.  Chains are the peaks at or above
 * delta_outer, numbered by box index.  Every row takes the chain of its
 * owner; boundaries come from every row and its n_merge - 1 listed
 * neighbours (not both padded); merge and labels then follow hop_merge,
 * counting local rows only.  Row densities: by default every row takes its
 * owner's density as well as its chain, and the links of local rows are
 * formed again from their first n_hop list entries with those densities
 * (equal densities to the smaller box index), so a padded particle whose
 * own list was cut short by the padding changes nothing; with
 * HOP_STITCH_TASK_DENSITIES every row keeps the density its subvolume gave
 * it and local rows keep hop_b's links, as independent tasks would.  With
 * HOP_STITCH_PREMERGE each subvolume first joins its own chains (peaks as
 * that subvolume sees them) that reach delta_peak and share a boundary >=
 * delta_saddle; the final merge keeps those joins.  By default, when every
 * local particle's list is its whole-box list (enough padding, rows of each
 * subvolume in increasing box index so that ties go the same way), every
 * output equals that of the whole-box run.
 *
 * offsets    HOST [n_sub + 1] row ranges of the batch, offsets[0] = 0
 * index      [rows] int64: the box index of each row
 * padded     [rows] uint8 (nonzero = padding row); required
 * density_b, nbr_b [rows][k_store], hop_b   hop_run_batch outputs (local
 *            to each subvolume); hop_b is read only with
 *            HOP_STITCH_TASK_DENSITIES (else it may be NULL)
 * p          the box's parameters (HOP_PADDED_RULES required; k_store is
 *            nbr_b's row length)
 * mode       HOP_STITCH_* bits
 * n          box particles; every box index must be the local row of
 *            exactly one subvolume (else HOP_ERR_ARG)
 * density, hop (or NULL), root, chain_of, group   [n] box outputs, box
 *            indices
 * n_chains, n_groups   HOST outputs
 * groups     [rows] device group table or NULL (peaks are box indices)
 * Synchronises `stream`; a row index or link outside its subvolume is
 * HOP_ERR_RANGE.
 */
#define HOP_STITCH_PREMERGE       0x1
#define HOP_STITCH_TASK_DENSITIES 0x2
int hop_stitch(hop_ctx *ctx, int32_t n_sub, const int64_t *offsets, const int64_t *index,
               const uint8_t *padded, const double *density_b, const int32_t *nbr_b,
               const int32_t *hop_b, const hop_params *p, int32_t mode, int64_t n,
               double *density, int32_t *hop, int32_t *root, int32_t *chain_of, int32_t *group,
               int32_t *n_chains, int32_t *n_groups, hop_group_info *groups, void *stream);

/*
 * hop_halo_stats -- per-halo statistics (section 3.1, the output step: each
 * task reports its halos' particle count, centre of mass, maximum radius
 * and bulk velocity; the paper gives no formulas, this is the reading).
 *
 * Members of halo g are the particles with group[i] == g.  Offsets are the
 * integer displacements from the halo's peak particle (groups[g].peak),
 * taken as the minimum image in [-G/2, G/2) under HOP_PERIODIC (G =
 * 2^grid_bits), plain differences otherwise.  With m = (sum of offsets) /
 * count (exact integer sum, one FP64 division):
 *   com[g]   = peak position + m, wrapped into [0, G) under HOP_PERIODIC;
 *   rmax[g]  = max over members of sqrt((dx-mx)^2 + (dy-my)^2 + (dz-mz)^2),
 *              FP64, x + y summed first, correctly rounded square root;
 *   vbulk[g] = mean member velocity, FP64 sum (atomic: the summation order,
 *              and so the last bits, vary within the FP64 summation bound).
 * com and rmax are exact functions of the inputs (the same in every run).
 *
 * pos      [n][3] uint32 as given to hop_density
 * vel      [n][3] float or NULL (then vbulk is not written)
 * group    [n] from hop_merge (-1 = no halo)
 * groups   [n_groups] the table from hop_merge (count and peak are read)
 * com      [n_groups][3] FP64 output
 * rmax     [n_groups] FP64 output
 * vbulk    [n_groups][3] FP64 output, or NULL when vel is NULL
 * Synchronises `stream`.
 * Errors: HOP_ERR_ARG for bad sizes or NULL outputs; HOP_ERR_RANGE when a
 * group number or a table peak is outside range (that group's outputs are
 * not written; nothing is read at the bad index).
 */
int hop_halo_stats(hop_ctx *ctx, int64_t n, const uint32_t *pos, const float *vel,
                   const int32_t *group, int32_t n_groups, const hop_group_info *groups,
                   const hop_params *p, double *com, double *rmax, double *vbulk, void *stream);

/*
 * hop_halo_stats_noalloc -- hop_halo_stats for callers that cannot allocate
 * device memory (code being captured into a HIP graph, serving loops,
 * harnesses that forbid allocation): the same outputs from the same kernels,
 * with the per-halo sums in a static device array of the library instead of
 * context memory.  It calls no allocating routine and does not synchronise:
 * errors on the device (a group number or peak out of range) are reported
 * by the next synchronising call (hop_sync).
 *
 * Limit: n_groups <= HOP_NOALLOC_MAX_GROUPS (else HOP_ERR_ARG); the array
 * (72 bytes per group, 18 MiB) is held on every GPU the library runs on
 * until the process ends.  All calls on one GPU share that array and each
 * clears it first: calls that overlap on one GPU (other streams, other
 * contexts, other threads) race and give wrong results.
 */
#define HOP_NOALLOC_MAX_GROUPS (1 << 18)
int hop_halo_stats_noalloc(hop_ctx *ctx, int64_t n, const uint32_t *pos, const float *vel,
                           const int32_t *group, int32_t n_groups, const hop_group_info *groups,
                           const hop_params *p, double *com, double *rmax, double *vbulk,
                           void *stream);

/*
 * hop_subhalos -- substructure inside the chains (the ADAPTAHOP-style
 * extension sketched in the paper's subhalo subsection: symmetric
 * boundaries between chains, boundary links below a level delta_s
 * destroyed, structures below the Poisson noise rejected, a hierarchy over
 * several levels).  The paper gives no formulas; the readings:
 *   - directed boundary A->B: max of 0.5 (delta_i + delta_j) over chained i
 *     in A and j in B among nbr[i][1 .. n_merge); symmetric boundary {A, B}
 *     when both directions exist, density min(D(A->B), D(B->A));
 *   - at level delta_s: chains joined by symmetric boundaries >= delta_s
 *     form a structure; its members are its particles with density >=
 *     delta_s; its peak the densest member (ties to the smaller id);
 *   - kept when peak density >= delta_s (1 + alpha / sqrt(members));
 *   - numbered per level like the halos (count desc, peak density desc,
 *     peak id asc); parent = the previous level's number at the peak
 *     particle (-1 at the first level or when it has none).
 * The boundary table is not premerged (all links are needed per level).
 *
 * nbr, density, chain_of, n_chains, id   as for hop_merge
 * levels     HOST [n_levels] ascending delta_s values, 1 <= n_levels <= 64
 * alpha      significance factor (0 keeps every structure with a member)
 * sub        [n_levels][n] device output: structure number or -1
 * t_off      HOST [n_levels + 1] output: level l's structures are table
 *            entries [t_off[l], t_off[l+1])
 * table      device [n_levels * n_chains] output, or NULL
 * Synchronises `stream`.
 */
typedef struct hop_subhalo_info {
    int64_t count;        /* members (density >= the level)          */
    int32_t peak;         /* input index of the densest member        */
    int32_t parent;       /* number at the previous level, or -1      */
    double peak_density;
} hop_subhalo_info;

int hop_subhalos(hop_ctx *ctx, int64_t n, const int32_t *nbr, const double *density,
                 const int32_t *chain_of, int32_t n_chains, const int64_t *id,
                 const hop_params *p, int32_t n_levels, const double *levels, double alpha,
                 int32_t *sub, int64_t *t_off, hop_subhalo_info *table, void *stream);

/*
 * hop_run_batch -- the whole path (density, links, chains, merge, labels)
 * for n_sub independent subvolumes in one call, with one persistent kNN
 * launch over all of them.  The shape is that of the paper's per-task work
 * (section 3.1): every subvolume is a separate non-periodic (or periodic,
 * by HOP_PERIODIC) problem with its own frame, its own padding flags and
 * the caller's mean density; neighbours, boundaries and merges never cross
 * subvolumes.  The result for each subvolume equals what hop_density,
 * hop_link, hop_groups and hop_merge give for it alone (ids are not taken:
 * ties go to the smaller index within the subvolume).
 *
 * n_sub         number of subvolumes, 1 <= n_sub <= 65536
 * offsets       HOST [n_sub+1]: subvolume s holds particles
 *               [offsets[s], offsets[s+1]) of every per-particle array;
 *               offsets[0] = 0, each subvolume holds >= n_dens particles,
 *               offsets[n_sub] < 2^31
 * pos           [n][3] uint32, each subvolume in its own coordinate frame
 * padded        [n] uint8 or NULL
 * mean_density  HOST [n_sub] normalisation per subvolume, or NULL; an entry
 *               <= 0 selects that subvolume's own count / 2^(3*grid_bits)
 * density, nbr, hop, root, chain_of, group
 *               [n] (nbr [n][k_store]) outputs, all required; every index
 *               and number is local to its subvolume (0-based)
 * n_chains, n_groups   HOST [n_sub] outputs
 * groups        device [sum of chains] group tables, or NULL: subvolume s
 *               owns entries [group_off[s], group_off[s+1]); peaks are local
 * group_off     HOST [n_sub+1] output, or NULL
 * Synchronises `stream`.
 */
int hop_run_batch(hop_ctx *ctx, int32_t n_sub, const int64_t *offsets, const uint32_t *pos,
                  const uint8_t *padded, const double *mean_density, const hop_params *p,
                  double *density, int32_t *nbr, int32_t *hop, int32_t *root, int32_t *chain_of,
                  int32_t *group, int32_t *n_chains, int32_t *n_groups, hop_group_info *groups,
                  int64_t *group_off, void *stream);

/*
 * Launch settings that change speed, never results.  hop_set_tuning takes
 * effect from the next call on the context.
 * front_cap         frontier entries the kNN walk may produce before it
 *                   stops descending and streams whole subtrees (1..1024,
 *                   default 1024)
 * persistent_waves  waves of the persistent kNN launches, of one box and of
 *                   a batch (0 = as many as fit: 4 per compute unit, one
 *                   per SIMD, or 2 when n_dens > 64; at least 8)
 * xcd_queues        batched launch: 1 = one work chunk per XCD, idle waves
 *                   move on to the other chunks (default); 0 = one queue
 * largest_first     batched launch: 1 = subvolumes in decreasing size
 *                   (default); 0 = in the given order
 * hash_slots        initial slots of the boundary table, rounded up to a
 *                   power of two (0 = sized from the chain and pair counts,
 *                   default; 1..2^30 otherwise).  A table that overflows is
 *                   doubled and rebuilt until it holds every chain pair.
 */
typedef struct hop_tuning {
    int32_t front_cap;
    int32_t persistent_waves;
    int32_t xcd_queues;
    int32_t largest_first;
    int32_t hash_slots;
} hop_tuning;

int hop_set_tuning(hop_ctx *ctx, const hop_tuning *t);
int hop_get_tuning(const hop_ctx *ctx, hop_tuning *t);

/*
 * Learned search radius.  The paper searches a fixed number of neighbours
 * per particle; this extension predicts each particle's search radius from
 * the particle counts of the 3x3x3 cells around its cell, so that the kNN
 * walk can prune with it from the start.  The prediction only prunes: a
 * particle whose n_dens-1 nearest others all lie within its radius keeps
 * the list found; every other particle ("miss") is searched again without
 * the radius.  Outputs are identical with and without the flag.
 *
 * Cells have side 2^cell_bits grid units.  Features of a particle: the 27
 * values log(1 + count) of the cells (cz+dz, cy+dy, cx+dx), dz outermost,
 * each of dz, dy, dx running -1, 0, 1 (periodic wrap under HOP_PERIODIC,
 * count 0 outside otherwise).  Target: log(r / 2^cell_bits), r the distance
 * to the particle's n_dens-th list entry.  The network maps the features to
 * the target: 27 -> 64 -> 64 -> 1 with ReLU after the hidden layers; its
 * parameters are one FP32 vector of HOP_MLP_PARAMS numbers in the order
 * W1 [27][64] (input-major), b1 [64], W2 [64][64], b2 [64], W3 [64], b3 [1].
 */
#define HOP_MLP_PARAMS      6017
#define HOP_RADIUS_MLP      1  /* the network, BF16 weights, FP32 accumulation      */
#define HOP_RADIUS_ANALYTIC 2  /* no network: the radius whose ball holds n_dens
                                  particles at the 27 cells' mean density          */

/* Cell side bits hop_density uses for n particles: cells of side
   2^cell_bits hold `occupancy` particles on average (between 2 and 2^9 cells
   per axis).  Host-only; -1 on bad arguments. */
int hop_radius_cell_bits(int64_t n, uint32_t grid_bits, float occupancy);

/* Features [n][27] (and, if target is non-NULL, targets [n] from the
   neighbour lists nbr [n][k_store], which need k_store = n_dens) for cells
   of side 2^cell_bits; at most 2^9 cells per axis.  Synchronises. */
int hop_radius_dataset(hop_ctx *ctx, int64_t n, const uint32_t *pos, const int32_t *nbr,
                       const hop_params *p, int32_t cell_bits, float *feats, float *target,
                       void *stream);

/* Mean squared error of the network w (device FP32 [HOP_MLP_PARAMS]) over
   `batch` rows of (feats, target), rows idx[0..batch) (device) or the
   first `batch` rows when idx is NULL, and its gradient grad
   [HOP_MLP_PARAMS] (device); loss (device, 1 float) may be NULL.  FP32,
   deterministic (fixed summation order).  Synchronises. */
int hop_mlp_grad(hop_ctx *ctx, int64_t n_samples, const float *feats, const float *target,
                 const int32_t *idx, int32_t batch, const float *w, float *grad, float *loss,
                 void *stream);

/* `steps` Adam steps (Kingma & Ba, bias-corrected) of the mean squared
   error, step t using rows idx[t*batch .. (t+1)*batch) (device; NULL = the
   first `batch` rows every step).  w, m, v (device FP32
   [HOP_MLP_PARAMS]) are updated in place; the first step is number
   first_step (>= 1) for the bias correction; loss (device [steps] or NULL)
   receives each step's loss before its update.  Synchronises. */
int hop_mlp_train(hop_ctx *ctx, int64_t n_samples, const float *feats, const float *target,
                  const int32_t *idx, int32_t steps, int32_t batch, int32_t first_step, float lr,
                  float beta1, float beta2, float eps, float *w, float *m, float *v, float *loss,
                  void *stream);

/* Loads the radius model used under HOP_LEARNED_RADIUS: kind 1 (w = device
   FP32 parameters, rounded to BF16 to nearest even) or 2 (w ignored), 0 to
   unload.  The search radius of a cell is 2^cell_bits * exp(prediction +
   margin); hop_density picks cell_bits so that cells hold `occupancy`
   particles on average.  Synchronises. */
int hop_radius_load(hop_ctx *ctx, int32_t kind, const float *w, float margin, float occupancy,
                    void *stream);

/* The loaded model's prediction (log(r / side), margin not added) for rows
   of features [rows][27] (device) into out [rows] (device).  Synchronises. */
int hop_radius_predict(hop_ctx *ctx, int64_t rows, const float *feats, int32_t n_dens, float *out,
                       void *stream);

/* Synchronises `stream` and reports any error the device recorded since the
   last synchronising call (see the conventions above). */
int hop_sync(hop_ctx *ctx, void *stream);

/* Per-call statistics of the last hop_density (and premerge count of the
   last hop_stitch) on this context. */
typedef struct hop_stats {
    double ms_sort;         /* Morton sort + tree build                          */
    double ms_knn;          /* kNN + density kernel(s), fallback pass included   */
    int64_t n;              /* particles                                          */
    int64_t nodes_visited;  /* tree nodes tested, summed over waves (0 if off)   */
    int64_t leaves_scanned; /* leaves whose points were tested                   */
    double ms_radius;       /* HOP_LEARNED_RADIUS: cell counts + per-cell model  */
    int64_t misses;         /* HOP_LEARNED_RADIUS: particles searched again      */
    int64_t redo_buckets;   /* HOP_LEARNED_RADIUS: buckets of the fallback pass  */
    int64_t premerged;      /* hop_stitch with premerge: row pairs that joined
                               two chains inside a subvolume; hop_subhalos:
                               symmetric chain boundaries                        */
    int64_t insert_iterations; /* kNN: heap-insertion loop iterations, summed
                                  over buckets (each runs for all 64 lanes);
                                  this and `offered` are counted by the main
                                  search of hop_density / hop_density_link, not
                                  by a learned-radius fallback pass or by
                                  hop_run_batch                                */
    int64_t offered;        /* kNN: candidates offered to a lane's heap (those
                               within the lane's bound when their batch was
                               tested; each costs the lane one iteration)        */
} hop_stats;

/* Profiling bits (default 0): 1 = time the sort/tree and kNN stages of
   hop_density with HIP events (synchronises the stream inside the call);
   2 = also count tree nodes tested, leaves scanned, heap-insertion loop
   iterations and offered candidates (device atomics). */
int hop_set_profiling(hop_ctx *ctx, int on);
int hop_get_stats(const hop_ctx *ctx, hop_stats *out);

#ifdef __cplusplus
}
#endif

#endif /* HOP_H */
