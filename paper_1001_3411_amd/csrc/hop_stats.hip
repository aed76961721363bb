// hop_stats.hip -- per-halo statistics after the labels: particle count,
// centre of mass, maximum radius and bulk velocity (the per-task output the
// paper lists in section 3.1 and section 5).
//
// Offsets are integer displacements from each halo's peak particle, the
// minimum image (representative in [-G/2, G/2)) in a periodic box of side
// G = 2^grid_bits, so halos straddling the box edge are unwrapped.  Their
// per-halo sums are 64-bit integer atomics (in LDS per block first for the
// largest halos), exact in any order; the mean
// offset is one FP64 division, so the centre is the same in every run.
// The maximum radius is an atomic maximum over the FP64 bits of each
// member's distance (non-negative doubles order like their bits).  The
// velocity sums are FP64 atomics: their order, and so their last bits,
// vary from run to run within the FP64 summation bound.
#include <algorithm>
#include <string>

#include "hop_internal.h"

namespace {

__device__ __forceinline__ int64_t min_image(int64_t d, int periodic, int64_t G)
{
    if (!periodic) return d;
    d &= G - 1;  // d mod G in [0, G) (G a power of two, two's complement)
    return d >= (G >> 1) ? d - G : d;
}

// Halos are numbered by size, largest first: the members of halos below
// kPriv are summed in LDS per block and flushed with one global atomic per
// block and sum, so the largest halos do not serialise on a few addresses.
// The blocks stride over the particles (a fixed grid), so each block's
// flush is paid once for many particles.
//
// The particles are taken in the order of `order` when it is given (the
// sorted copy of the last kNN call on n particles: Morton order, a
// permutation of [0, n)), else in input order.  In Morton order the 64
// lanes of a wave are neighbours in space and mostly members of one halo,
// so each wave first adds up its runs of lanes with equal halo numbers
// (a segmented scan over the lanes) and the last lane of each run makes
// the run's atomics: one per run and sum instead of one per particle.  The
// offset sums are integers, exact in any order; only the velocity sums'
// last bits depend on the order (as they do on the atomics').
constexpr int kPriv = 1024;
constexpr int kStatsBlock = 256;

// the lane-order neighbours' halo numbers and run boundaries of a wave
__device__ __forceinline__ bool run_head(int32_t g, int lane)
{
    const int32_t gp = __shfl_up(g, 1);
    return lane == 0 || gp != g;
}

__device__ __forceinline__ bool run_tail(int32_t g, int lane)
{
    const int32_t gn = __shfl_down(g, 1);
    return lane == 63 || gn != g;
}

__global__ void __launch_bounds__(kStatsBlock)
k_stats_sum(int64_t n, const uint32_t *__restrict__ pos, const float *__restrict__ vel,
            const int32_t *__restrict__ group, int32_t n_groups,
            const hop_group_info *__restrict__ groups, int periodic, int64_t G,
            const SortedRec *__restrict__ order, unsigned long long *__restrict__ osum,
            double *__restrict__ vsum, uint32_t *__restrict__ dflags)
{
    __shared__ unsigned long long lo[kPriv * 3];
    __shared__ double lv[kPriv * 3];
    for (int t = threadIdx.x; t < kPriv * 3; t += kStatsBlock) {
        lo[t] = 0ull;
        lv[t] = 0.0;
    }
    __syncthreads();
    const int lane = (int)(threadIdx.x & 63);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t base = wave * 64; base < n; base += n_waves * 64) {
        const int64_t t = base + lane;
        int32_t g = -1;
        long long d[3] = {0, 0, 0};
        double v[3] = {0.0, 0.0, 0.0};
        const int64_t i = t < n ? (order ? (int64_t)order[t].j : t) : -1;
        if (t < n && (i < 0 || i >= n)) atomicOr(dflags, DERR_INDEX);
        if (i >= 0 && i < n) {
            g = group[i];
            if (g >= n_groups) {
                atomicOr(dflags, DERR_INDEX);
                g = -1;
            } else if (g >= 0) {
                const int32_t pk = groups[g].peak;
                if (pk < 0 || pk >= n) {
                    atomicOr(dflags, DERR_INDEX);
                    g = -1;
                } else {
#pragma unroll
                    for (int k = 0; k < 3; k++) {
                        d[k] = min_image((int64_t)pos[3 * i + k] - (int64_t)pos[3 * (int64_t)pk + k],
                                         periodic, G);
                        if (vel) v[k] = (double)vel[3 * i + k];
                    }
                }
            }
        }
        // segmented inclusive sums over the runs of equal g: a lane adds the
        // partial sum `off` lanes below until its range reaches its run's head
        bool f = run_head(g, lane);
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            long long du[3];
            double vu[3];
#pragma unroll
            for (int k = 0; k < 3; k++) {
                du[k] = __shfl_up(d[k], off);
                vu[k] = vel ? __shfl_up(v[k], off) : 0.0;
            }
            const bool fu = __shfl_up((int)f, off) != 0;
            if (lane >= off && !f) {
#pragma unroll
                for (int k = 0; k < 3; k++) {
                    d[k] += du[k];
                    v[k] = vu[k] + v[k];
                }
                f = fu;
            }
        }
        const bool tail = run_tail(g, lane);  // (every lane takes part in the shuffle)
        if (g >= 0 && tail) {
#pragma unroll
            for (int k = 0; k < 3; k++) {
                if (g < kPriv) {
                    atomicAdd(&lo[3 * g + k], (unsigned long long)d[k]);  // two's complement sum
                    if (vel) atomicAdd(&lv[3 * g + k], v[k]);
                } else {
                    atomicAdd(&osum[3 * (int64_t)g + k], (unsigned long long)d[k]);
                    if (vel) atomicAdd(&vsum[3 * (int64_t)g + k], v[k]);
                }
            }
        }
    }
    __syncthreads();
    const int lim = min(n_groups, kPriv) * 3;
    for (int t = threadIdx.x; t < lim; t += kStatsBlock) {
        if (lo[t]) atomicAdd(&osum[t], lo[t]);
        if (vel && lv[t] != 0.0) atomicAdd(&vsum[t], lv[t]);
    }
}

// per halo: mean offset, centre, bulk velocity
// A group whose peak lies outside [0, n) (a table that does not belong to
// these particles) gets no centre and sets DERR_INDEX; nothing is read at
// the bad index.
__global__ void k_stats_halo(int64_t n, int32_t n_groups, const uint32_t *__restrict__ pos,
                             const hop_group_info *__restrict__ groups, int periodic, int64_t G,
                             const unsigned long long *__restrict__ osum, const double *__restrict__ vsum,
                             double *__restrict__ mean, double *__restrict__ com, double *__restrict__ vbulk,
                             uint32_t *__restrict__ dflags)
{
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_groups) return;
    const double c = (double)groups[g].count;
    const int64_t p = groups[g].peak;
    if (p < 0 || p >= n) {
        atomicOr(dflags, DERR_INDEX);
        return;
    }
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const double m = (double)(int64_t)osum[3 * g + k] / c;
        mean[3 * g + k] = m;
        double x = (double)pos[3 * p + k] + m;
        if (periodic) {
            const double Gd = (double)G;
            x = x < 0.0 ? x + Gd : (x >= Gd ? x - Gd : x);
        }
        com[3 * g + k] = x;
        if (vbulk) vbulk[3 * g + k] = vsum[3 * g + k] / c;
    }
}

// Maximum radius per halo, in input order: its reads are contiguous there,
// and with one atomic maximum per member it is faster than in Morton order
// with gathered reads (3.7 against 5.4 ms at 134M particles).
__global__ void __launch_bounds__(kStatsBlock)
k_stats_radius(int64_t n, const uint32_t *__restrict__ pos, const int32_t *__restrict__ group,
               int32_t n_groups, const hop_group_info *__restrict__ groups, int periodic,
               int64_t G, const double *__restrict__ mean,
               unsigned long long *__restrict__ rmax_bits)
{
    __shared__ unsigned long long lr[kPriv];
    for (int t = threadIdx.x; t < kPriv; t += kStatsBlock) lr[t] = 0ull;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t g = group[i];
        if (g < 0 || g >= n_groups) continue;
        const int64_t pk = groups[g].peak;
        if (pk < 0 || pk >= n) continue;
        double e[3];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const int64_t d = min_image((int64_t)pos[3 * i + k] - (int64_t)pos[3 * pk + k], periodic, G);
            e[k] = (double)d - mean[3 * (int64_t)g + k];
        }
        const double r = __builtin_sqrt((e[0] * e[0] + e[1] * e[1]) + e[2] * e[2]);
        // non-negative doubles order like their bit patterns
        const unsigned long long rb = (unsigned long long)__double_as_longlong(r);
        if (g < kPriv) atomicMax(&lr[g], rb);
        else atomicMax(&rmax_bits[g], rb);
    }
    __syncthreads();
    const int lim = min(n_groups, kPriv);
    for (int t = threadIdx.x; t < lim; t += kStatsBlock)
        if (lr[t]) atomicMax(&rmax_bits[t], lr[t]);
}

}  // namespace

namespace {

__global__ void k_zero_u64(unsigned long long *__restrict__ p, int64_t n)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0ull;
}

// Argument checks shared by both entry points.
int stats_args(hop_ctx *ctx, int64_t n, const uint32_t *pos, const float *vel, const int32_t *group,
               int32_t n_groups, const hop_group_info *groups, const hop_params *p, double *com,
               double *rmax, double *vbulk)
{
    if (!p) return hop_fail(ctx, HOP_ERR_ARG, "params is NULL");
    if (n < 1 || n >= ((int64_t)1 << 31)) return hop_fail(ctx, HOP_ERR_ARG, "need 1 <= n < 2^31");
    if (n_groups < 0) return hop_fail(ctx, HOP_ERR_ARG, "n_groups < 0");
    if (p->grid_bits < 1 || p->grid_bits > 21) return hop_fail(ctx, HOP_ERR_ARG, "grid_bits must be in [1, 21]");
    if (!pos || !group || (n_groups > 0 && (!groups || !com || !rmax)))
        return hop_fail(ctx, HOP_ERR_ARG, "pos, group, groups, com and rmax must be non-NULL");
    if (vel && !vbulk) return hop_fail(ctx, HOP_ERR_ARG, "vbulk must be non-NULL when vel is given");
    return HOP_OK;
}

// The three passes over scratch osum/vsum/mean (3 n_groups words each),
// cleared here with fill kernels (no memset nodes, no allocation).
int stats_launch(hop_ctx *ctx, int64_t n, const uint32_t *pos, const float *vel, const int32_t *group,
                 int32_t n_groups, const hop_group_info *groups, const hop_params *p, double *com,
                 double *rmax, double *vbulk, unsigned long long *osum, double *vsum, double *mean,
                 hipStream_t s)
{
    const int periodic = (p->flags & HOP_PERIODIC) ? 1 : 0;
    const int64_t G = (int64_t)1 << p->grid_bits;
    const int64_t g3 = (int64_t)n_groups * 3;
    k_zero_u64<<<hop_grid(2 * g3, 256), 256, 0, s>>>(osum, 2 * g3);  // osum and vsum are adjacent
    k_zero_u64<<<hop_grid(n_groups, 256), 256, 0, s>>>((unsigned long long *)rmax, n_groups);
    const int grid = (int)std::min<int64_t>(hop_grid(n, kStatsBlock), (int64_t)ctx->n_cu * 8);
    // the sums in Morton order when the context's last kNN call sorted n
    // particles (any permutation gives the same offsets; an index outside [0, n),
    // which only a sorted copy left incomplete by a failed call could hold,
    // is reported like a bad group number)
    const SortedRec *order = (ctx->perm_n == n && ctx->recs.bytes >= (size_t)n * sizeof(SortedRec))
                                 ? (const SortedRec *)ctx->recs.ptr
                                 : nullptr;
    k_stats_sum<<<grid, kStatsBlock, 0, s>>>(n, pos, vel, group, n_groups, groups, periodic, G, order,
                                             osum, vel ? vsum : nullptr, (uint32_t *)ctx->flags.ptr);
    HOPCHK(ctx, hipGetLastError());
    k_stats_halo<<<hop_grid(n_groups, 256), 256, 0, s>>>(n, n_groups, pos, groups, periodic, G, osum,
                                                         vsum, mean, com, vel ? vbulk : nullptr,
                                                         (uint32_t *)ctx->flags.ptr);
    HOPCHK(ctx, hipGetLastError());
    k_stats_radius<<<grid, kStatsBlock, 0, s>>>(n, pos, group, n_groups, groups, periodic, G, mean,
                                                (unsigned long long *)rmax);
    HOPCHK(ctx, hipGetLastError());
    return HOP_OK;
}

// Scratch of hop_halo_stats_noalloc: 9 words per group (offset sums,
// velocity sums, mean offsets), for up to HOP_NOALLOC_MAX_GROUPS groups.
// Each GPU the library runs on holds its own copy until the process ends;
// host code uses the address hipGetSymbolAddress gives on that device
// (hop_ctx.noalloc_scratch), never the array's name.
static __device__ __align__(256) unsigned long long scratch[(size_t)HOP_NOALLOC_MAX_GROUPS * 9];

}  // namespace

int hop_noalloc_init(hop_ctx *ctx)
{
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return hop_fail(ctx, HOP_ERR_HIP, "hipGetSymbolAddress of the static statistics scratch failed");
    }
    ctx->noalloc_scratch = ptr;
    return HOP_OK;
}

extern "C" int hop_halo_stats(hop_ctx *ctx, int64_t n, const uint32_t *pos, const float *vel,
                              const int32_t *group, int32_t n_groups, const hop_group_info *groups,
                              const hop_params *p, double *com, double *rmax, double *vbulk,
                              void *stream)
{
    if (!ctx) return HOP_ERR_ARG;
    ctx->err.clear();
    HOPTRY(stats_args(ctx, n, pos, vel, group, n_groups, groups, p, com, rmax, vbulk));
    HOPTRY(hop_set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    if (n_groups == 0) return HOP_OK;
    const size_t g3 = (size_t)n_groups * 3;
    HOPTRY(hop_reserve(ctx, ctx->work_e, g3 * 8 * 3));  // offset sums, velocity sums, mean offsets
    unsigned long long *osum = (unsigned long long *)ctx->work_e.ptr;
    double *vsum = (double *)(osum + g3);
    double *mean = vsum + g3;
    HOPTRY(stats_launch(ctx, n, pos, vel, group, n_groups, groups, p, com, rmax, vbulk, osum, vsum, mean, s));
    return hop_check_device(ctx, s, "hop_halo_stats");
}

extern "C" int hop_halo_stats_noalloc(hop_ctx *ctx, int64_t n, const uint32_t *pos, const float *vel,
                                      const int32_t *group, int32_t n_groups,
                                      const hop_group_info *groups, const hop_params *p, double *com,
                                      double *rmax, double *vbulk, void *stream)
{
    if (!ctx) return HOP_ERR_ARG;
    ctx->err.clear();
    HOPTRY(stats_args(ctx, n, pos, vel, group, n_groups, groups, p, com, rmax, vbulk));
    if (n_groups > HOP_NOALLOC_MAX_GROUPS)
        return hop_fail(ctx, HOP_ERR_ARG, "n_groups exceeds HOP_NOALLOC_MAX_GROUPS (" +
                                              std::to_string(HOP_NOALLOC_MAX_GROUPS) + ")");
    if (!ctx->noalloc_scratch) return hop_fail(ctx, HOP_ERR_HIP, "static scratch not set up");
    HOPTRY(hop_set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    if (n_groups == 0) return HOP_OK;
    const size_t g3 = (size_t)n_groups * 3;
    unsigned long long *osum = (unsigned long long *)ctx->noalloc_scratch;
    double *vsum = (double *)(osum + g3);
    double *mean = vsum + g3;
    return stats_launch(ctx, n, pos, vel, group, n_groups, groups, p, com, rmax, vbulk, osum, vsum, mean, s);
}
