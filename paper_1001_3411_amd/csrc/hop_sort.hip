// hop_sort.hip -- device-wide exclusive scan and stable LSD radix sort.
//
// Both are tiled for 64-lane wavefronts: a block is 256 threads (4 waves)
// and owns a tile of 4096 items (16 per lane).  The radix sort ranks the
// items of a tile with wave ballots (an 8-bit digit needs 8 ballots per
// round of 64 items), so every pass is stable without a per-item sort.
#include "hop_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;  // 4096
constexpr int kWaves = kThreads / 64;

__device__ inline uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread; returns the exclusive
// prefix and writes the block total to *total.
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t *lds_wave, uint32_t *total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) lds_wave[w] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kWaves; k++) {
        uint32_t s = lds_wave[k];
        if (k < w) base += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

__global__ __launch_bounds__(kThreads) void k_scan_reduce(const uint32_t *__restrict__ in,
                                                          int64_t n, uint32_t *__restrict__ part)
{
    __shared__ uint32_t lw[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < kItems; r++) {
        int64_t i = base + (int64_t)r * kThreads + threadIdx.x;
        if (i < n) s += in[i];
    }
    uint32_t tot;
    block_excl_scan(s, lw, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Exclusive scan of one tile, adding part[blockIdx.x] (NULL = 0).
__global__ __launch_bounds__(kThreads) void k_scan_tile(uint32_t *__restrict__ data, int64_t n,
                                                        const uint32_t *__restrict__ part,
                                                        uint32_t *__restrict__ total_out)
{
    __shared__ uint32_t tile[kTile + kTile / 32];
    __shared__ uint32_t lw[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
    for (int r = 0; r < kItems; r++) {
        int li = r * kThreads + threadIdx.x;
        int64_t i = base + li;
        tile[li + (li >> 5)] = i < n ? data[i] : 0u;
    }
    __syncthreads();
    uint32_t v[kItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kItems; k++) {
        int li = threadIdx.x * kItems + k;
        v[k] = tile[li + (li >> 5)];
        s += v[k];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan(s, lw, &tot);
    if (part) run += part[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kItems; k++) {
        int li = threadIdx.x * kItems + k;
        tile[li + (li >> 5)] = run;
        run += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kItems; r++) {
        int li = r * kThreads + threadIdx.x;
        int64_t i = base + li;
        if (i < n) data[i] = tile[li + (li >> 5)];
    }
    if (total_out && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        uint32_t last_base = part ? part[blockIdx.x] : 0u;
        *total_out = last_base + tot;
    }
}

int scan_rec(hop_ctx *ctx, uint32_t *data, int64_t n, uint32_t *total_dev, uint32_t *scratch,
             hipStream_t s)
{
    if (n <= 0) {
        if (total_dev) HOPCHK(ctx, hipMemsetAsync(total_dev, 0, sizeof(uint32_t), s));
        return HOP_OK;
    }
    int64_t nb = hop_div_up(n, kTile);
    if (nb == 1) {
        k_scan_tile<<<1, kThreads, 0, s>>>(data, n, nullptr, total_dev);
        HOPCHK(ctx, hipGetLastError());
        return HOP_OK;
    }
    uint32_t *part = scratch;
    k_scan_reduce<<<(int)nb, kThreads, 0, s>>>(data, n, part);
    HOPCHK(ctx, hipGetLastError());
    HOPTRY(scan_rec(ctx, part, nb, nullptr, scratch + nb, s));
    k_scan_tile<<<(int)nb, kThreads, 0, s>>>(data, n, part, total_dev);
    HOPCHK(ctx, hipGetLastError());
    return HOP_OK;
}

// ---------------------------------------------------------------------------
// radix sort
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_radix_hist(const uint64_t *__restrict__ keys,
                                                         int64_t n, int shift, int64_t nblocks,
                                                         uint32_t *__restrict__ hist)
{
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
    for (int r = 0; r < kItems; r++) {
        int64_t i = base + (int64_t)r * kThreads + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(kThreads) void k_radix_scatter(
    const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals, int64_t n, int shift,
    int64_t nblocks, const uint32_t *__restrict__ offs, uint64_t *__restrict__ okeys,
    uint32_t *__restrict__ ovals)
{
    __shared__ uint32_t wcnt[kWaves][256];
    __shared__ uint32_t wbase[kWaves][256];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kWaves; k++) wcnt[k][threadIdx.x] = 0;
    __syncthreads();
    // wave w owns items [base + w*1024, +1024); round r covers 64 consecutive
    const int64_t wbase_i = (int64_t)blockIdx.x * kTile + (int64_t)w * (64 * kItems);
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint64_t key[kItems];
    uint32_t val[kItems];
    uint32_t loc[kItems];
#pragma unroll
    for (int r = 0; r < kItems; r++) {
        int64_t i = wbase_i + r * 64 + lane;
        bool act = i < n;
        key[r] = act ? keys[i] : 0;
        val[r] = act ? vals[i] : 0;
        uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
        uint64_t m = __ballot(act);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            uint64_t bb = __ballot((d >> b) & 1u);
            m &= ((d >> b) & 1u) ? bb : ~bb;
        }
        uint32_t before = wcnt[w][d];
        uint32_t rank = (uint32_t)__popcll(m & lt_mask);
        loc[r] = before + rank;
        __builtin_amdgcn_wave_barrier();
        if (act && (m & lt_mask) == 0) wcnt[w][d] = before + (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    {
        const int d = threadIdx.x;
        uint32_t run = offs[(int64_t)d * nblocks + blockIdx.x];
#pragma unroll
        for (int k = 0; k < kWaves; k++) {
            wbase[k][d] = run;
            run += wcnt[k][d];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kItems; r++) {
        int64_t i = wbase_i + r * 64 + lane;
        if (i < n) {
            uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
            uint32_t dst = wbase[w][d] + loc[r];
            okeys[dst] = key[r];
            ovals[dst] = val[r];
        }
    }
}

}  // namespace

int hop_scan_u32(hop_ctx *ctx, uint32_t *data, int64_t n, uint32_t *total_dev, hipStream_t s)
{
    // partial sums of all recursion levels
    int64_t need = 0, m = n;
    while (m > kTile) {
        m = hop_div_up(m, kTile);
        need += m;
    }
    HOPTRY(hop_reserve(ctx, ctx->scan_tmp, (size_t)(need + 16) * sizeof(uint32_t)));
    return scan_rec(ctx, data, n, total_dev, (uint32_t *)ctx->scan_tmp.ptr, s);
}

int hop_radix_sort(hop_ctx *ctx, uint64_t *keys, uint32_t *vals, uint64_t *tkeys, uint32_t *tvals,
                   int64_t n, int bits, hipStream_t s, int lo_bit)
{
    if (n <= 1 || bits <= lo_bit) return HOP_OK;
    const int64_t nb = hop_div_up(n, kTile);
    if (nb * 256 >= (int64_t)1 << 31) return hop_fail(ctx, HOP_ERR_ARG, "radix sort too large");
    DevBuf &hb = ctx->work_f;
    HOPTRY(hop_reserve(ctx, hb, (size_t)nb * 256 * sizeof(uint32_t)));
    uint32_t *hist = (uint32_t *)hb.ptr;
    uint64_t *ka = keys, *kb = tkeys;
    uint32_t *va = vals, *vb = tvals;
    int passes = 0;
    for (int shift = lo_bit; shift < bits; shift += 8, passes++) {
        k_radix_hist<<<(int)nb, kThreads, 0, s>>>(ka, n, shift, nb, hist);
        HOPCHK(ctx, hipGetLastError());
        HOPTRY(hop_scan_u32(ctx, hist, nb * 256, nullptr, s));
        k_radix_scatter<<<(int)nb, kThreads, 0, s>>>(ka, va, n, shift, nb, hist, kb, vb);
        HOPCHK(ctx, hipGetLastError());
        uint64_t *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
    if (passes & 1) {
        HOPCHK(ctx, hipMemcpyAsync(keys, ka, (size_t)n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        HOPCHK(ctx, hipMemcpyAsync(vals, va, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    }
    return HOP_OK;
}
