// hop_radius.hip -- the learned search radius: cell counts, the 27 features
// and the target of each particle, the 27-64-64-1 network's training in
// FP32 (forward, backward, Adam) and its BF16 inference per cell.
//
// The paper searches a fixed number of neighbours per particle and names
// the neighbour search as the cost that dominates (its sections 2 and 5);
// predicting each particle's search radius from its surroundings is this
// project's addition.  The kNN kernel uses the prediction only to prune:
// a particle whose N_dens-1 nearest others all lie within the predicted
// radius has its exact list; any other particle is searched again without
// the radius, so results never depend on the model.
//
// Features: f_k = log(1 + n_k) for the cells (cz+dz, cy+dy, cx+dx) around
// the particle's cell, dz outermost, each of dz, dy, dx in -1, 0, 1
// (periodic wrap, or 0 outside a non-periodic box).  Target: log(r / side)
// with r the distance to the particle's last listed neighbour.
//
// Parameters, one flat FP32 vector of 6017: W1 [27][64] (input-major), b1,
// W2 [64][64], b2, W3 [64], b3.
#include <cmath>

#include "hop_internal.h"

namespace {

constexpr int NI = 27, NH = 64;
constexpr int O_B1 = NI * NH;
constexpr int O_W2 = O_B1 + NH;
constexpr int O_B2 = O_W2 + NH * NH;
constexpr int O_W3 = O_B2 + NH;
constexpr int O_B3 = O_W3 + NH;
constexpr int NP = O_B3 + 1;  // 6017
static_assert(NP == HOP_MLP_PARAMS, "parameter count");

constexpr int kTile = 64;      // samples per training workgroup
constexpr int kTileThreads = 256;

__device__ __forceinline__ int64_t cell_index(uint32_t x, uint32_t y, uint32_t z, int cb, int gb)
{
    return ((int64_t)(z >> cb) << (2 * gb)) | ((int64_t)(y >> cb) << gb) | (int64_t)(x >> cb);
}

__global__ void k_cell_count(int64_t n, const uint32_t *__restrict__ pos, uint32_t glim, int cb, int gb,
                             uint32_t *__restrict__ counts, uint32_t *__restrict__ dflags)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    if (x >= glim || y >= glim || z >= glim) {
        atomicOr(dflags, DERR_RANGE);
        return;
    }
    atomicAdd(&counts[cell_index(x, y, z, cb, gb)], 1u);
}

// the 27 features of cell (cx, cy, cz)
__device__ __forceinline__ void cell_features(const uint32_t *__restrict__ counts, int cx, int cy, int cz,
                                              int gb, int periodic, float f[NI])
{
    const int g = 1 << gb, m = g - 1;
    int k = 0;
#pragma unroll
    for (int dz = -1; dz <= 1; dz++)
#pragma unroll
        for (int dy = -1; dy <= 1; dy++)
#pragma unroll
            for (int dx = -1; dx <= 1; dx++) {
                int x = cx + dx, y = cy + dy, z = cz + dz;
                uint32_t c = 0;
                if (periodic) {
                    c = counts[((int64_t)(z & m) << (2 * gb)) | ((int64_t)(y & m) << gb) | (x & m)];
                } else if (x >= 0 && x < g && y >= 0 && y < g && z >= 0 && z < g) {
                    c = counts[((int64_t)z << (2 * gb)) | ((int64_t)y << gb) | x];
                }
                f[k++] = log1pf((float)c);
            }
}

__global__ void k_features(int64_t n, const uint32_t *__restrict__ pos, const uint32_t *__restrict__ counts,
                           int cb, int gb, int periodic, float *__restrict__ feats)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float f[NI];
    cell_features(counts, (int)(pos[3 * i] >> cb), (int)(pos[3 * i + 1] >> cb), (int)(pos[3 * i + 2] >> cb),
                  gb, periodic, f);
#pragma unroll
    for (int k = 0; k < NI; k++) feats[i * NI + k] = f[k];
}

__device__ __forceinline__ int64_t axis_d(uint32_t a, uint32_t b, uint32_t glim, int periodic)
{
    int64_t d = a > b ? (int64_t)(a - b) : (int64_t)(b - a);
    if (periodic && d > (int64_t)glim - d) d = (int64_t)glim - d;
    return d;
}

__global__ void k_targets(int64_t n, const uint32_t *__restrict__ pos, const int32_t *__restrict__ nbr,
                          int k_store, int col, uint32_t glim, int periodic, int cb,
                          float *__restrict__ target, uint32_t *__restrict__ dflags)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t j = nbr[i * k_store + col];
    if (j < 0 || j >= n) {
        atomicOr(dflags, DERR_INDEX);
        target[i] = 0.0f;
        return;
    }
    const int64_t dx = axis_d(pos[3 * i], pos[3 * (int64_t)j], glim, periodic);
    const int64_t dy = axis_d(pos[3 * i + 1], pos[3 * (int64_t)j + 1], glim, periodic);
    const int64_t dz = axis_d(pos[3 * i + 2], pos[3 * (int64_t)j + 2], glim, periodic);
    const int64_t d2 = dx * dx + dy * dy + dz * dz;
    if (d2 == 0) atomicOr(dflags, DERR_DEGENERATE);
    target[i] = (float)(0.5 * log((double)(d2 > 0 ? d2 : 1)) - (double)cb * 0.69314718055994530942);
}

// One training tile: forward and backward of up to 64 samples, their
// gradient sum written to part[tile][NP] and their squared-error sum to
// lpart[tile].  Samples past `rows` contribute nothing.
__global__ __launch_bounds__(kTileThreads) void k_mlp_tile(const float *__restrict__ feats,
                                                           const float *__restrict__ target,
                                                           const int32_t *__restrict__ idx, int64_t rows,
                                                           int64_t n_samples, float inv_b,
                                                           const float *__restrict__ w,
                                                           float *__restrict__ part,
                                                           float *__restrict__ lpart,
                                                           uint32_t *__restrict__ dflags)
{
    __shared__ float sw[NP];
    __shared__ float X[kTile][NI + 1];
    __shared__ float H1[kTile][NH + 1];
    __shared__ float H2[kTile][NH + 1];
    __shared__ float D1[kTile][NH + 1];
    __shared__ float D2[kTile][NH + 1];
    __shared__ float dy[kTile];
    __shared__ float se[kTile];
    const int tid = threadIdx.x;
    const int64_t s0 = (int64_t)blockIdx.x * kTile;

    for (int q = tid; q < NP; q += kTileThreads) sw[q] = w[q];
    for (int e = tid; e < kTile * NI; e += kTileThreads) {
        const int s = e / NI, k = e - s * NI;
        float v = 0.0f;
        if (s0 + s < rows) {
            int64_t r = idx ? (int64_t)idx[s0 + s] : s0 + s;
            if (r < 0 || r >= n_samples) {
                atomicOr(dflags, DERR_INDEX);
                r = 0;
            }
            v = feats[r * NI + k];
        }
        X[s][k] = v;
    }
    __syncthreads();
    for (int e = tid; e < kTile * NH; e += kTileThreads) {
        const int s = e >> 6, j = e & 63;
        float a = sw[O_B1 + j];
        for (int k = 0; k < NI; k++) a += X[s][k] * sw[k * NH + j];
        H1[s][j] = a > 0.0f ? a : 0.0f;
    }
    __syncthreads();
    for (int e = tid; e < kTile * NH; e += kTileThreads) {
        const int s = e >> 6, j = e & 63;
        float a = sw[O_B2 + j];
        for (int k = 0; k < NH; k++) a += H1[s][k] * sw[O_W2 + k * NH + j];
        H2[s][j] = a > 0.0f ? a : 0.0f;
    }
    __syncthreads();
    if (tid < kTile) {
        const int s = tid;
        float y = sw[O_B3];
        for (int j = 0; j < NH; j++) y += H2[s][j] * sw[O_W3 + j];
        bool valid = s0 + s < rows;
        float t = 0.0f;
        if (valid) {
            int64_t r = idx ? (int64_t)idx[s0 + s] : s0 + s;
            if (r < 0 || r >= n_samples) r = 0;
            t = target[r];
        }
        const float res = y - t;
        dy[s] = valid ? 2.0f * res * inv_b : 0.0f;
        se[s] = valid ? res * res : 0.0f;
    }
    __syncthreads();
    for (int e = tid; e < kTile * NH; e += kTileThreads) {
        const int s = e >> 6, j = e & 63;
        D2[s][j] = H2[s][j] > 0.0f ? dy[s] * sw[O_W3 + j] : 0.0f;
    }
    __syncthreads();
    for (int e = tid; e < kTile * NH; e += kTileThreads) {
        const int s = e >> 6, k = e & 63;
        float a = 0.0f;
        for (int j = 0; j < NH; j++) a += D2[s][j] * sw[O_W2 + k * NH + j];
        D1[s][k] = H1[s][k] > 0.0f ? a : 0.0f;
    }
    __syncthreads();
    float *out = part + (int64_t)blockIdx.x * NP;
    for (int q = tid; q < NP; q += kTileThreads) {
        float g = 0.0f;
        if (q < O_B1) {
            const int k = q >> 6, j = q & 63;
            for (int s = 0; s < kTile; s++) g += X[s][k] * D1[s][j];
        } else if (q < O_W2) {
            const int j = q - O_B1;
            for (int s = 0; s < kTile; s++) g += D1[s][j];
        } else if (q < O_B2) {
            const int k = (q - O_W2) >> 6, j = (q - O_W2) & 63;
            for (int s = 0; s < kTile; s++) g += H1[s][k] * D2[s][j];
        } else if (q < O_W3) {
            const int j = q - O_B2;
            for (int s = 0; s < kTile; s++) g += D2[s][j];
        } else if (q < O_B3) {
            const int j = q - O_W3;
            for (int s = 0; s < kTile; s++) g += H2[s][j] * dy[s];
        } else {
            for (int s = 0; s < kTile; s++) g += dy[s];
        }
        out[q] = g;
    }
    if (tid == 0) {
        float l = 0.0f;
        for (int s = 0; s < kTile; s++) l += se[s];
        lpart[blockIdx.x] = l;
    }
}

// Sum of the tile partials in tile order (deterministic), then optionally
// one Adam step; thread NP writes the mean loss.
__global__ void k_mlp_reduce(int n_tiles, const float *__restrict__ part, const float *__restrict__ lpart,
                             float inv_b, float *__restrict__ grad, float *__restrict__ loss,
                             int adam, float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                             float lr, float beta1, float beta2, float eps, float bc1, float bc2)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < NP) {
        float g = 0.0f;
        for (int t = 0; t < n_tiles; t++) g += part[(int64_t)t * NP + q];
        if (grad) grad[q] = g;
        if (adam) {
            const float mq = beta1 * m[q] + (1.0f - beta1) * g;
            const float vq = beta2 * v[q] + (1.0f - beta2) * g * g;
            m[q] = mq;
            v[q] = vq;
            const float mh = mq / bc1, vh = vq / bc2;
            w[q] = w[q] - lr * mh / (sqrtf(vh) + eps);
        }
    } else if (q == NP && loss) {
        float l = 0.0f;
        for (int t = 0; t < n_tiles; t++) l += lpart[t];
        *loss = l * inv_b;
    }
}

// Round to nearest even BF16 (NaN kept quiet).
__device__ __forceinline__ uint16_t to_bf16(float x)
{
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__global__ void k_to_bf16(const float *__restrict__ w, uint16_t *__restrict__ out)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < NP) out[q] = to_bf16(w[q]);
}

// The network with BF16 weights (already widened into sw) and FP32
// accumulation; f are the 27 features.
__device__ __forceinline__ float mlp_infer(const float *sw, const float f[NI])
{
    float h1[NH];
#pragma unroll
    for (int j = 0; j < NH; j++) h1[j] = sw[O_B1 + j];
    for (int k = 0; k < NI; k++) {
        const float x = f[k];
#pragma unroll
        for (int j = 0; j < NH; j++) h1[j] += x * sw[k * NH + j];
    }
#pragma unroll
    for (int j = 0; j < NH; j++) h1[j] = h1[j] > 0.0f ? h1[j] : 0.0f;
    float y = sw[O_B3];
    for (int j = 0; j < NH; j++) {
        float a = sw[O_B2 + j];
#pragma unroll
        for (int k = 0; k < NH; k++) a += h1[k] * sw[O_W2 + k * NH + j];
        y += (a > 0.0f ? a : 0.0f) * sw[O_W3 + j];
    }
    return y;
}

// log(r / side) from the uniform-density estimate of the 27 cells: the
// radius whose ball holds n_dens particles at density N27 / (27 side^3)
__device__ __forceinline__ float analytic_predict(float n27, int n_dens)
{
    const float nn = n27 > 1.0f ? n27 : 1.0f;
    return (1.0f / 3.0f) * logf(81.0f * (float)n_dens / (4.0f * 3.14159265f * nn));
}

__global__ __launch_bounds__(256) void k_radius_predict(int64_t rows, const float *__restrict__ feats, int kind,
                                                        const uint16_t *__restrict__ wbf, int n_dens,
                                                        float *__restrict__ out)
{
    __shared__ float sw[NP];
    if (kind == HOP_RADIUS_MLP)
        for (int q = threadIdx.x; q < NP; q += blockDim.x) sw[q] = from_bf16(wbf[q]);
    __syncthreads();
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    float f[NI];
#pragma unroll
    for (int k = 0; k < NI; k++) f[k] = feats[r * NI + k];
    if (kind == HOP_RADIUS_MLP) {
        out[r] = mlp_infer(sw, f);
    } else {
        float n27 = 0.0f;
#pragma unroll
        for (int k = 0; k < NI; k++) n27 += rintf(expm1f(f[k]));
        out[r] = analytic_predict(n27, n_dens);
    }
}

// search radius of every cell: side * exp(prediction + margin)
__global__ __launch_bounds__(256) void k_cell_radius(int64_t n_cells, const uint32_t *__restrict__ counts,
                                                     int gb, int periodic, int kind,
                                                     const uint16_t *__restrict__ wbf, int n_dens,
                                                     float margin, float side, float *__restrict__ cell_r)
{
    __shared__ float sw[NP];
    if (kind == HOP_RADIUS_MLP)
        for (int q = threadIdx.x; q < NP; q += blockDim.x) sw[q] = from_bf16(wbf[q]);
    __syncthreads();
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    const int m = (1 << gb) - 1;
    const int cx = (int)(c & m), cy = (int)((c >> gb) & m), cz = (int)(c >> (2 * gb));
    float y;
    if (kind == HOP_RADIUS_MLP) {
        float f[NI];
        cell_features(counts, cx, cy, cz, gb, periodic, f);
        y = mlp_infer(sw, f);
    } else {
        float f[NI];
        cell_features(counts, cx, cy, cz, gb, periodic, f);
        float n27 = 0.0f;
#pragma unroll
        for (int k = 0; k < NI; k++) n27 += rintf(expm1f(f[k]));
        y = analytic_predict(n27, n_dens);
    }
    cell_r[c] = side * expf(y + margin);
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

int hop_cell_bits(const hop_ctx *ctx, int64_t n, const hop_params *p)
{
    return hop_radius_cell_bits(n, p->grid_bits, ctx->radius_occupancy);
}

static int count_cells(hop_ctx *ctx, int64_t n, const uint32_t *pos, const hop_params *p, int cb,
                       hipStream_t s)
{
    const int gb = (int)p->grid_bits - cb;
    const int64_t cells = (int64_t)1 << (3 * gb);
    HOPTRY(hop_reserve(ctx, ctx->cell_counts, (size_t)cells * 4));
    HOPCHK(ctx, hipMemsetAsync(ctx->cell_counts.ptr, 0, (size_t)cells * 4, s));
    k_cell_count<<<hop_grid(n, 256), 256, 0, s>>>(n, pos, 1u << p->grid_bits, cb, gb,
                                                 (uint32_t *)ctx->cell_counts.ptr, (uint32_t *)ctx->flags.ptr);
    HOPCHK(ctx, hipGetLastError());
    return HOP_OK;
}

int hop_radius_cells(hop_ctx *ctx, int64_t n, const uint32_t *pos, const hop_params *p, hipStream_t s,
                     const float **cell_r, int *cb_out, int *gb_out)
{
    if (ctx->radius_kind == 0) return hop_fail(ctx, HOP_ERR_ARG, "HOP_LEARNED_RADIUS needs a loaded radius model");
    const int cb = hop_cell_bits(ctx, n, p);
    const int gb = (int)p->grid_bits - cb;
    HOPTRY(count_cells(ctx, n, pos, p, cb, s));
    const int64_t cells = (int64_t)1 << (3 * gb);
    HOPTRY(hop_reserve(ctx, ctx->cell_r, (size_t)cells * 4));
    k_cell_radius<<<hop_grid(cells, 256), 256, 0, s>>>(cells, (const uint32_t *)ctx->cell_counts.ptr, gb,
                                                       (p->flags & HOP_PERIODIC) ? 1 : 0, ctx->radius_kind,
                                                       (const uint16_t *)ctx->radius_w.ptr, p->n_dens,
                                                       ctx->radius_margin, (float)std::ldexp(1.0, cb),
                                                       (float *)ctx->cell_r.ptr);
    HOPCHK(ctx, hipGetLastError());
    *cell_r = (const float *)ctx->cell_r.ptr;
    *cb_out = cb;
    *gb_out = gb;
    return HOP_OK;
}

extern "C" {

int hop_radius_cell_bits(int64_t n, uint32_t grid_bits, float occupancy)
{
    // cells of side 2^cb holding `occupancy` particles on average
    if (n < 1 || grid_bits < 1 || grid_bits > 21 || !(occupancy >= 1.0f)) return -1;
    const double per_axis = std::cbrt((double)n / (double)occupancy);
    int gb = (int)std::lround(std::log2(per_axis > 1.0 ? per_axis : 1.0));
    if (gb < 1) gb = 1;
    if (gb > 9) gb = 9;  // at most 2^27 cells
    if (gb > (int)grid_bits) gb = (int)grid_bits;
    return (int)grid_bits - gb;
}

int hop_radius_dataset(hop_ctx *ctx, int64_t n, const uint32_t *pos, const int32_t *nbr,
                       const hop_params *p, int32_t cell_bits, float *feats, float *target, void *stream)
{
    if (!ctx) return HOP_ERR_ARG;
    ctx->err.clear();
    HOPTRY(hop_check_params(ctx, n, p));
    if (!pos || !feats || (target && !nbr))
        return hop_fail(ctx, HOP_ERR_ARG, "pos and feats must be non-NULL, and nbr when target is asked for");
    if (cell_bits < 0 || cell_bits >= (int)p->grid_bits || (int)p->grid_bits - cell_bits > 9)
        return hop_fail(ctx, HOP_ERR_ARG, "need 0 <= cell_bits < grid_bits with at most 2^9 cells per axis");
    if (target && p->k_store < p->n_dens)
        return hop_fail(ctx, HOP_ERR_ARG, "the target needs k_store = n_dens (the last neighbour)");
    HOPTRY(hop_set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    const int gb = (int)p->grid_bits - cell_bits;
    HOPTRY(count_cells(ctx, n, pos, p, cell_bits, s));
    k_features<<<hop_grid(n, 256), 256, 0, s>>>(n, pos, (const uint32_t *)ctx->cell_counts.ptr, cell_bits, gb,
                                               (p->flags & HOP_PERIODIC) ? 1 : 0, feats);
    HOPCHK(ctx, hipGetLastError());
    if (target) {
        k_targets<<<hop_grid(n, 256), 256, 0, s>>>(n, pos, nbr, p->k_store, p->n_dens - 1, 1u << p->grid_bits,
                                                  (p->flags & HOP_PERIODIC) ? 1 : 0, cell_bits, target,
                                                  (uint32_t *)ctx->flags.ptr);
        HOPCHK(ctx, hipGetLastError());
    }
    return hop_check_device(ctx, s, "hop_radius_dataset");
}

static int mlp_steps(hop_ctx *ctx, int64_t n_samples, const float *feats, const float *target,
                     const int32_t *idx, int32_t steps, int32_t batch, int adam, int32_t first_step,
                     float lr, float beta1, float beta2, float eps, float *w, float *m, float *v,
                     float *grad, float *loss, hipStream_t s)
{
    const int64_t tiles = hop_div_up(batch, kTile);
    HOPTRY(hop_reserve(ctx, ctx->mlp_part, (size_t)(tiles * NP + tiles) * 4));
    float *part = (float *)ctx->mlp_part.ptr;
    float *lpart = part + tiles * NP;
    const float inv_b = 1.0f / (float)batch;
    for (int32_t st = 0; st < steps; st++) {
        const int32_t *ix = idx ? idx + (int64_t)st * batch : nullptr;
        k_mlp_tile<<<(int)tiles, kTileThreads, 0, s>>>(feats, target, ix, batch, n_samples, inv_b, w, part, lpart,
                                                        (uint32_t *)ctx->flags.ptr);
        HOPCHK(ctx, hipGetLastError());
        const double t = (double)first_step + st;
        const float bc1 = (float)(1.0 - std::pow((double)beta1, t));
        const float bc2 = (float)(1.0 - std::pow((double)beta2, t));
        k_mlp_reduce<<<hop_grid(NP + 1, 256), 256, 0, s>>>((int)tiles, part, lpart, inv_b, grad,
                                                           loss ? loss + st : nullptr, adam, w, m, v, lr,
                                                           beta1, beta2, eps, bc1, bc2);
        HOPCHK(ctx, hipGetLastError());
    }
    return HOP_OK;
}

int hop_mlp_grad(hop_ctx *ctx, int64_t n_samples, const float *feats, const float *target,
                 const int32_t *idx, int32_t batch, const float *w, float *grad, float *loss, void *stream)
{
    if (!ctx) return HOP_ERR_ARG;
    ctx->err.clear();
    if (!feats || !target || !w || !grad) return hop_fail(ctx, HOP_ERR_ARG, "feats, target, w and grad must be non-NULL");
    if (batch < 1 || batch > (1 << 24) || n_samples < 1 || (!idx && batch > n_samples))
        return hop_fail(ctx, HOP_ERR_ARG, "need 1 <= batch <= 2^24 rows within the samples");
    HOPTRY(hop_set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    HOPTRY(mlp_steps(ctx, n_samples, feats, target, idx, 1, batch, 0, 1, 0.f, 0.f, 0.f, 0.f, (float *)w, nullptr,
                     nullptr, grad, loss, s));
    return hop_check_device(ctx, s, "hop_mlp_grad");
}

int hop_mlp_train(hop_ctx *ctx, int64_t n_samples, const float *feats, const float *target,
                  const int32_t *idx, int32_t steps, int32_t batch, int32_t first_step, float lr,
                  float beta1, float beta2, float eps, float *w, float *m, float *v, float *loss, void *stream)
{
    if (!ctx) return HOP_ERR_ARG;
    ctx->err.clear();
    if (!feats || !target || !w || !m || !v) return hop_fail(ctx, HOP_ERR_ARG, "feats, target, w, m and v must be non-NULL");
    if (steps < 0 || batch < 1 || batch > (1 << 24) || first_step < 1 || n_samples < 1 ||
        (!idx && batch > n_samples))
        return hop_fail(ctx, HOP_ERR_ARG, "need steps >= 0, 1 <= batch <= 2^24, first_step >= 1");
    if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return hop_fail(ctx, HOP_ERR_ARG, "bad Adam constants");
    HOPTRY(hop_set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    HOPTRY(mlp_steps(ctx, n_samples, feats, target, idx, steps, batch, 1, first_step, lr, beta1, beta2, eps, w, m,
                     v, nullptr, loss, s));
    return hop_check_device(ctx, s, "hop_mlp_train");
}

int hop_radius_load(hop_ctx *ctx, int32_t kind, const float *w, float margin, float occupancy, void *stream)
{
    if (!ctx) return HOP_ERR_ARG;
    ctx->err.clear();
    if (kind != HOP_RADIUS_MLP && kind != HOP_RADIUS_ANALYTIC && kind != 0)
        return hop_fail(ctx, HOP_ERR_ARG, "unknown radius model kind");
    if (kind == HOP_RADIUS_MLP && !w) return hop_fail(ctx, HOP_ERR_ARG, "the MLP needs its weights");
    if (!std::isfinite(margin) || !(occupancy >= 1.0f && occupancy <= 4096.0f))
        return hop_fail(ctx, HOP_ERR_ARG, "margin must be finite and occupancy in [1, 4096]");
    HOPTRY(hop_set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    if (kind == HOP_RADIUS_MLP) {
        HOPTRY(hop_reserve(ctx, ctx->radius_w, NP * 2));
        k_to_bf16<<<hop_grid(NP, 256), 256, 0, s>>>(w, (uint16_t *)ctx->radius_w.ptr);
        HOPCHK(ctx, hipGetLastError());
    }
    ctx->radius_kind = kind;
    ctx->radius_margin = margin;
    ctx->radius_occupancy = occupancy;
    return hop_check_device(ctx, s, "hop_radius_load");
}

int hop_radius_predict(hop_ctx *ctx, int64_t rows, const float *feats, int32_t n_dens, float *out, void *stream)
{
    if (!ctx) return HOP_ERR_ARG;
    ctx->err.clear();
    if (ctx->radius_kind == 0) return hop_fail(ctx, HOP_ERR_ARG, "no radius model loaded");
    if (!feats || !out || rows < 0 || n_dens < 2 || n_dens > 64) return hop_fail(ctx, HOP_ERR_ARG, "bad arguments");
    HOPTRY(hop_set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    if (rows > 0) {
        k_radius_predict<<<hop_grid(rows, 256), 256, 0, s>>>(rows, feats, ctx->radius_kind,
                                                             (const uint16_t *)ctx->radius_w.ptr, n_dens, out);
        HOPCHK(ctx, hipGetLastError());
    }
    return hop_check_device(ctx, s, "hop_radius_predict");
}

}  // extern "C"
