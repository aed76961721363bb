// hop_merge.hip -- chain boundaries, merge and group labels (the paper's
// section 2, merge steps 2-5, and the output rules of section 3.1).
//
// Boundaries.  Every chained particle offers its n_merge-1 nearest others
// that sit in a different chain; the boundary density 0.5*(d_i + d_j) of the
// chain pair is kept by a 64-bit atomic max in an open-addressing hash
// table keyed by (lo << 32 | hi).  Boundary densities are >= 0, so their
// IEEE bit patterns order like the values and the max runs on the bits.
//
// Merge.  Proto-halos (peak >= delta_peak) all start in the component of a
// virtual root; Boruvka rounds then build the maximum spanning forest of
// the chain graph under the strict order (s desc, lo asc, hi asc): every
// component picks its best outgoing boundary (an atomic max on s, then an
// atomic min on the pair key among equal s) and hooks to the other side.
// That forest is unique, and in it every sub-peak chain reaches a proto-halo
// through its densest chain of boundaries, or reaches none.  Halos are the
// connected pieces of forest edges plus the proto-halo pairs with a
// boundary >= delta_saddle, found with a lock-free union-find whose roots
// are the smallest chain of each piece.
//
// Labels.  Halo sizes and peaks by atomics, then three stable radix sorts
// order the halos by (count desc, peak density desc, peak tie key asc).
#include "hop_internal.h"

#include <algorithm>

namespace {

constexpr uint64_t kEmpty = ~0ull;

__device__ __forceinline__ uint64_t pair_hash(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

// Per chain: its root and peak density, and the number of its members that
// count towards a halo (padded particles do not under the padded rules).
__global__ void k_chain_table(int64_t n, const int32_t *__restrict__ root,
                              const int32_t *__restrict__ chain_of, const double *__restrict__ dens,
                              const uint8_t *__restrict__ padded, int padded_rules, int32_t C,
                              int32_t *__restrict__ croot, double *__restrict__ cpeak,
                              uint32_t *__restrict__ ccount, uint32_t *__restrict__ dflags)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t c = chain_of[i];
    if (c < -1 || c >= C) {
        atomicOr(dflags, DERR_INDEX);
        return;
    }
    int32_t r = root[i];
    if (r < 0 || r >= n) {
        atomicOr(dflags, DERR_INDEX);
        return;
    }
    if (c < 0) return;
    if (r == (int32_t)i) {
        croot[c] = (int32_t)i;
        cpeak[c] = dens[i];
    }
    if (!(padded_rules && padded && padded[i])) atomicAdd(&ccount[c], 1u);
}

__global__ void k_saddle_insert(int64_t n, const int32_t *__restrict__ nbr, int k_store,
                                int n_merge, const double *__restrict__ dens,
                                const int32_t *__restrict__ chain_of,
                                const uint8_t *__restrict__ padded, int padded_rules, int32_t C,
                                uint64_t *__restrict__ hkeys, unsigned long long *__restrict__ hvals,
                                uint64_t mask, int log2cap, uint32_t *__restrict__ dflags)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t ci = chain_of[i];
    if (ci < 0 || ci >= C) return;
    const bool pi = padded_rules && padded && padded[i];
    const double di = dens[i];
    for (int t = 1; t < n_merge; t++) {
        const int32_t j = nbr[i * k_store + t];
        if (j < 0 || j >= n) {
            atomicOr(dflags, DERR_INDEX);
            continue;
        }
        const int32_t cj = chain_of[j];
        if (cj < 0 || cj >= C || cj == ci) continue;
        if (pi && padded[j]) continue;
        const double sv = (di + dens[j]) * 0.5;
        const unsigned long long sb = (unsigned long long)__double_as_longlong(sv);
        const uint64_t key = ((uint64_t)(uint32_t)min(ci, cj) << 32) | (uint32_t)max(ci, cj);
        uint64_t slot = log2cap > 0 ? pair_hash(key) >> (64 - log2cap) : 0;
        bool done = false;
        for (uint64_t probe = 0; probe <= mask; probe++) {
            uint64_t k = hkeys[slot];
            if (k == kEmpty) {
                k = atomicCAS((unsigned long long *)&hkeys[slot], (unsigned long long)kEmpty,
                              (unsigned long long)key);
                if (k == kEmpty) k = key;
            }
            if (k == key) {
                atomicMax(&hvals[slot], sb);
                done = true;
                break;
            }
            slot = (slot + 1) & mask;
        }
        if (!done) atomicOr(dflags, DERR_CAPACITY);
    }
}

// Compaction of the boundary hash (the order of the compacted edges is
// immaterial: the merge orders edges by saddle density and key itself).
// Atomics on one counter serialise in the L2, so each wave takes a run of
// kCompactRounds * 64 consecutive slots: it counts its kept slots, takes
// its output range with one atomic, then writes them.
constexpr int kCompactRounds = 64;

template <typename Keep, typename Emit>
__device__ __forceinline__ void wave_compact(int64_t cap, uint32_t *count, Keep keep, Emit emit)
{
    const int lane = (int)(threadIdx.x & 63);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t first = wave * 64 * kCompactRounds;
    const uint64_t lt = (1ull << lane) - 1ull;
    uint32_t total = 0;
    for (int r = 0; r < kCompactRounds; r++) {
        const int64_t t = first + (int64_t)r * 64 + lane;
        total += (uint32_t)__popcll(__ballot(t < cap && keep(t)));
    }
    uint32_t base = 0;
    if (lane == 0 && total != 0) base = atomicAdd(count, total);
    base = (uint32_t)__shfl((int)base, 0);
    for (int r = 0; r < kCompactRounds; r++) {
        const int64_t t = first + (int64_t)r * 64 + lane;
        const bool k = t < cap && keep(t);
        const uint64_t m = __ballot(k);
        if (k) emit(t, base + (uint32_t)__popcll(m & lt));
        base += (uint32_t)__popcll(m);
    }
}

static inline int compact_grid(int64_t cap)
{
    return hop_grid(hop_div_up(cap, kCompactRounds), 256);
}

__global__ void k_edge_compact(int64_t cap, const uint64_t *__restrict__ hkeys,
                               const unsigned long long *__restrict__ hvals,
                               int32_t *__restrict__ elo, int32_t *__restrict__ ehi,
                               uint64_t *__restrict__ es, uint32_t *__restrict__ count)
{
    wave_compact(
        cap, count, [&](int64_t t) { return hkeys[t] != kEmpty; },
        [&](int64_t t, uint32_t at) {
            const uint64_t k = hkeys[t];
            elo[at] = (int32_t)(k >> 32);
            ehi[at] = (int32_t)(k & 0xffffffffu);
            es[at] = hvals[t];
        });
}

__global__ void k_bor_init(int32_t C, const double *__restrict__ cpeak, double delta_peak,
                           int32_t *__restrict__ par)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c > C) return;
    par[c] = (c < C && cpeak[c] >= delta_peak) ? C : (int32_t)c;
}

__global__ void k_bor_reset(int32_t C, unsigned long long *__restrict__ bs,
                            unsigned long long *__restrict__ bk)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c > C) return;
    bs[c] = 0ull;
    bk[c] = ~0ull;
}

__global__ void k_bor_best_s(int64_t E, const int32_t *__restrict__ elo,
                             const int32_t *__restrict__ ehi, const uint64_t *__restrict__ es,
                             const int32_t *__restrict__ par, unsigned long long *__restrict__ bs)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    int32_t A = par[elo[e]], B = par[ehi[e]];
    if (A == B) return;
    atomicMax(&bs[A], (unsigned long long)es[e]);
    atomicMax(&bs[B], (unsigned long long)es[e]);
}

__global__ void k_bor_best_k(int64_t E, const int32_t *__restrict__ elo,
                             const int32_t *__restrict__ ehi, const uint64_t *__restrict__ es,
                             const int32_t *__restrict__ par,
                             const unsigned long long *__restrict__ bs,
                             unsigned long long *__restrict__ bk)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    int32_t A = par[elo[e]], B = par[ehi[e]];
    if (A == B) return;
    unsigned long long key = ((unsigned long long)(uint32_t)elo[e] << 32) | (uint32_t)ehi[e];
    if (es[e] == bs[A]) atomicMin(&bk[A], key);
    if (es[e] == bs[B]) atomicMin(&bk[B], key);
}

// Every root component with a best boundary hooks to the other side, except
// the smaller-numbered side of a mutual pick.  Hooks go to tgt (applied by
// k_bor_apply) so that par stays unchanged while this kernel reads it.
__global__ void k_bor_hook(int32_t C, const int32_t *__restrict__ par,
                           const unsigned long long *__restrict__ bk, int32_t *__restrict__ tgt,
                           int32_t *__restrict__ msf_lo, int32_t *__restrict__ msf_hi,
                           uint32_t *__restrict__ counters)
{
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x > C) return;
    tgt[x] = par[x];
    if (par[x] != (int32_t)x) return;
    unsigned long long k = bk[x];
    if (k == ~0ull) return;
    int32_t lo = (int32_t)(k >> 32), hi = (int32_t)(k & 0xffffffffu);
    int32_t A = par[lo], B = par[hi];
    int32_t other = (A == (int32_t)x) ? B : A;
    if (bk[other] == k && (int32_t)x < other) return;  // mutual: the other side hooks
    tgt[x] = other;
    uint32_t at = atomicAdd(&counters[0], 1u);
    msf_lo[at] = lo;
    msf_hi[at] = hi;
}

__global__ void k_bor_apply(int32_t C, const int32_t *__restrict__ tgt, int32_t *__restrict__ par)
{
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x > C) return;
    par[x] = tgt[x];
}

// Full path compression of a static forest (no hooks run concurrently).
// A path in a forest of m nodes has fewer than m steps, which bounds the loop.
__global__ void k_compress(int64_t m, int32_t *__restrict__ par)
{
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= m) return;
    int32_t r = par[x];
    for (int64_t guard = 0; guard < m; guard++) {
        int32_t rr = par[r];
        if (rr == r) break;
        r = rr;
    }
    par[x] = r;
}

__global__ void k_iota(int64_t m, int32_t *__restrict__ p)
{
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < m) p[x] = (int32_t)x;
}

__device__ __forceinline__ int32_t uf_find(const int32_t *p, int32_t x)
{
    for (;;) {
        int32_t y = __atomic_load_n(&p[x], __ATOMIC_RELAXED);
        if (y == x) return x;
        x = y;
    }
}

__device__ __forceinline__ void uf_union(int32_t *p, int32_t a, int32_t b)
{
    for (;;) {
        a = uf_find(p, a);
        b = uf_find(p, b);
        if (a == b) return;
        if (a < b) {
            int32_t t = a;
            a = b;
            b = t;
        }
        // link the larger root under the smaller one
        if (atomicCAS(&p[a], a, b) == a) return;
    }
}

__global__ void k_union_msf(int64_t m, const int32_t *__restrict__ lo,
                            const int32_t *__restrict__ hi, int32_t *__restrict__ hp)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    uf_union(hp, lo[e], hi[e]);
}

__global__ void k_union_saddle(int64_t E, const int32_t *__restrict__ elo,
                               const int32_t *__restrict__ ehi, const uint64_t *__restrict__ es,
                               const double *__restrict__ cpeak, double delta_peak,
                               double delta_saddle, int32_t *__restrict__ hp)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    int32_t a = elo[e], b = ehi[e];
    double s = __longlong_as_double((long long)es[e]);
    if (cpeak[a] >= delta_peak && cpeak[b] >= delta_peak && s >= delta_saddle) uf_union(hp, a, b);
}

__global__ void k_rooted(int32_t C, const int32_t *__restrict__ hp, const double *__restrict__ cpeak,
                         double delta_peak, uint32_t *__restrict__ rooted)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    if (cpeak[c] >= delta_peak) rooted[hp[c]] = 1u;
}

__global__ void k_halo_accum(int32_t C, const int32_t *__restrict__ hp,
                             const uint32_t *__restrict__ rooted, const uint32_t *__restrict__ ccount,
                             const double *__restrict__ cpeak, uint32_t *__restrict__ hcount,
                             unsigned long long *__restrict__ hpeak)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    int32_t h = hp[c];
    if (!rooted[h]) return;
    if (ccount[c]) atomicAdd(&hcount[h], ccount[c]);
    atomicMax(&hpeak[h], (unsigned long long)__double_as_longlong(cpeak[c]));
}

__global__ void k_halo_peak_tk(int32_t C, const int32_t *__restrict__ hp,
                               const uint32_t *__restrict__ rooted, const double *__restrict__ cpeak,
                               const unsigned long long *__restrict__ hpeak,
                               const int32_t *__restrict__ croot, const int32_t *__restrict__ tk,
                               uint32_t *__restrict__ hptk)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    int32_t h = hp[c];
    if (!rooted[h]) return;
    if ((unsigned long long)__double_as_longlong(cpeak[c]) != hpeak[h]) return;
    int32_t r = croot[c];
    atomicMin(&hptk[h], (uint32_t)(tk ? tk[r] : r));
}

// halos with at least one labelled particle -> compact list, sort key = peak tie key
__global__ void k_halo_list(int32_t C, const int32_t *__restrict__ hp,
                            const uint32_t *__restrict__ rooted, const uint32_t *__restrict__ hcount,
                            const uint32_t *__restrict__ hptk, uint64_t *__restrict__ keys,
                            uint32_t *__restrict__ vals, uint32_t *__restrict__ counter)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    if (hp[c] != (int32_t)c || !rooted[c] || hcount[c] == 0) return;
    uint32_t at = atomicAdd(counter, 1u);
    keys[at] = hptk[c];
    vals[at] = (uint32_t)c;
}

__global__ void k_key_peak(int64_t G, const uint32_t *__restrict__ vals,
                           const unsigned long long *__restrict__ hpeak, uint64_t *__restrict__ keys)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= G) return;
    keys[t] = ~(uint64_t)hpeak[vals[t]];  // descending density
}

__global__ void k_key_count(int64_t G, const uint32_t *__restrict__ vals,
                            const uint32_t *__restrict__ hcount, uint64_t *__restrict__ keys)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= G) return;
    keys[t] = (uint64_t)(~hcount[vals[t]]);  // descending count (32 bits)
}

__global__ void k_number(int64_t G, const uint32_t *__restrict__ vals,
                         const uint32_t *__restrict__ hcount,
                         const unsigned long long *__restrict__ hpeak,
                         const uint32_t *__restrict__ hptk, const int32_t *__restrict__ tk2j,
                         int32_t *__restrict__ num, hop_group_info *__restrict__ out)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= G) return;
    uint32_t h = vals[t];
    num[h] = (int32_t)t;
    if (out) {
        hop_group_info g;
        g.count = hcount[h];
        uint32_t ptk = hptk[h];
        g.peak = tk2j ? tk2j[ptk] : (int32_t)ptk;
        g.reserved = 0;
        g.peak_density = __longlong_as_double((long long)hpeak[h]);
        out[t] = g;
    }
}

__global__ void k_group(int64_t n, const int32_t *__restrict__ chain_of, int32_t C,
                        const int32_t *__restrict__ hp, const uint32_t *__restrict__ rooted,
                        const int32_t *__restrict__ num, const uint8_t *__restrict__ padded,
                        int padded_rules, int32_t *__restrict__ group)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t c = chain_of[i];
    int32_t g = -1;
    if (c >= 0 && c < C && !(padded_rules && padded && padded[i])) {
        int32_t h = hp[c];
        if (rooted[h]) g = num[h];
    }
    group[i] = g;
}

// subvolume of chain c: the largest s < n_sub with chain_base[s] <= c
__device__ __forceinline__ int sub_of_chain(const int32_t *__restrict__ cbase, int n_sub, int32_t c)
{
    int lo = 0, hi = n_sub;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cbase[mid] <= c) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void k_key_sub(int64_t G, const uint32_t *__restrict__ vals,
                          const int32_t *__restrict__ cbase, int n_sub, uint64_t *__restrict__ keys)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= G) return;
    keys[t] = (uint64_t)sub_of_chain(cbase, n_sub, (int32_t)vals[t]);
}

__global__ void k_group_first(int64_t G, const uint32_t *__restrict__ vals,
                              const int32_t *__restrict__ cbase, int n_sub,
                              int32_t *__restrict__ gfirst)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= G) return;
    const int sv = sub_of_chain(cbase, n_sub, (int32_t)vals[t]);
    if (t == 0 || sub_of_chain(cbase, n_sub, (int32_t)vals[t - 1]) != sv) gfirst[sv] = (int32_t)t;
}

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

// carve aligned sub-arrays out of one buffer
struct Carver {
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

inline int64_t pow2ceil(int64_t v)
{
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

}  // namespace

int hop_merge_impl(hop_ctx *ctx, int64_t n, const int32_t *nbr, const double *density,
                   const int32_t *root, const int32_t *chain_of, int32_t n_chains,
                   const int32_t *tk, const uint8_t *padded, const hop_params *p, int32_t *group,
                   int32_t *n_groups, hop_group_info *groups, const MergeExtra &x, hipStream_t s)
{
    const int32_t *chain_base = x.chain_base;
    const int32_t n_sub = x.n_sub;
    int32_t *group_first = x.group_first;
    uint32_t *dflags = (uint32_t *)ctx->flags.ptr;
    uint32_t *dcnt = dflags + 4;  // [0] edges, [1] msf edges, [2] halos
    const int32_t C = n_chains;
    const int pr = (p->flags & HOP_PADDED_RULES) ? 1 : 0;
    const int32_t *tk2j = (tk && !x.tk_is_index) ? (const int32_t *)ctx->tk2j.ptr : nullptr;
    if (C <= 0) {
        k_fill_i32<<<hop_grid(n, 256), 256, 0, s>>>(group, n, -1);
        HOPCHK(ctx, hipGetLastError());
        HOPTRY(hop_check_device(ctx, s, "hop_merge"));
        *n_groups = 0;
        return HOP_OK;
    }

    // workspace for the chain-sized arrays
    const int64_t C1 = (int64_t)C + 1;
    size_t need = 0;
    need += (size_t)C1 * (4 + 8 + 4 + 4 + 8 + 8 + 4 + 4 + 4 + 4 + 8 + 4 + 4 + 4 + 4) + 20 * 256;
    HOPTRY(hop_reserve(ctx, ctx->work_b, need));
    Carver cv{(char *)ctx->work_b.ptr};
    int32_t *croot = cv.take<int32_t>(C1);
    double *cpeak = cv.take<double>(C1);
    int32_t *par = cv.take<int32_t>(C1);
    int32_t *tgt = cv.take<int32_t>(C1);
    unsigned long long *bs = cv.take<unsigned long long>(C1);
    unsigned long long *bk = cv.take<unsigned long long>(C1);
    int32_t *msf_lo = cv.take<int32_t>(C1);
    int32_t *msf_hi = cv.take<int32_t>(C1);
    int32_t *hp = cv.take<int32_t>(C1);
    uint32_t *rooted = cv.take<uint32_t>(C1);
    unsigned long long *hpeak = cv.take<unsigned long long>(C1);
    uint32_t *hptk = cv.take<uint32_t>(C1);
    uint32_t *ccount = cv.take<uint32_t>(C1);
    uint32_t *hcount = cv.take<uint32_t>(C1);
    int32_t *num = cv.take<int32_t>(C1);

    HOPCHK(ctx, hipMemsetAsync(ccount, 0, (size_t)C * 4, s));
    k_chain_table<<<hop_grid(n, 256), 256, 0, s>>>(n, root, chain_of, density, padded, pr, C, croot,
                                                   cpeak, ccount, dflags);
    HOPCHK(ctx, hipGetLastError());

    // --- boundary table -----------------------------------------------------
    const int64_t pairs_max = (int64_t)(p->n_merge - 1) * n;
    int64_t cap = ctx->tuning.hash_slots > 0
                      ? pow2ceil(ctx->tuning.hash_slots)
                      : pow2ceil(std::max<int64_t>(4096, std::min<int64_t>(16 * (int64_t)C, 2 * pairs_max + 1)));
    const int64_t cap_max = pow2ceil(2 * pairs_max + 1);
    int64_t E = 0;
    for (;;) {
        int log2cap = 0;
        while (((int64_t)1 << log2cap) < cap) log2cap++;
        HOPTRY(hop_reserve(ctx, ctx->hash_keys, (size_t)cap * 8));
        HOPTRY(hop_reserve(ctx, ctx->hash_vals, (size_t)cap * 8));
        uint64_t *hk = (uint64_t *)ctx->hash_keys.ptr;
        unsigned long long *hv = (unsigned long long *)ctx->hash_vals.ptr;
        HOPCHK(ctx, hipMemsetAsync(hk, 0xff, (size_t)cap * 8, s));
        HOPCHK(ctx, hipMemsetAsync(hv, 0, (size_t)cap * 8, s));
        HOPCHK(ctx, hipMemsetAsync(dcnt, 0, 16, s));
        k_saddle_insert<<<hop_grid(n, 256), 256, 0, s>>>(n, nbr, p->k_store, p->n_merge, density,
                                                        chain_of, padded, pr, C, hk, hv,
                                                        (uint64_t)(cap - 1), log2cap, dflags);
        HOPCHK(ctx, hipGetLastError());
        HOPCHK(ctx, hipMemcpyAsync(ctx->hflags + 2, dflags, 4, hipMemcpyDeviceToHost, s));
        HOPCHK(ctx, hipStreamSynchronize(s));
        uint32_t fl = (uint32_t)ctx->hflags[2];
        if ((fl & DERR_CAPACITY) && cap < cap_max) {
            // keep any other error bits, drop the capacity bit, retry larger
            ctx->hflags[3] = (int64_t)(fl & ~DERR_CAPACITY);
            HOPCHK(ctx, hipMemcpyAsync(dflags, &ctx->hflags[3], 4, hipMemcpyHostToDevice, s));
            cap *= 2;
            continue;
        }
        HOPTRY(hop_reserve(ctx, ctx->edges_lo, (size_t)cap * 4));
        HOPTRY(hop_reserve(ctx, ctx->edges_hi, (size_t)cap * 4));
        HOPTRY(hop_reserve(ctx, ctx->edges_s, (size_t)cap * 8));
        k_edge_compact<<<compact_grid(cap), 256, 0, s>>>(
            cap, hk, hv, (int32_t *)ctx->edges_lo.ptr, (int32_t *)ctx->edges_hi.ptr,
            (uint64_t *)ctx->edges_s.ptr, dcnt);
        HOPCHK(ctx, hipGetLastError());
        HOPCHK(ctx, hipMemcpyAsync(ctx->hflags + 2, dcnt, 4, hipMemcpyDeviceToHost, s));
        HOPCHK(ctx, hipStreamSynchronize(s));
        E = (int64_t)(uint32_t)ctx->hflags[2];
        break;
    }
    const int32_t *elo = (const int32_t *)ctx->edges_lo.ptr;
    const int32_t *ehi = (const int32_t *)ctx->edges_hi.ptr;
    const uint64_t *es = (const uint64_t *)ctx->edges_s.ptr;

    // --- maximum spanning forest with a virtual root (Boruvka) --------------
    k_bor_init<<<hop_grid(C1, 256), 256, 0, s>>>(C, cpeak, p->delta_peak, par);
    HOPCHK(ctx, hipGetLastError());
    HOPCHK(ctx, hipMemsetAsync(dcnt + 1, 0, 4, s));  // msf edge counter
    for (int round = 0; round < 64; round++) {
        HOPCHK(ctx, hipMemsetAsync(dcnt + 2, 0, 4, s));
        uint32_t before = 0;
        HOPCHK(ctx, hipMemcpyAsync(&ctx->hflags[4], dcnt + 1, 4, hipMemcpyDeviceToHost, s));
        k_bor_reset<<<hop_grid(C1, 256), 256, 0, s>>>(C, bs, bk);
        k_bor_best_s<<<hop_grid(E, 256), 256, 0, s>>>(E, elo, ehi, es, par, bs);
        k_bor_best_k<<<hop_grid(E, 256), 256, 0, s>>>(E, elo, ehi, es, par, bs, bk);
        k_bor_hook<<<hop_grid(C1, 256), 256, 0, s>>>(C, par, bk, tgt, msf_lo, msf_hi, dcnt + 1);
        k_bor_apply<<<hop_grid(C1, 256), 256, 0, s>>>(C, tgt, par);
        k_compress<<<hop_grid(C1, 256), 256, 0, s>>>(C1, par);
        HOPCHK(ctx, hipGetLastError());
        HOPCHK(ctx, hipMemcpyAsync(&ctx->hflags[5], dcnt + 1, 4, hipMemcpyDeviceToHost, s));
        HOPCHK(ctx, hipStreamSynchronize(s));
        before = (uint32_t)ctx->hflags[4];
        uint32_t after = (uint32_t)ctx->hflags[5];
        if (after == before) break;
        if (round == 63) return hop_fail(ctx, HOP_ERR_ARG, "merge did not converge");
    }
    const int64_t M = (int64_t)(uint32_t)ctx->hflags[5];

    // --- halos: forest edges + proto-halo saddles ---------------------------
    k_iota<<<hop_grid(C, 256), 256, 0, s>>>(C, hp);
    if (M > 0) k_union_msf<<<hop_grid(M, 256), 256, 0, s>>>(M, msf_lo, msf_hi, hp);
    if (E > 0)
        k_union_saddle<<<hop_grid(E, 256), 256, 0, s>>>(E, elo, ehi, es, cpeak, p->delta_peak,
                                                        p->delta_saddle, hp);
    if (x.n_pre > 0) k_union_msf<<<hop_grid(x.n_pre, 256), 256, 0, s>>>(x.n_pre, x.pre_lo, x.pre_hi, hp);
    k_compress<<<hop_grid(C, 256), 256, 0, s>>>(C, hp);
    HOPCHK(ctx, hipMemsetAsync(rooted, 0, (size_t)C * 4, s));
    k_rooted<<<hop_grid(C, 256), 256, 0, s>>>(C, hp, cpeak, p->delta_peak, rooted);
    HOPCHK(ctx, hipGetLastError());

    // --- labels --------------------------------------------------------------
    HOPCHK(ctx, hipMemsetAsync(hcount, 0, (size_t)C * 4, s));
    HOPCHK(ctx, hipMemsetAsync(hpeak, 0, (size_t)C * 8, s));
    HOPCHK(ctx, hipMemsetAsync(hptk, 0xff, (size_t)C * 4, s));
    k_halo_accum<<<hop_grid(C, 256), 256, 0, s>>>(C, hp, rooted, ccount, cpeak, hcount, hpeak);
    k_halo_peak_tk<<<hop_grid(C, 256), 256, 0, s>>>(C, hp, rooted, cpeak, hpeak, croot, tk, hptk);
    HOPCHK(ctx, hipGetLastError());
    HOPTRY(hop_reserve(ctx, ctx->keys_a, (size_t)C * 8));
    HOPTRY(hop_reserve(ctx, ctx->keys_b, (size_t)C * 8));
    HOPTRY(hop_reserve(ctx, ctx->vals_a, (size_t)C * 4));
    HOPTRY(hop_reserve(ctx, ctx->vals_b, (size_t)C * 4));
    uint64_t *keys = (uint64_t *)ctx->keys_a.ptr;
    uint32_t *vals = (uint32_t *)ctx->vals_a.ptr;
    HOPCHK(ctx, hipMemsetAsync(dcnt + 2, 0, 4, s));
    k_halo_list<<<hop_grid(C, 256), 256, 0, s>>>(C, hp, rooted, hcount, hptk, keys, vals, dcnt + 2);
    HOPCHK(ctx, hipGetLastError());
    HOPCHK(ctx, hipMemcpyAsync(&ctx->hflags[6], dcnt + 2, 4, hipMemcpyDeviceToHost, s));
    HOPCHK(ctx, hipStreamSynchronize(s));
    const int64_t G = (int64_t)(uint32_t)ctx->hflags[6];
    uint64_t *tkeys = (uint64_t *)ctx->keys_b.ptr;
    uint32_t *tvals = (uint32_t *)ctx->vals_b.ptr;
    if (G > 1) {
        HOPTRY(hop_radix_sort(ctx, keys, vals, tkeys, tvals, G, 32, s));
        k_key_peak<<<hop_grid(G, 256), 256, 0, s>>>(G, vals, hpeak, keys);
        HOPTRY(hop_radix_sort(ctx, keys, vals, tkeys, tvals, G, 64, s));
        k_key_count<<<hop_grid(G, 256), 256, 0, s>>>(G, vals, hcount, keys);
        HOPTRY(hop_radix_sort(ctx, keys, vals, tkeys, tvals, G, 32, s));
        if (chain_base) {
            // a batch: subvolume first, so each subvolume's groups are contiguous
            int sub_bits = 1;
            while (((int64_t)1 << sub_bits) < n_sub) sub_bits++;
            k_key_sub<<<hop_grid(G, 256), 256, 0, s>>>(G, vals, chain_base, n_sub, keys);
            HOPCHK(ctx, hipGetLastError());
            HOPTRY(hop_radix_sort(ctx, keys, vals, tkeys, tvals, G, sub_bits, s));
        }
    }
    if (chain_base && group_first && G > 0) {
        k_group_first<<<hop_grid(G, 256), 256, 0, s>>>(G, vals, chain_base, n_sub, group_first);
        HOPCHK(ctx, hipGetLastError());
    }
    if (G > 0)
        k_number<<<hop_grid(G, 256), 256, 0, s>>>(G, vals, hcount, hpeak, hptk, tk2j, num, groups);
    k_group<<<hop_grid(n, 256), 256, 0, s>>>(n, chain_of, C, hp, rooted, num, padded, pr, group);
    HOPCHK(ctx, hipGetLastError());
    HOPTRY(hop_check_device(ctx, s, "hop_merge"));
    *n_groups = (int32_t)G;
    return HOP_OK;
}

// ---------------------------------------------------------------------------
// Subhalos (the ADAPTAHOP-style extension of the paper's section 6): chain
// boundaries kept by direction, symmetric ones only, and at each level the
// structures of chains joined at or above it.  The boundary hash and the
// union-find are those of the merge above.
// ---------------------------------------------------------------------------

namespace {

// directed boundary maxima per chain pair: up = lo -> hi, down = hi -> lo
// (densities are positive, so a maximum of 0 means no pair)
__global__ void k_dir_insert(int64_t n, const int32_t *__restrict__ nbr, int k_store, int n_merge,
                             const double *__restrict__ dens, const int32_t *__restrict__ chain_of,
                             int32_t C, uint64_t *__restrict__ hkeys,
                             unsigned long long *__restrict__ hup,
                             unsigned long long *__restrict__ hdown, uint64_t mask, int log2cap,
                             uint32_t *__restrict__ dflags)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t ci = chain_of[i];
    if (ci < 0 || ci >= C) return;
    const double di = dens[i];
    for (int t = 1; t < n_merge; t++) {
        const int32_t j = nbr[i * k_store + t];
        if (j < 0 || j >= n) {
            atomicOr(dflags, DERR_INDEX);
            continue;
        }
        const int32_t cj = chain_of[j];
        if (cj < 0 || cj >= C || cj == ci) continue;
        const double sv = (di + dens[j]) * 0.5;
        const unsigned long long sb = (unsigned long long)__double_as_longlong(sv);
        const uint64_t key = ((uint64_t)(uint32_t)min(ci, cj) << 32) | (uint32_t)max(ci, cj);
        uint64_t slot = log2cap > 0 ? pair_hash(key) >> (64 - log2cap) : 0;
        bool done = false;
        for (uint64_t probe = 0; probe <= mask; probe++) {
            uint64_t k = hkeys[slot];
            if (k == kEmpty) {
                k = atomicCAS((unsigned long long *)&hkeys[slot], (unsigned long long)kEmpty,
                              (unsigned long long)key);
                if (k == kEmpty) k = key;
            }
            if (k == key) {
                atomicMax(ci < cj ? &hup[slot] : &hdown[slot], sb);
                done = true;
                break;
            }
            slot = (slot + 1) & mask;
        }
        if (!done) atomicOr(dflags, DERR_CAPACITY);
    }
}

// symmetric boundaries: both directions present; density the smaller maximum
__global__ void k_sym_compact(int64_t cap, const uint64_t *__restrict__ hkeys,
                              const unsigned long long *__restrict__ hup,
                              const unsigned long long *__restrict__ hdown,
                              int32_t *__restrict__ elo, int32_t *__restrict__ ehi,
                              double *__restrict__ es, uint32_t *__restrict__ count)
{
    wave_compact(
        cap, count,
        [&](int64_t t) { return hkeys[t] != kEmpty && hup[t] != 0ull && hdown[t] != 0ull; },
        [&](int64_t t, uint32_t at) {
            const uint64_t k = hkeys[t];
            elo[at] = (int32_t)(k >> 32);
            ehi[at] = (int32_t)(k & 0xffffffffu);
            es[at] = __longlong_as_double((long long)min(hup[t], hdown[t]));
        });
}

__global__ void k_union_level(int64_t E, const int32_t *__restrict__ elo,
                              const int32_t *__restrict__ ehi, const double *__restrict__ es,
                              double level, int32_t *__restrict__ hp)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    if (es[e] >= level) uf_union(hp, elo[e], ehi[e]);
}

// members (chained, density >= level): count and densest per structure
__global__ void k_sub_accum(int64_t n, const int32_t *__restrict__ chain_of, int32_t C,
                            const double *__restrict__ dens, double level,
                            const int32_t *__restrict__ hp, uint32_t *__restrict__ hcount,
                            unsigned long long *__restrict__ hpeak)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t c = chain_of[i];
    if (c < 0 || c >= C || !(dens[i] >= level)) return;
    const int32_t h = hp[c];
    atomicAdd(&hcount[h], 1u);
    atomicMax(&hpeak[h], (unsigned long long)__double_as_longlong(dens[i]));
}

__global__ void k_sub_peak_tk(int64_t n, const int32_t *__restrict__ chain_of, int32_t C,
                              const double *__restrict__ dens, double level,
                              const int32_t *__restrict__ hp,
                              const unsigned long long *__restrict__ hpeak,
                              const int32_t *__restrict__ tk, uint32_t *__restrict__ hptk)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t c = chain_of[i];
    if (c < 0 || c >= C || !(dens[i] >= level)) return;
    const int32_t h = hp[c];
    if ((unsigned long long)__double_as_longlong(dens[i]) != hpeak[h]) return;
    atomicMin(&hptk[h], (uint32_t)(tk ? tk[i] : (int32_t)i));
}

// structures with a member that pass the peak test -> list (key = peak tie key)
__global__ void k_sub_list(int32_t C, const int32_t *__restrict__ hp,
                           const uint32_t *__restrict__ hcount,
                           const unsigned long long *__restrict__ hpeak,
                           const uint32_t *__restrict__ hptk, double level, double alpha,
                           uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
                           uint32_t *__restrict__ counter)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    if (hp[c] != (int32_t)c || hcount[c] == 0) return;
    const double pk = __longlong_as_double((long long)hpeak[c]);
    if (!(pk >= level * (1.0 + alpha / __builtin_sqrt((double)hcount[c])))) return;
    const uint32_t at = atomicAdd(counter, 1u);
    keys[at] = hptk[c];
    vals[at] = (uint32_t)c;
}

__global__ void k_sub_number(int64_t G, const uint32_t *__restrict__ vals,
                             const uint32_t *__restrict__ hcount,
                             const unsigned long long *__restrict__ hpeak,
                             const uint32_t *__restrict__ hptk, const int32_t *__restrict__ tk2j,
                             const int32_t *__restrict__ prev, int32_t *__restrict__ num,
                             hop_subhalo_info *__restrict__ out)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= G) return;
    const uint32_t h = vals[t];
    num[h] = (int32_t)t;
    if (out) {
        hop_subhalo_info g;
        g.count = hcount[h];
        const uint32_t ptk = hptk[h];
        g.peak = tk2j ? tk2j[ptk] : (int32_t)ptk;
        g.parent = prev ? prev[g.peak] : -1;
        g.peak_density = __longlong_as_double((long long)hpeak[h]);
        out[t] = g;
    }
}

__global__ void k_sub_label(int64_t n, const int32_t *__restrict__ chain_of, int32_t C,
                            const double *__restrict__ dens, double level,
                            const int32_t *__restrict__ hp, const int32_t *__restrict__ num,
                            int32_t *__restrict__ sub)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t c = chain_of[i];
    int32_t lab = -1;
    if (c >= 0 && c < C && dens[i] >= level) lab = num[hp[c]];
    sub[i] = lab;
}

}  // namespace

extern "C" int hop_subhalos(hop_ctx *ctx, int64_t n, const int32_t *nbr, const double *density,
                            const int32_t *chain_of, int32_t n_chains, const int64_t *id,
                            const hop_params *p, int32_t n_levels, const double *levels,
                            double alpha, int32_t *sub, int64_t *t_off, hop_subhalo_info *table,
                            void *stream)
{
    if (!ctx) return HOP_ERR_ARG;
    ctx->err.clear();
    HOPTRY(hop_check_params(ctx, n, p));
    if (!nbr || !density || !chain_of || !sub || !t_off || !levels)
        return hop_fail(ctx, HOP_ERR_ARG, "nbr, density, chain_of, levels, sub and t_off must be non-NULL");
    if (n_chains < 0 || n_chains > n) return hop_fail(ctx, HOP_ERR_ARG, "n_chains outside [0, n]");
    if (n_levels < 1 || n_levels > 64) return hop_fail(ctx, HOP_ERR_ARG, "need 1 <= n_levels <= 64");
    if (!(alpha >= 0) || !(alpha < 1e300)) return hop_fail(ctx, HOP_ERR_ARG, "alpha must be finite and >= 0");
    for (int l = 0; l < n_levels; l++) {
        if (!(levels[l] >= 0) || !(levels[l] < 1e300))
            return hop_fail(ctx, HOP_ERR_ARG, "levels must be finite and >= 0");
        if (l > 0 && !(levels[l] > levels[l - 1])) return hop_fail(ctx, HOP_ERR_ARG, "levels must ascend");
    }
    HOPTRY(hop_set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    uint32_t *dflags = (uint32_t *)ctx->flags.ptr;
    uint32_t *dcnt = dflags + 4;
    const int32_t C = n_chains;
    const int32_t *tk = nullptr, *tk2j = nullptr;
    if (id) {
        HOPTRY(hop_build_tiekeys(ctx, n, id, s));
        tk = (const int32_t *)ctx->tk.ptr;
        tk2j = (const int32_t *)ctx->tk2j.ptr;
    }
    if (C == 0) {
        for (int l = 0; l <= n_levels; l++) t_off[l] = 0;
        k_fill_i32<<<hop_grid(n * n_levels, 256), 256, 0, s>>>(sub, n * n_levels, -1);
        HOPCHK(ctx, hipGetLastError());
        return hop_check_device(ctx, s, "hop_subhalos");
    }

    // 1. directed boundary maxima, then the symmetric ones
    const int64_t pairs_max = (int64_t)(p->n_merge - 1) * n;
    int64_t cap = ctx->tuning.hash_slots > 0
                      ? pow2ceil(ctx->tuning.hash_slots)
                      : pow2ceil(std::max<int64_t>(4096, std::min<int64_t>(16 * (int64_t)C, 2 * pairs_max + 1)));
    const int64_t cap_max = pow2ceil(2 * pairs_max + 1);
    for (;;) {
        int log2cap = 0;
        while (((int64_t)1 << log2cap) < cap) log2cap++;
        HOPTRY(hop_reserve(ctx, ctx->hash_keys, (size_t)cap * 8));
        HOPTRY(hop_reserve(ctx, ctx->hash_vals, (size_t)cap * 16));
        uint64_t *hk = (uint64_t *)ctx->hash_keys.ptr;
        unsigned long long *hup = (unsigned long long *)ctx->hash_vals.ptr;
        unsigned long long *hdown = hup + cap;
        HOPCHK(ctx, hipMemsetAsync(hk, 0xff, (size_t)cap * 8, s));
        HOPCHK(ctx, hipMemsetAsync(hup, 0, (size_t)cap * 16, s));
        k_dir_insert<<<hop_grid(n, 256), 256, 0, s>>>(n, nbr, p->k_store, p->n_merge, density, chain_of, C,
                                                      hk, hup, hdown, (uint64_t)(cap - 1), log2cap, dflags);
        HOPCHK(ctx, hipGetLastError());
        HOPCHK(ctx, hipMemcpyAsync(ctx->hflags + 2, dflags, 4, hipMemcpyDeviceToHost, s));
        HOPCHK(ctx, hipStreamSynchronize(s));
        const uint32_t fl = (uint32_t)ctx->hflags[2];
        if ((fl & DERR_CAPACITY) && cap < cap_max) {
            ctx->hflags[3] = (int64_t)(fl & ~DERR_CAPACITY);
            HOPCHK(ctx, hipMemcpyAsync(dflags, &ctx->hflags[3], 4, hipMemcpyHostToDevice, s));
            cap *= 2;
            continue;
        }
        break;
    }
    HOPTRY(hop_reserve(ctx, ctx->edges_lo, (size_t)cap * 4));
    HOPTRY(hop_reserve(ctx, ctx->edges_hi, (size_t)cap * 4));
    HOPTRY(hop_reserve(ctx, ctx->edges_s, (size_t)cap * 8));
    int32_t *elo = (int32_t *)ctx->edges_lo.ptr;
    int32_t *ehi = (int32_t *)ctx->edges_hi.ptr;
    double *es = (double *)ctx->edges_s.ptr;
    {
        const uint64_t *hk = (const uint64_t *)ctx->hash_keys.ptr;
        const unsigned long long *hup = (const unsigned long long *)ctx->hash_vals.ptr;
        HOPCHK(ctx, hipMemsetAsync(dcnt, 0, 4, s));
        k_sym_compact<<<compact_grid(cap), 256, 0, s>>>(cap, hk, hup, hup + cap, elo, ehi, es, dcnt);
        HOPCHK(ctx, hipGetLastError());
        HOPCHK(ctx, hipMemcpyAsync(ctx->hflags + 2, dcnt, 4, hipMemcpyDeviceToHost, s));
        HOPCHK(ctx, hipStreamSynchronize(s));
    }
    const int64_t E = (int64_t)(uint32_t)ctx->hflags[2];

    // 2. every level
    const int64_t C1 = (int64_t)C + 1;
    HOPTRY(hop_reserve(ctx, ctx->work_b, (size_t)C1 * (4 + 4 + 8 + 4 + 4) + 8 * 256));
    Carver cv{(char *)ctx->work_b.ptr};
    int32_t *hp = cv.take<int32_t>(C1);
    uint32_t *hcount = cv.take<uint32_t>(C1);
    unsigned long long *hpeak = cv.take<unsigned long long>(C1);
    uint32_t *hptk = cv.take<uint32_t>(C1);
    int32_t *num = cv.take<int32_t>(C1);
    HOPTRY(hop_reserve(ctx, ctx->keys_a, (size_t)C * 8));
    HOPTRY(hop_reserve(ctx, ctx->keys_b, (size_t)C * 8));
    HOPTRY(hop_reserve(ctx, ctx->vals_a, (size_t)C * 4));
    HOPTRY(hop_reserve(ctx, ctx->vals_b, (size_t)C * 4));
    uint64_t *keys = (uint64_t *)ctx->keys_a.ptr;
    uint32_t *vals = (uint32_t *)ctx->vals_a.ptr;
    uint64_t *tkeys = (uint64_t *)ctx->keys_b.ptr;
    uint32_t *tvals = (uint32_t *)ctx->vals_b.ptr;
    int64_t base = 0;
    for (int l = 0; l < n_levels; l++) {
        const double lev = levels[l];
        k_iota<<<hop_grid(C, 256), 256, 0, s>>>(C, hp);
        k_fill_i32<<<hop_grid(C, 256), 256, 0, s>>>(num, C, -1);  // structures not kept: no number
        if (E > 0) k_union_level<<<hop_grid(E, 256), 256, 0, s>>>(E, elo, ehi, es, lev, hp);
        k_compress<<<hop_grid(C, 256), 256, 0, s>>>(C, hp);
        HOPCHK(ctx, hipMemsetAsync(hcount, 0, (size_t)C * 4, s));
        HOPCHK(ctx, hipMemsetAsync(hpeak, 0, (size_t)C * 8, s));
        HOPCHK(ctx, hipMemsetAsync(hptk, 0xff, (size_t)C * 4, s));
        k_sub_accum<<<hop_grid(n, 256), 256, 0, s>>>(n, chain_of, C, density, lev, hp, hcount, hpeak);
        k_sub_peak_tk<<<hop_grid(n, 256), 256, 0, s>>>(n, chain_of, C, density, lev, hp, hpeak, tk, hptk);
        HOPCHK(ctx, hipMemsetAsync(dcnt + 2, 0, 4, s));
        k_sub_list<<<hop_grid(C, 256), 256, 0, s>>>(C, hp, hcount, hpeak, hptk, lev, alpha, keys, vals,
                                                    dcnt + 2);
        HOPCHK(ctx, hipGetLastError());
        HOPCHK(ctx, hipMemcpyAsync(&ctx->hflags[6], dcnt + 2, 4, hipMemcpyDeviceToHost, s));
        HOPCHK(ctx, hipStreamSynchronize(s));
        const int64_t G = (int64_t)(uint32_t)ctx->hflags[6];
        if (G > 1) {
            HOPTRY(hop_radix_sort(ctx, keys, vals, tkeys, tvals, G, 32, s));
            k_key_peak<<<hop_grid(G, 256), 256, 0, s>>>(G, vals, hpeak, keys);
            HOPTRY(hop_radix_sort(ctx, keys, vals, tkeys, tvals, G, 64, s));
            k_key_count<<<hop_grid(G, 256), 256, 0, s>>>(G, vals, hcount, keys);
            HOPTRY(hop_radix_sort(ctx, keys, vals, tkeys, tvals, G, 32, s));
        }
        int32_t *sub_l = sub + (int64_t)l * n;
        if (G > 0)
            k_sub_number<<<hop_grid(G, 256), 256, 0, s>>>(G, vals, hcount, hpeak, hptk, tk2j,
                                                          l > 0 ? sub_l - n : nullptr, num,
                                                          table ? table + base : nullptr);
        k_sub_label<<<hop_grid(n, 256), 256, 0, s>>>(n, chain_of, C, density, lev, hp, num, sub_l);
        HOPCHK(ctx, hipGetLastError());
        t_off[l] = base;
        base += G;
    }
    t_off[n_levels] = base;
    ctx->stats.premerged = E;
    return hop_check_device(ctx, s, "hop_subhalos");
}
