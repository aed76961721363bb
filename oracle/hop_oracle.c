/*
 * hop_oracle.c -- plain CPU oracle for the HOP hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file's library.  It shares no code,
 * header, table or helper with the GPU implementation; the two meet only in
 * the seeded particle arrays that the generator module produces.
 *
 * What it computes (Skory et al., "Parallel HOP", section 2 "HOP", and the
 * per-task rules of section 3.1):
 *   1. the N_dens nearest neighbours of every particle, self included
 *      (section 2, first stage), found either by brute force -- the plain
 *      definition -- or by a bucketed kd-tree, the paper's own search
 *      structure (section 2, second paragraph; exact, no loss of accuracy);
 *   2. an SPH cubic-spline (M4) density over those neighbours, normalised by
 *      the mean particle density (section 2, first paragraph);
 *   3. the link of each particle to the densest of its N_hop nearest, which
 *      may be itself (section 2, third paragraph); padded particles link to
 *      themselves (section 3.1, chain-building rule);
 *   4. chains followed uphill to a self-linked particle, with particles below
 *      delta_outer excluded (section 2, merging step one);
 *   5. the boundary table: for chained particles, their N_merge nearest in a
 *      different chain, keeping the maximum pair-mean density per chain pair,
 *      both directions counted, padded-padded pairs skipped (section 2,
 *      merging step three; section 3.1, premerge paragraph);
 *   6. the merge: proto-halos at peak >= delta_peak, unions of proto-halo
 *      pairs with boundary >= delta_saddle, and the attachment of sub-peak
 *      chains along the densest (propagated) boundaries, done here as a
 *      Kruskal pass in decreasing boundary density that never joins two
 *      components that already hold a proto-halo (section 2, merging steps
 *      four and five; Figure 1);
 *   7. group labels: halos ordered by particle count (section 4 appendix:
 *      halos are sorted by mass), padded particles dropped (section 3.1, last
 *      step).
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - kernel: M4 cubic spline with h = half the distance to the N_dens-th
 *     neighbour (self counted as the first), unit masses;
 *   - ties: neighbours ordered by (d^2, id, index); densest-neighbour ties
 *     go to the smallest (id, index); chains are numbered by their root's
 *     (id, index); the merge orders boundaries by (s desc, lo asc, hi asc);
 *   - N_merge counts self, so the boundary search uses ranks 1..N_merge-1;
 *   - a particle is excluded when delta < delta_outer; a boundary needs both
 *     particles in chains; proto-halo when peak >= delta_peak;
 *   - delta_link = 0.5*(delta_i + delta_j) in FP64;
 *   - sub-peak chains that reach no proto-halo are dropped;
 *   - groups are numbered by count desc, peak density desc, peak (id, index)
 *     asc; a halo with no unpadded member is not a group.
 *
 * Floating point: FP64, round to nearest, no contraction (build with
 * -ffp-contract=off), correctly rounded division and square root.  The
 * spline weights of one particle are summed pairwise over a zero-padded
 * power-of-two array (adding +0.0 is exact), which fixes the summation order.
 *
 * Every entry point returns 0 on success and a negative code on error.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_ARG (-1)
#define ORC_ERR_DEGENERATE (-3)
#define ORC_ERR_NOMEM (-5)

#define ORC_MAX_K 128

/* pi rounded to the nearest double (bits 0x400921FB54442D18) */
#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* distances                                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    const uint32_t *pos; /* [n][3] */
    const int64_t *id;   /* [n] or NULL */
    int64_t n;
    int periodic;
    uint32_t gmask;      /* 2^grid_bits - 1 */
    uint64_t gsize;      /* 2^grid_bits */
} space_t;

static int64_t axis_sep(const space_t *s, uint32_t a, uint32_t b)
{
    if (s->periodic) {
        uint64_t u = (uint64_t)((a - b) & s->gmask);
        uint64_t v = s->gsize - u;
        return (int64_t)(u < v ? u : v);
    }
    return a > b ? (int64_t)(a - b) : (int64_t)(b - a);
}

static int64_t dist2(const space_t *s, int64_t i, int64_t j)
{
    int64_t d2 = 0;
    for (int a = 0; a < 3; a++) {
        int64_t d = axis_sep(s, s->pos[3 * i + a], s->pos[3 * j + a]);
        d2 += d * d;
    }
    return d2;
}

static int64_t tie_id(const space_t *s, int64_t j)
{
    return s->id ? s->id[j] : j;
}

/* neighbour candidate, ordered by (d2, id, index) */
typedef struct {
    int64_t d2;
    int64_t id;
    int64_t idx;
} cand_t;

static int cand_less(const cand_t *a, const cand_t *b)
{
    if (a->d2 != b->d2) return a->d2 < b->d2;
    if (a->id != b->id) return a->id < b->id;
    return a->idx < b->idx;
}

/* bounded max-heap holding the K smallest candidates seen so far */
typedef struct {
    cand_t e[ORC_MAX_K];
    int size, cap;
} kheap_t;

static void kheap_offer(kheap_t *h, cand_t c)
{
    if (h->size < h->cap) {
        int i = h->size++;
        h->e[i] = c;
        while (i > 0) {
            int p = (i - 1) / 2;
            if (!cand_less(&h->e[p], &h->e[i])) break;
            cand_t t = h->e[p]; h->e[p] = h->e[i]; h->e[i] = t;
            i = p;
        }
        return;
    }
    if (!cand_less(&c, &h->e[0])) return;
    h->e[0] = c;
    int i = 0;
    for (;;) {
        int l = 2 * i + 1, r = l + 1, m = i;
        if (l < h->size && cand_less(&h->e[m], &h->e[l])) m = l;
        if (r < h->size && cand_less(&h->e[m], &h->e[r])) m = r;
        if (m == i) break;
        cand_t t = h->e[m]; h->e[m] = h->e[i]; h->e[i] = t;
        i = m;
    }
}

static int cand_cmp(const void *a, const void *b)
{
    const cand_t *x = (const cand_t *)a, *y = (const cand_t *)b;
    if (cand_less(x, y)) return -1;
    if (cand_less(y, x)) return 1;
    return 0;
}

/* write L_q = [q, then the K nearest others ascending]; d2 of each */
static void kheap_emit(kheap_t *h, int64_t q, int k, int32_t *nbr_row, int64_t *d2_row)
{
    qsort(h->e, (size_t)h->size, sizeof(cand_t), cand_cmp);
    nbr_row[0] = (int32_t)q;
    if (d2_row) d2_row[0] = 0;
    for (int t = 1; t < k; t++) {
        nbr_row[t] = (int32_t)h->e[t - 1].idx;
        if (d2_row) d2_row[t] = h->e[t - 1].d2;
    }
}

/* ------------------------------------------------------------------------ */
/* 1a. brute-force kNN: the plain definition                                 */
/* ------------------------------------------------------------------------ */

/*
 * For each query q in queries[0..nq): L_q[0] = q, then the k-1 particles
 * j != q with the smallest (d^2, id, index).  Rows go to nbr[t*k ...] and
 * (optionally) d2[t*k ...].
 */
int orc_knn_brute(int64_t n, const uint32_t *pos, const int64_t *id, int periodic,
                  int grid_bits, int k, const int64_t *queries, int64_t nq,
                  int32_t *nbr, int64_t *d2)
{
    if (n < k || k < 1 || k > ORC_MAX_K || grid_bits < 1 || grid_bits > 21)
        return ORC_ERR_ARG;
    space_t s = {pos, id, n, periodic, (uint32_t)((1u << grid_bits) - 1u),
                 (uint64_t)1 << grid_bits};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nq; t++) {
        int64_t q = queries ? queries[t] : t;
        kheap_t h;
        h.size = 0;
        h.cap = k - 1;
        for (int64_t j = 0; j < n; j++) {
            if (j == q) continue;
            cand_t c = {dist2(&s, q, j), tie_id(&s, j), j};
            kheap_offer(&h, c);
        }
        kheap_emit(&h, q, k, nbr + t * k, d2 ? d2 + t * k : NULL);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* 1b. kd-tree kNN (the paper's search structure: buckets of tens of points) */
/* ------------------------------------------------------------------------ */

#define KD_BUCKET 16

typedef struct {
    uint32_t lo[3], hi[3];
    int64_t start, end;   /* range in the index array */
    int64_t left, right;  /* child nodes, -1 for a bucket */
} kdnode_t;

typedef struct {
    const space_t *s;
    int64_t *idx;
    kdnode_t *nodes;
    int64_t n_nodes;
} kdtree_t;

static void kd_swap(int64_t *a, int64_t *b) { int64_t t = *a; *a = *b; *b = t; }

/* quickselect: place the element of rank m (by coordinate on axis, then index) */
static void kd_select(const space_t *s, int64_t *idx, int64_t lo, int64_t hi,
                      int64_t m, int axis)
{
    while (hi - lo > 1) {
        int64_t mid = lo + (hi - lo) / 2;
        /* median of three as pivot */
        int64_t a = idx[lo], b = idx[mid], c = idx[hi - 1];
        uint32_t va = s->pos[3 * a + axis], vb = s->pos[3 * b + axis], vc = s->pos[3 * c + axis];
        int64_t piv;
        if ((va <= vb && vb <= vc) || (vc <= vb && vb <= va)) piv = mid;
        else if ((vb <= va && va <= vc) || (vc <= va && va <= vb)) piv = lo;
        else piv = hi - 1;
        kd_swap(&idx[piv], &idx[hi - 1]);
        uint32_t pv = s->pos[3 * idx[hi - 1] + axis];
        int64_t pi = idx[hi - 1];
        int64_t store = lo;
        for (int64_t i = lo; i < hi - 1; i++) {
            uint32_t v = s->pos[3 * idx[i] + axis];
            if (v < pv || (v == pv && idx[i] < pi)) {
                kd_swap(&idx[i], &idx[store]);
                store++;
            }
        }
        kd_swap(&idx[store], &idx[hi - 1]);
        if (store == m) return;
        if (m < store) hi = store;
        else lo = store + 1;
    }
}

static int64_t kd_build(kdtree_t *t, int64_t start, int64_t end)
{
    int64_t me = t->n_nodes++;
    kdnode_t *nd = &t->nodes[me];
    nd->start = start;
    nd->end = end;
    for (int a = 0; a < 3; a++) { nd->lo[a] = UINT32_MAX; nd->hi[a] = 0; }
    for (int64_t i = start; i < end; i++)
        for (int a = 0; a < 3; a++) {
            uint32_t v = t->s->pos[3 * t->idx[i] + a];
            if (v < nd->lo[a]) nd->lo[a] = v;
            if (v > nd->hi[a]) nd->hi[a] = v;
        }
    if (end - start <= KD_BUCKET) {
        nd->left = nd->right = -1;
        return me;
    }
    int axis = 0;
    uint32_t ext = nd->hi[0] - nd->lo[0];
    for (int a = 1; a < 3; a++)
        if (nd->hi[a] - nd->lo[a] > ext) { ext = nd->hi[a] - nd->lo[a]; axis = a; }
    int64_t mid = start + (end - start) / 2;
    kd_select(t->s, t->idx, start, end, mid, axis);
    int64_t l = kd_build(t, start, mid);
    int64_t r = kd_build(t, mid, end);
    t->nodes[me].left = l;
    t->nodes[me].right = r;
    return me;
}

/* squared distance from particle q to a node's bounding box */
static int64_t kd_boxdist2(const space_t *s, int64_t q, const kdnode_t *nd)
{
    int64_t d2 = 0;
    for (int a = 0; a < 3; a++) {
        uint32_t x = s->pos[3 * q + a];
        int64_t d = 0;
        if (x < nd->lo[a] || x > nd->hi[a]) {
            if (s->periodic) {
                uint64_t up = (uint64_t)((nd->lo[a] - x) & s->gmask); /* x -> lo going up */
                uint64_t dn = (uint64_t)((x - nd->hi[a]) & s->gmask); /* x -> hi going down */
                d = (int64_t)(up < dn ? up : dn);
            } else {
                d = x < nd->lo[a] ? (int64_t)(nd->lo[a] - x) : (int64_t)(x - nd->hi[a]);
            }
        }
        d2 += d * d;
    }
    return d2;
}

static void kd_search(const kdtree_t *t, int64_t node, int64_t q, kheap_t *h)
{
    const kdnode_t *nd = &t->nodes[node];
    if (nd->left < 0) {
        for (int64_t i = nd->start; i < nd->end; i++) {
            int64_t j = t->idx[i];
            if (j == q) continue;
            cand_t c = {dist2(t->s, q, j), tie_id(t->s, j), j};
            kheap_offer(h, c);
        }
        return;
    }
    int64_t a = nd->left, b = nd->right;
    int64_t da = kd_boxdist2(t->s, q, &t->nodes[a]);
    int64_t db = kd_boxdist2(t->s, q, &t->nodes[b]);
    if (db < da) { int64_t tt = a; a = b; b = tt; int64_t td = da; da = db; db = td; }
    /* a box is skipped only when every point in it is strictly farther */
    if (h->size < h->cap || da <= h->e[0].d2) kd_search(t, a, q, h);
    if (h->size < h->cap || db <= h->e[0].d2) kd_search(t, b, q, h);
}

/* build the tree over all n particles (t->s must be set) */
static int kd_make(kdtree_t *t, int64_t n)
{
    t->idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    /* every bucket holds at least KD_BUCKET/2 points, so nodes < n/4 + 2 */
    t->nodes = (kdnode_t *)malloc(sizeof(kdnode_t) * (size_t)(n / 2 + 16));
    t->n_nodes = 0;
    if (!t->idx || !t->nodes) {
        free(t->idx);
        free(t->nodes);
        return ORC_ERR_NOMEM;
    }
    for (int64_t i = 0; i < n; i++) t->idx[i] = i;
    kd_build(t, 0, n);
    return ORC_OK;
}

static void kd_free(kdtree_t *t)
{
    free(t->idx);
    free(t->nodes);
}

int orc_knn_kdtree(int64_t n, const uint32_t *pos, const int64_t *id, int periodic,
                   int grid_bits, int k, const int64_t *queries, int64_t nq,
                   int32_t *nbr, int64_t *d2)
{
    if (n < k || k < 1 || k > ORC_MAX_K || grid_bits < 1 || grid_bits > 21)
        return ORC_ERR_ARG;
    space_t s = {pos, id, n, periodic, (uint32_t)((1u << grid_bits) - 1u),
                 (uint64_t)1 << grid_bits};
    kdtree_t t;
    t.s = &s;
    int err = kd_make(&t, n);
    if (err) return err;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < nq; r++) {
        int64_t q = queries ? queries[r] : r;
        kheap_t h;
        h.size = 0;
        h.cap = k - 1;
        kd_search(&t, 0, q, &h);
        kheap_emit(&h, q, k, nbr + r * k, d2 ? d2 + r * k : NULL);
    }
    kd_free(&t);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* 2. SPH density                                                            */
/* ------------------------------------------------------------------------ */

/* M4 cubic spline shape, without the 1/(pi h^3) factor; q2 = (r/h)^2 */
static double m4_shape(double q2)
{
    double q = sqrt(q2);
    if (q2 < 1.0) return 1.0 - (0.75 * (2.0 - q)) * q2;          /* 1 - 1.5q^2 + 0.75q^3 */
    if (q2 < 4.0) return 0.25 * (((2.0 - q) * (2.0 - q)) * (2.0 - q)); /* 0.25 (2-q)^3 */
    return 0.0;
}

static double pairwise_sum(const double *w, int len)
{
    /* len is a power of two */
    if (len == 1) return w[0];
    int h = len / 2;
    return pairwise_sum(w, h) + pairwise_sum(w + h, h);
}

/*
 * density of one particle from the squared distances of its k = N_dens
 * neighbours (d2_row[0] = 0 is self; d2_row[k-1] is the farthest).
 *   h = r_max / 2, R = r_max^2, q^2 = 4 d^2 / R,
 *   delta = (sum_t w(q_t)) * norm / h^3, norm = 1 / (pi * mean_density).
 */
static int density_one(const int64_t *d2_row, int k, double norm, double *out)
{
    int64_t R = d2_row[k - 1];
    if (R <= 0) return ORC_ERR_DEGENERATE;
    double w[ORC_MAX_K];
    int p2 = 1;
    while (p2 < k) p2 *= 2;
    for (int t = 0; t < p2; t++) {
        if (t < k) {
            double q2 = (double)(4 * d2_row[t]) / (double)R;
            w[t] = m4_shape(q2);
        } else {
            w[t] = 0.0;
        }
    }
    double S = pairwise_sum(w, p2);
    double h2 = (double)R * 0.25;
    double h = sqrt(h2);
    double h3 = h2 * h;
    *out = (S * norm) / h3;
    return ORC_OK;
}

/* norm as the caller computes it: 1 / (pi * mean_density) */
double orc_norm(double mean_density)
{
    return 1.0 / (ORC_PI * mean_density);
}

int orc_density(int64_t nq, int k, const int64_t *d2, double mean_density, double *dens)
{
    if (k < 1 || k > ORC_MAX_K || !(mean_density > 0)) return ORC_ERR_ARG;
    double norm = orc_norm(mean_density);
    int err = ORC_OK;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < nq; t++) {
        int e = density_one(d2 + t * k, k, norm, &dens[t]);
        if (e) {
#pragma omp atomic write
            err = e;
        }
    }
    return err;
}

/* ------------------------------------------------------------------------ */
/* 3. densest-neighbour link                                                 */
/* ------------------------------------------------------------------------ */

/* key order for "densest": larger delta wins; equal delta -> smaller (id, index) */
static int denser(double da, int64_t ida, int64_t a, double db, int64_t idb, int64_t b)
{
    if (da != db) return da > db;
    if (ida != idb) return ida < idb;
    return a < b;
}

/*
 * hop[i] = the densest of nbr[i][0..n_hop) (row stride k_store), self
 * included.  Padded particles (padded_rules and padded[i]) link to
 * themselves.
 */
int orc_hop(int64_t n, int k_store, int n_hop, const int32_t *nbr, const double *dens,
            const int64_t *id, const uint8_t *padded, int padded_rules, int32_t *hop)
{
    if (n_hop < 1 || n_hop > k_store) return ORC_ERR_ARG;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        if (padded_rules && padded && padded[i]) { hop[i] = (int32_t)i; continue; }
        int64_t best = i;
        for (int t = 0; t < n_hop; t++) {
            int64_t j = nbr[i * k_store + t];
            if (denser(dens[j], id ? id[j] : j, j, dens[best], id ? id[best] : best, best))
                best = j;
        }
        hop[i] = (int32_t)best;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* 4. chains                                                                 */
/* ------------------------------------------------------------------------ */

static const int64_t *g_sort_id; /* qsort context (single-threaded use) */

static int root_cmp(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    int64_t ix = g_sort_id ? g_sort_id[x] : x, iy = g_sort_id ? g_sort_id[y] : y;
    if (ix != iy) return ix < iy ? -1 : 1;
    return (x > y) - (x < y);
}

/*
 * root[i]: follow hop to the self-linked particle.  Alive particles are
 * those with delta >= delta_outer; chains are the alive roots numbered by
 * (id, index) of the root; chain_of[i] = that number for alive i, else -1.
 * chain_root[c] and chain_peak[c] (= delta of the root) have room for n.
 */
int orc_chains(int64_t n, const int32_t *hop, const double *dens, const int64_t *id,
               double delta_outer, int32_t *root, int32_t *chain_of, int32_t *chain_root,
               double *chain_peak, int64_t *n_chains)
{
    int err = ORC_OK;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        int64_t r = i;
        int64_t steps = 0;
        while (hop[r] != r) {
            r = hop[r];
            if (++steps > n) break;
        }
        if (steps > n) {
#pragma omp atomic write
            err = ORC_ERR_ARG; /* a cycle: links did not go uphill */
        }
        root[i] = (int32_t)r;
    }
    if (err) return err;
    int64_t *roots = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int32_t *num = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!roots || !num) { free(roots); free(num); return ORC_ERR_NOMEM; }
    int64_t c = 0;
    for (int64_t i = 0; i < n; i++)
        if (root[i] == i && dens[i] >= delta_outer) roots[c++] = i;
    g_sort_id = id;
    qsort(roots, (size_t)c, sizeof(int64_t), root_cmp);
    g_sort_id = NULL;
    for (int64_t i = 0; i < n; i++) num[i] = -1;
    for (int64_t t = 0; t < c; t++) {
        num[roots[t]] = (int32_t)t;
        chain_root[t] = (int32_t)roots[t];
        chain_peak[t] = dens[roots[t]];
    }
    for (int64_t i = 0; i < n; i++)
        chain_of[i] = dens[i] >= delta_outer ? num[root[i]] : -1;
    *n_chains = c;
    free(roots);
    free(num);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* 5. boundary (saddle) table                                                */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t lo, hi;
    double s;
} edge_t;

static int edge_key_cmp(const void *a, const void *b)
{
    const edge_t *x = (const edge_t *)a, *y = (const edge_t *)b;
    if (x->lo != y->lo) return x->lo < y->lo ? -1 : 1;
    if (x->hi != y->hi) return x->hi < y->hi ? -1 : 1;
    if (x->s != y->s) return x->s > y->s ? -1 : 1; /* max first */
    return 0;
}

/*
 * For every particle i in a chain and every j among nbr[i][1..n_merge)
 * that is in a different chain (and not both padded when padded_rules):
 * s = 0.5*(delta_i + delta_j) for the unordered chain pair; the table keeps
 * the maximum per pair.  Output: edges sorted by (lo, hi), lo < hi, with
 * room for cap entries; *n_edges is the count (ORC_ERR_ARG if cap is short).
 */
int orc_saddles(int64_t n, int k_store, int n_merge, const int32_t *nbr, const double *dens,
                const int32_t *chain_of, const uint8_t *padded, int padded_rules,
                int32_t *e_lo, int32_t *e_hi, double *e_s, int64_t cap, int64_t *n_edges)
{
    if (n_merge < 1 || n_merge > k_store) return ORC_ERR_ARG;
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++) {
        if (chain_of[i] < 0) continue;
        for (int t = 1; t < n_merge; t++) {
            int64_t j = nbr[i * k_store + t];
            if (chain_of[j] < 0 || chain_of[j] == chain_of[i]) continue;
            if (padded_rules && padded && padded[i] && padded[j]) continue;
            m++;
        }
    }
    edge_t *all = (edge_t *)malloc(sizeof(edge_t) * (size_t)(m > 0 ? m : 1));
    if (!all) return ORC_ERR_NOMEM;
    int64_t w = 0;
    for (int64_t i = 0; i < n; i++) {
        if (chain_of[i] < 0) continue;
        for (int t = 1; t < n_merge; t++) {
            int64_t j = nbr[i * k_store + t];
            if (chain_of[j] < 0 || chain_of[j] == chain_of[i]) continue;
            if (padded_rules && padded && padded[i] && padded[j]) continue;
            int32_t a = chain_of[i], b = chain_of[j];
            all[w].lo = a < b ? a : b;
            all[w].hi = a < b ? b : a;
            all[w].s = (dens[i] + dens[j]) * 0.5;
            w++;
        }
    }
    qsort(all, (size_t)m, sizeof(edge_t), edge_key_cmp);
    int64_t e = 0;
    for (int64_t r = 0; r < m; r++) {
        if (r > 0 && all[r].lo == all[r - 1].lo && all[r].hi == all[r - 1].hi) continue;
        if (e >= cap) { free(all); return ORC_ERR_ARG; }
        e_lo[e] = all[r].lo;
        e_hi[e] = all[r].hi;
        e_s[e] = all[r].s;
        e++;
    }
    *n_edges = e;
    free(all);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* 6. merge                                                                  */
/* ------------------------------------------------------------------------ */

static int64_t uf_find(int64_t *par, int64_t x)
{
    while (par[x] != x) {
        par[x] = par[par[x]];
        x = par[x];
    }
    return x;
}

static int edge_merge_cmp(const void *a, const void *b)
{
    const edge_t *x = (const edge_t *)a, *y = (const edge_t *)b;
    if (x->s != y->s) return x->s > y->s ? -1 : 1;
    if (x->lo != y->lo) return x->lo < y->lo ? -1 : 1;
    if (x->hi != y->hi) return x->hi < y->hi ? -1 : 1;
    return 0;
}

/*
 * chain_halo[c] = the smallest chain number in c's halo, or -1 when the
 * chain reaches no proto-halo.
 */
int orc_merge(int64_t n_chains, const double *chain_peak, int64_t n_edges,
              const int32_t *e_lo, const int32_t *e_hi, const double *e_s,
              double delta_saddle, double delta_peak, int32_t *chain_halo)
{
    int64_t C = n_chains;
    int64_t *par = (int64_t *)malloc(sizeof(int64_t) * (size_t)(C > 0 ? C : 1));
    uint8_t *rooted = (uint8_t *)calloc((size_t)(C > 0 ? C : 1), 1);
    edge_t *ed = (edge_t *)malloc(sizeof(edge_t) * (size_t)(n_edges > 0 ? n_edges : 1));
    if (!par || !rooted || !ed) { free(par); free(rooted); free(ed); return ORC_ERR_NOMEM; }
    for (int64_t c = 0; c < C; c++) {
        par[c] = c;
        rooted[c] = chain_peak[c] >= delta_peak; /* proto-halo */
    }
    for (int64_t e = 0; e < n_edges; e++) {
        if (e_lo[e] < 0 || e_hi[e] >= C || e_lo[e] >= e_hi[e]) {
            free(par); free(rooted); free(ed);
            return ORC_ERR_ARG;
        }
        ed[e].lo = e_lo[e];
        ed[e].hi = e_hi[e];
        ed[e].s = e_s[e];
    }
    /* proto-halos sharing a boundary >= delta_saddle always merge */
    for (int64_t e = 0; e < n_edges; e++) {
        if (!(chain_peak[ed[e].lo] >= delta_peak && chain_peak[ed[e].hi] >= delta_peak)) continue;
        if (!(ed[e].s >= delta_saddle)) continue;
        int64_t a = uf_find(par, ed[e].lo), b = uf_find(par, ed[e].hi);
        if (a == b) continue;
        if (a < b) par[b] = a; else par[a] = b;
    }
    /* densest boundaries first; a component holding a proto-halo never
       joins another such component */
    qsort(ed, (size_t)n_edges, sizeof(edge_t), edge_merge_cmp);
    for (int64_t e = 0; e < n_edges; e++) {
        int64_t a = uf_find(par, ed[e].lo), b = uf_find(par, ed[e].hi);
        if (a == b) continue;
        if (rooted[a] && rooted[b]) continue;
        uint8_t r = rooted[a] | rooted[b];
        if (a < b) { par[b] = a; rooted[a] = r; }
        else { par[a] = b; rooted[b] = r; }
    }
    for (int64_t c = 0; c < C; c++) {
        int64_t r = uf_find(par, c);
        chain_halo[c] = rooted[r] ? (int32_t)r : -1;
    }
    free(par);
    free(rooted);
    free(ed);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* 7. labels                                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t count;
    double peak_dens;
    int64_t peak_id;
    int64_t peak_idx;
    int32_t halo; /* representative chain */
} grp_t;

static int grp_cmp(const void *a, const void *b)
{
    const grp_t *x = (const grp_t *)a, *y = (const grp_t *)b;
    if (x->count != y->count) return x->count > y->count ? -1 : 1;
    if (x->peak_dens != y->peak_dens) return x->peak_dens > y->peak_dens ? -1 : 1;
    if (x->peak_id != y->peak_id) return x->peak_id < y->peak_id ? -1 : 1;
    return (x->peak_idx > y->peak_idx) - (x->peak_idx < y->peak_idx);
}

/*
 * group[i] = number of the halo holding chain_of[i], or -1 (no chain, no
 * halo, or padded under padded_rules).  Halos are numbered by (unpadded
 * member count desc, peak density desc, peak (id, index) asc); halos with no
 * unpadded member get no number.  g_count/g_peak/g_peak_dens have room for
 * n_chains entries.
 */
int orc_labels(int64_t n, const int32_t *chain_of, int64_t n_chains, const int32_t *chain_root,
               const double *chain_peak, const int32_t *chain_halo, const int64_t *id,
               const uint8_t *padded, int padded_rules, int32_t *group, int64_t *n_groups,
               int64_t *g_count, int32_t *g_peak, double *g_peak_dens)
{
    int64_t C = n_chains;
    grp_t *g = (grp_t *)malloc(sizeof(grp_t) * (size_t)(C > 0 ? C : 1));
    int32_t *num = (int32_t *)malloc(sizeof(int32_t) * (size_t)(C > 0 ? C : 1));
    if (!g || !num) { free(g); free(num); return ORC_ERR_NOMEM; }
    for (int64_t c = 0; c < C; c++) {
        g[c].count = 0;
        g[c].peak_dens = -1.0;
        g[c].peak_id = INT64_MAX;
        g[c].peak_idx = INT64_MAX;
        g[c].halo = (int32_t)c;
        num[c] = -1;
    }
    for (int64_t i = 0; i < n; i++) {
        int32_t c = chain_of[i];
        if (c < 0 || chain_halo[c] < 0) continue;
        if (padded_rules && padded && padded[i]) continue;
        g[chain_halo[c]].count++;
    }
    for (int64_t c = 0; c < C; c++) {
        int32_t h = chain_halo[c];
        if (h < 0) continue;
        int64_t r = chain_root[c];
        int64_t rid = id ? id[r] : r;
        if (denser(chain_peak[c], rid, r, g[h].peak_dens, g[h].peak_id, g[h].peak_idx)) {
            g[h].peak_dens = chain_peak[c];
            g[h].peak_id = rid;
            g[h].peak_idx = r;
        }
    }
    int64_t G = 0;
    for (int64_t c = 0; c < C; c++)
        if (g[c].count > 0) g[G++] = g[c];
    qsort(g, (size_t)G, sizeof(grp_t), grp_cmp);
    for (int64_t t = 0; t < G; t++) {
        num[g[t].halo] = (int32_t)t;
        if (g_count) g_count[t] = g[t].count;
        if (g_peak) g_peak[t] = (int32_t)g[t].peak_idx;
        if (g_peak_dens) g_peak_dens[t] = g[t].peak_dens;
    }
    for (int64_t i = 0; i < n; i++) {
        int32_t c = chain_of[i];
        int32_t lab = -1;
        if (c >= 0 && chain_halo[c] >= 0 && !(padded_rules && padded && padded[i]))
            lab = num[chain_halo[c]];
        group[i] = lab;
    }
    *n_groups = G;
    free(g);
    free(num);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* 8. subhalos (ADAPTAHOP-style extension, section 6)                        */
/* ------------------------------------------------------------------------ */

/*
 * The paper sketches subhalo finding as an extension: chains are found as in
 * HOP; only "symmetric" boundaries between chains are kept (both chains
 * link to the other); boundaries below a level delta_s are destroyed; the
 * remaining structure at each level gives the subhalos; structures below
 * the level of Poisson noise are rejected; several levels give a hierarchy.
 * It fixes no formulas; the readings taken here:
 *   - directed boundary A->B: the maximum of 0.5 (delta_i + delta_j) over
 *     chained i in A and j in B among nbr[i][1 .. n_merge) (the HOP boundary
 *     pairs, kept by direction);
 *   - symmetric boundary {A, B}: present when both A->B and B->A are, with
 *     density min(D(A->B), D(B->A)): the level down to which each chain
 *     reaches the other;
 *   - at level delta_s: chains joined by symmetric boundaries >= delta_s form
 *     structures; a structure's members are its particles with density >=
 *     delta_s; its peak is its densest member (ties to the smaller (id,
 *     index));
 *   - significance: a structure of N members is kept when its peak density
 *     is >= delta_s (1 + alpha / sqrt(N)) (alpha = 0 keeps every structure
 *     with a member);
 *   - numbering per level as the halos (count desc, peak density desc, peak
 *     (id, index) asc); parent = the previous level's number of the
 *     structure holding the peak particle (-1 at the first level or when
 *     that particle is in none).
 * Levels must ascend.  sub[l * n + i] = number of particle i's structure at
 * level l or -1; per level l the tables start at t_off[l] (t_off has
 * n_levels + 1 entries; capacity n_levels * n_chains).
 */
typedef struct {
    int32_t a, b;  /* ordered: from chain a to chain b */
    double s;
} dedge_t;

static int dedge_cmp(const void *x, const void *y)
{
    const dedge_t *p = (const dedge_t *)x, *q = (const dedge_t *)y;
    int32_t pl = p->a < p->b ? p->a : p->b, ph = p->a < p->b ? p->b : p->a;
    int32_t ql = q->a < q->b ? q->a : q->b, qh = q->a < q->b ? q->b : q->a;
    if (pl != ql) return pl < ql ? -1 : 1;
    if (ph != qh) return ph < qh ? -1 : 1;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    return 0;
}

int orc_subhalos(int64_t n, int k_cols, int n_merge, const int32_t *nbr, const double *dens,
                 const int32_t *chain_of, int64_t n_chains, const int64_t *id,
                 const double *levels, int n_levels, double alpha, int32_t *sub,
                 int64_t *t_off, int64_t *t_count, int32_t *t_peak, double *t_peak_dens,
                 int32_t *t_parent, int64_t *n_sym)
{
    if (n_merge < 1 || n_merge > k_cols || n_levels < 1 || !(alpha >= 0)) return ORC_ERR_ARG;
    for (int l = 1; l < n_levels; l++)
        if (!(levels[l] > levels[l - 1])) return ORC_ERR_ARG;
    const int64_t C = n_chains;
    /* 1. directed pairs */
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++) {
        if (chain_of[i] < 0) continue;
        for (int t = 1; t < n_merge; t++) {
            int64_t j = nbr[i * k_cols + t];
            if (chain_of[j] >= 0 && chain_of[j] != chain_of[i]) m++;
        }
    }
    dedge_t *d = (dedge_t *)malloc(sizeof(dedge_t) * (size_t)(m > 0 ? m : 1));
    int32_t *s_lo = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int32_t *s_hi = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    double *s_v = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    int64_t *par = (int64_t *)malloc(sizeof(int64_t) * (size_t)(C > 0 ? C : 1));
    grp_t *g = (grp_t *)malloc(sizeof(grp_t) * (size_t)(C > 0 ? C : 1));
    int32_t *num = (int32_t *)malloc(sizeof(int32_t) * (size_t)(C > 0 ? C : 1));
    if (!d || !s_lo || !s_hi || !s_v || !par || !g || !num) {
        free(d); free(s_lo); free(s_hi); free(s_v); free(par); free(g); free(num);
        return ORC_ERR_NOMEM;
    }
    int64_t w = 0;
    for (int64_t i = 0; i < n; i++) {
        if (chain_of[i] < 0) continue;
        for (int t = 1; t < n_merge; t++) {
            int64_t j = nbr[i * k_cols + t];
            if (chain_of[j] < 0 || chain_of[j] == chain_of[i]) continue;
            d[w].a = chain_of[i];
            d[w].b = chain_of[j];
            d[w].s = (dens[i] + dens[j]) * 0.5;
            w++;
        }
    }
    /* 2. per unordered pair: the maximum of each direction, kept when both exist */
    qsort(d, (size_t)m, sizeof(dedge_t), dedge_cmp);
    int64_t E = 0;
    for (int64_t r = 0; r < m;) {
        int32_t lo = d[r].a < d[r].b ? d[r].a : d[r].b, hi = d[r].a < d[r].b ? d[r].b : d[r].a;
        double up = -1.0, down = -1.0; /* lo -> hi, hi -> lo */
        int64_t q = r;
        for (; q < m; q++) {
            int32_t l2 = d[q].a < d[q].b ? d[q].a : d[q].b, h2 = d[q].a < d[q].b ? d[q].b : d[q].a;
            if (l2 != lo || h2 != hi) break;
            if (d[q].a == lo) { if (d[q].s > up) up = d[q].s; }
            else if (d[q].s > down) down = d[q].s;
        }
        if (up >= 0.0 && down >= 0.0) {
            s_lo[E] = lo;
            s_hi[E] = hi;
            s_v[E] = up < down ? up : down;
            E++;
        }
        r = q;
    }
    *n_sym = E;
    /* 3. every level */
    int64_t base = 0;
    for (int l = 0; l < n_levels; l++) {
        const double lev = levels[l];
        for (int64_t c = 0; c < C; c++) par[c] = c;
        for (int64_t e = 0; e < E; e++) {
            if (!(s_v[e] >= lev)) continue;
            int64_t a = uf_find(par, s_lo[e]), b = uf_find(par, s_hi[e]);
            if (a == b) continue;
            if (a < b) par[b] = a; else par[a] = b;
        }
        for (int64_t c = 0; c < C; c++) {
            g[c].count = 0;
            g[c].peak_dens = -1.0;
            g[c].peak_id = INT64_MAX;
            g[c].peak_idx = INT64_MAX;
            g[c].halo = (int32_t)c;
            num[c] = -1;
        }
        for (int64_t i = 0; i < n; i++) {
            if (chain_of[i] < 0 || !(dens[i] >= lev)) continue;
            int64_t r = uf_find(par, chain_of[i]);
            g[r].count++;
            int64_t iid = id ? id[i] : i;
            if (denser(dens[i], iid, i, g[r].peak_dens, g[r].peak_id, g[r].peak_idx)) {
                g[r].peak_dens = dens[i];
                g[r].peak_id = iid;
                g[r].peak_idx = i;
            }
        }
        int64_t G = 0;
        for (int64_t c = 0; c < C; c++) {
            if (g[c].count < 1) continue;
            if (!(g[c].peak_dens >= lev * (1.0 + alpha / sqrt((double)g[c].count)))) continue;
            g[G++] = g[c];
        }
        qsort(g, (size_t)G, sizeof(grp_t), grp_cmp);
        for (int64_t t = 0; t < G; t++) {
            num[g[t].halo] = (int32_t)t;
            t_count[base + t] = g[t].count;
            t_peak[base + t] = (int32_t)g[t].peak_idx;
            t_peak_dens[base + t] = g[t].peak_dens;
            t_parent[base + t] = l > 0 ? sub[(int64_t)(l - 1) * n + g[t].peak_idx] : -1;
        }
        for (int64_t i = 0; i < n; i++) {
            int32_t lab = -1;
            if (chain_of[i] >= 0 && dens[i] >= lev) lab = num[uf_find(par, chain_of[i])];
            sub[(int64_t)l * n + i] = lab;
        }
        t_off[l] = base;
        base += G;
    }
    t_off[n_levels] = base;
    free(d); free(s_lo); free(s_hi); free(s_v); free(par); free(g); free(num);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* whole pipeline                                                            */
/* ------------------------------------------------------------------------ */

/*
 * Stages 3-7 (links, chains, boundaries, merge, labels) from the densities
 * and the first k_cols list columns (k_cols >= n_hop, n_merge).
 */
static int run_stages(int64_t n, const int64_t *id, const uint8_t *padded, int n_hop,
                      int n_merge, int k_cols, double delta_outer, double delta_saddle,
                      double delta_peak, int padded_rules, const double *dens,
                      const int32_t *nbr, int32_t *hop, int32_t *root, int32_t *chain_of,
                      int32_t *group, int64_t *g_count, int32_t *g_peak, double *g_peak_dens,
                      int64_t *counts)
{
    int err = orc_hop(n, k_cols, n_hop, nbr, dens, id, padded, padded_rules, hop);
    if (err) return err;
    int32_t *chain_root = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *chain_peak = (double *)malloc(sizeof(double) * (size_t)n);
    int64_t cap = (int64_t)n * (n_merge > 1 ? n_merge - 1 : 1) + 1;
    int32_t *e_lo = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    int32_t *e_hi = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    double *e_s = (double *)malloc(sizeof(double) * (size_t)cap);
    int32_t *chain_halo = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t C = 0, E = 0, G = 0;
    if (!chain_root || !chain_peak || !e_lo || !e_hi || !e_s || !chain_halo) {
        err = ORC_ERR_NOMEM;
        goto done;
    }
    err = orc_chains(n, hop, dens, id, delta_outer, root, chain_of, chain_root, chain_peak, &C);
    if (err) goto done;
    err = orc_saddles(n, k_cols, n_merge, nbr, dens, chain_of, padded, padded_rules, e_lo, e_hi,
                      e_s, cap, &E);
    if (err) goto done;
    err = orc_merge(C, chain_peak, E, e_lo, e_hi, e_s, delta_saddle, delta_peak, chain_halo);
    if (err) goto done;
    err = orc_labels(n, chain_of, C, chain_root, chain_peak, chain_halo, id, padded, padded_rules,
                     group, &G, g_count, g_peak, g_peak_dens);
done:
    counts[0] = C;
    counts[1] = E;
    counts[2] = G;
    free(chain_root);
    free(chain_peak);
    free(e_lo);
    free(e_hi);
    free(e_s);
    free(chain_halo);
    return err;
}

/*
 * Runs stages 1-7 for all particles.  search: 0 = brute force, 1 = kd-tree.
 * Output arrays are caller-owned: dens[n], nbr[n*k_store], hop[n], root[n],
 * chain_of[n], group[n], and g_count/g_peak/g_peak_dens with room for n.
 * counts[0..2] = n_chains, n_edges, n_groups.
 */
int orc_run(int64_t n, const uint32_t *pos, const int64_t *id, const uint8_t *padded,
            int periodic, int grid_bits, int n_dens, int n_hop, int n_merge, int k_store,
            double delta_outer, double delta_saddle, double delta_peak, double mean_density,
            int padded_rules, int search,
            double *dens, int32_t *nbr, int32_t *hop, int32_t *root, int32_t *chain_of,
            int32_t *group, int64_t *g_count, int32_t *g_peak, double *g_peak_dens,
            int64_t *counts)
{
    if (!(1 <= n_merge && n_merge <= n_hop && n_hop <= k_store && k_store <= n_dens &&
          n_dens <= ORC_MAX_K))
        return ORC_ERR_ARG;
    if (n < n_dens) return ORC_ERR_ARG;
    int k = n_dens;
    int32_t *full = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * (size_t)k);
    int64_t *d2 = (int64_t *)malloc(sizeof(int64_t) * (size_t)n * (size_t)k);
    if (!full || !d2) { free(full); free(d2); return ORC_ERR_NOMEM; }
    int err = search ? orc_knn_kdtree(n, pos, id, periodic, grid_bits, k, NULL, n, full, d2)
                     : orc_knn_brute(n, pos, id, periodic, grid_bits, k, NULL, n, full, d2);
    if (!err) err = orc_density(n, k, d2, mean_density, dens);
    free(d2);
    if (err) { free(full); return err; }
    for (int64_t i = 0; i < n; i++)
        memcpy(nbr + i * k_store, full + i * k, sizeof(int32_t) * (size_t)k_store);
    free(full);
    return run_stages(n, id, padded, n_hop, n_merge, k_store, delta_outer, delta_saddle,
                      delta_peak, padded_rules, dens, nbr, hop, root, chain_of, group, g_count,
                      g_peak, g_peak_dens, counts);
}

/*
 * Word-wise FNV-1a over a list row (offset basis 0xcbf29ce484222325, prime
 * 0x100000001b3, one step per 32-bit entry): a fingerprint of a row kept
 * when the row itself is too long to keep for every particle.
 */
static uint64_t row_fnv1a(const int32_t *row, int k)
{
    uint64_t h = 0xcbf29ce484222325ull;
    for (int t = 0; t < k; t++) {
        h ^= (uint64_t)(uint32_t)row[t];
        h *= 0x100000001b3ull;
    }
    return h;
}

/*
 * The same pipeline as orc_run in bounded memory, for boxes whose n x N_dens
 * lists do not fit: the kd-tree is built once (orc_lite_begin) and queried
 * in pieces (orc_lite_query, by ranges of the tree's leaf order, which only
 * changes which particles share a piece); each piece's full lists give the
 * densities and are then reduced to
 *   nbr[n][k_keep]   the first k_keep entries of every list (k_keep >= n_hop,
 *                    n_merge: the later stages read nothing else),
 *   row_hash[n]      row_fnv1a of the first k_store entries,
 *   r2max[n]         (optional) d^2 to the N_dens-th entry.
 * Stages 3-7 then run as in orc_run on the kept columns (orc_stages), so
 * every output equals orc_run's (the list columns by their fingerprint).
 * The caller keeps pos and id alive until orc_lite_end.
 */
typedef struct {
    space_t s;
    kdtree_t t;
    int k, k_store, k_keep;
    double norm;
} orc_lite_t;

void *orc_lite_begin(int64_t n, const uint32_t *pos, const int64_t *id, int periodic,
                     int grid_bits, int n_dens, int k_store, int k_keep, double mean_density)
{
    if (!(1 <= k_keep && k_keep <= k_store && k_store <= n_dens && n_dens <= ORC_MAX_K))
        return NULL;
    if (n < n_dens || grid_bits < 1 || grid_bits > 21 || !(mean_density > 0)) return NULL;
    orc_lite_t *L = (orc_lite_t *)calloc(1, sizeof(orc_lite_t));
    if (!L) return NULL;
    space_t s = {pos, id, n, periodic, (uint32_t)((1u << grid_bits) - 1u),
                 (uint64_t)1 << grid_bits};
    L->s = s;
    L->t.s = &L->s;
    L->k = n_dens;
    L->k_store = k_store;
    L->k_keep = k_keep;
    L->norm = orc_norm(mean_density);
    if (kd_make(&L->t, n)) {
        free(L);
        return NULL;
    }
    return L;
}

/* the particles at tree positions [c0, c1); outputs indexed by particle */
int orc_lite_query(void *h, int64_t c0, int64_t c1, double *dens, int32_t *nbr,
                   uint64_t *row_hash, int64_t *r2max)
{
    orc_lite_t *L = (orc_lite_t *)h;
    if (!L || c0 < 0 || c1 > L->s.n || c0 > c1) return ORC_ERR_ARG;
    const int k = L->k;
    const int64_t m = c1 - c0;
    int32_t *full = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1) * (size_t)k);
    int64_t *d2 = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1) * (size_t)k);
    if (!full || !d2) {
        free(full);
        free(d2);
        return ORC_ERR_NOMEM;
    }
    int err = ORC_OK;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < m; r++) {
        const int64_t q = L->t.idx[c0 + r];
        kheap_t hp;
        hp.size = 0;
        hp.cap = k - 1;
        kd_search(&L->t, 0, q, &hp);
        int32_t *row = full + r * k;
        int64_t *drow = d2 + r * k;
        kheap_emit(&hp, q, k, row, drow);
        int e = density_one(drow, k, L->norm, &dens[q]);
        if (e) {
#pragma omp atomic write
            err = e;
        }
        row_hash[q] = row_fnv1a(row, L->k_store);
        memcpy(nbr + q * L->k_keep, row, sizeof(int32_t) * (size_t)L->k_keep);
        if (r2max) r2max[q] = drow[k - 1];
    }
    free(full);
    free(d2);
    return err;
}

void orc_lite_end(void *h)
{
    orc_lite_t *L = (orc_lite_t *)h;
    if (!L) return;
    kd_free(&L->t);
    free(L);
}

/* stages 3-7 from densities and the first k_cols list columns */
int orc_stages(int64_t n, const int64_t *id, const uint8_t *padded, int n_hop, int n_merge,
               int k_cols, double delta_outer, double delta_saddle, double delta_peak,
               int padded_rules, const double *dens, const int32_t *nbr, int32_t *hop,
               int32_t *root, int32_t *chain_of, int32_t *group, int64_t *g_count,
               int32_t *g_peak, double *g_peak_dens, int64_t *counts)
{
    if (!(1 <= n_merge && n_merge <= n_hop && n_hop <= k_cols && k_cols <= ORC_MAX_K))
        return ORC_ERR_ARG;
    return run_stages(n, id, padded, n_hop, n_merge, k_cols, delta_outer, delta_saddle,
                      delta_peak, padded_rules, dens, nbr, hop, root, chain_of, group, g_count,
                      g_peak, g_peak_dens, counts);
}

/* all of the above in one call, in pieces of `chunk` particles */
int orc_run_lite(int64_t n, const uint32_t *pos, const int64_t *id, const uint8_t *padded,
                 int periodic, int grid_bits, int n_dens, int n_hop, int n_merge, int k_store,
                 int k_keep, double delta_outer, double delta_saddle, double delta_peak,
                 double mean_density, int padded_rules, int64_t chunk,
                 double *dens, int32_t *nbr, uint64_t *row_hash, int64_t *r2max,
                 int32_t *hop, int32_t *root, int32_t *chain_of, int32_t *group,
                 int64_t *g_count, int32_t *g_peak, double *g_peak_dens, int64_t *counts)
{
    if (!(1 <= n_merge && n_merge <= n_hop && n_hop <= k_keep) || chunk < 1) return ORC_ERR_ARG;
    void *L = orc_lite_begin(n, pos, id, periodic, grid_bits, n_dens, k_store, k_keep,
                             mean_density);
    if (!L) return ORC_ERR_ARG;
    int err = ORC_OK;
    for (int64_t c0 = 0; c0 < n && !err; c0 += chunk)
        err = orc_lite_query(L, c0, n - c0 < chunk ? n : c0 + chunk, dens, nbr, row_hash, r2max);
    orc_lite_end(L);
    if (err) return err;
    return orc_stages(n, id, padded, n_hop, n_merge, k_keep, delta_outer, delta_saddle,
                      delta_peak, padded_rules, dens, nbr, hop, root, chain_of, group, g_count,
                      g_peak, g_peak_dens, counts);
}

/* threads of the OpenMP loops from now on (n >= 1) */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
