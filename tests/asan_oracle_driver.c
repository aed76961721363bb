/*
 * Memory-safety driver for the C oracle: built together with
 * oracle/hop_oracle.c under AddressSanitizer and UndefinedBehaviorSanitizer
 * by tests/test_oracle_asan.py and run on the CPU.  It calls every stage on
 * small clustered boxes (periodic and not, with ids, padded particles,
 * N_dens 64 and 128), the bounded-memory pipeline in pieces, the subhalos,
 * and the argument checks; any out-of-bounds access, leak or undefined
 * operation ends the run with a sanitizer report.  It also checks that the
 * kd-tree search equals the brute-force one and that the bounded-memory
 * pipeline gives the same groups as the full one.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_run(int64_t n, const uint32_t *pos, const int64_t *id, const uint8_t *padded,
            int periodic, int grid_bits, int n_dens, int n_hop, int n_merge, int k_store,
            double delta_outer, double delta_saddle, double delta_peak, double mean_density,
            int padded_rules, int search, double *dens, int32_t *nbr, int32_t *hop,
            int32_t *root, int32_t *chain_of, int32_t *group, int64_t *g_count,
            int32_t *g_peak, double *g_peak_dens, int64_t *counts);
int orc_run_lite(int64_t n, const uint32_t *pos, const int64_t *id, const uint8_t *padded,
                 int periodic, int grid_bits, int n_dens, int n_hop, int n_merge, int k_store,
                 int k_keep, double delta_outer, double delta_saddle, double delta_peak,
                 double mean_density, int padded_rules, int64_t chunk, double *dens,
                 int32_t *nbr, uint64_t *row_hash, int64_t *r2max, int32_t *hop, int32_t *root,
                 int32_t *chain_of, int32_t *group, int64_t *g_count, int32_t *g_peak,
                 double *g_peak_dens, int64_t *counts);
int orc_subhalos(int64_t n, int k_cols, int n_merge, const int32_t *nbr, const double *dens,
                 const int32_t *chain_of, int64_t n_chains, const int64_t *id,
                 const double *levels, int n_levels, double alpha, int32_t *sub,
                 int64_t *t_off, int64_t *t_count, int32_t *t_peak, double *t_peak_dens,
                 int32_t *t_parent, int64_t *n_sym);

#define GRID_BITS 16

static uint64_t rng_state;

static uint64_t next_u64(void)
{
    /* splitmix64 */
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* n particles: a third uniform, the rest in 6 compact clumps */
static void make_box(int64_t n, uint64_t seed, uint32_t *pos)
{
    const uint32_t G = 1u << GRID_BITS;
    rng_state = seed;
    uint32_t cx[6], cy[6], cz[6];
    for (int c = 0; c < 6; c++) {
        cx[c] = (uint32_t)(next_u64() % G);
        cy[c] = (uint32_t)(next_u64() % G);
        cz[c] = (uint32_t)(next_u64() % G);
    }
    for (int64_t i = 0; i < n; i++) {
        if (i % 3 == 0) {
            for (int k = 0; k < 3; k++) pos[3 * i + k] = (uint32_t)(next_u64() % G);
        } else {
            const int c = (int)(next_u64() % 6);
            const uint32_t r = 64u + (uint32_t)(c * 96);
            pos[3 * i + 0] = (cx[c] + (uint32_t)(next_u64() % (2 * r)) - r) & (G - 1);
            pos[3 * i + 1] = (cy[c] + (uint32_t)(next_u64() % (2 * r)) - r) & (G - 1);
            pos[3 * i + 2] = (cz[c] + (uint32_t)(next_u64() % (2 * r)) - r) & (G - 1);
        }
    }
}

typedef struct {
    double *dens;
    int32_t *nbr, *hop, *root, *chain_of, *group, *g_peak;
    int64_t *g_count;
    double *g_peak_dens;
    int64_t counts[3];
} outputs;

static void alloc_out(outputs *o, int64_t n, int k)
{
    o->dens = malloc(sizeof(double) * (size_t)n);
    o->nbr = malloc(sizeof(int32_t) * (size_t)n * (size_t)k);
    o->hop = malloc(sizeof(int32_t) * (size_t)n);
    o->root = malloc(sizeof(int32_t) * (size_t)n);
    o->chain_of = malloc(sizeof(int32_t) * (size_t)n);
    o->group = malloc(sizeof(int32_t) * (size_t)n);
    o->g_peak = malloc(sizeof(int32_t) * (size_t)n);
    o->g_count = malloc(sizeof(int64_t) * (size_t)n);
    o->g_peak_dens = malloc(sizeof(double) * (size_t)n);
}

static void free_out(outputs *o)
{
    free(o->dens);
    free(o->nbr);
    free(o->hop);
    free(o->root);
    free(o->chain_of);
    free(o->group);
    free(o->g_peak);
    free(o->g_count);
    free(o->g_peak_dens);
}

static int fail(const char *what, int rc)
{
    fprintf(stderr, "asan driver: %s returned %d\n", what, rc);
    return 1;
}

static int run_case(int64_t n, int periodic, int n_dens, int k_store, int with_ids,
                    int with_padded, uint64_t seed)
{
    const double mean_density = (double)n / ((double)(1u << GRID_BITS) * (1u << GRID_BITS) *
                                             (1u << GRID_BITS));
    const int n_hop = k_store < 16 ? k_store : 16, n_merge = n_hop < 4 ? n_hop : 4;
    uint32_t *pos = malloc(sizeof(uint32_t) * 3 * (size_t)n);
    int64_t *id = NULL;
    uint8_t *padded = NULL;
    make_box(n, seed, pos);
    if (with_ids) {
        id = malloc(sizeof(int64_t) * (size_t)n);
        for (int64_t i = 0; i < n; i++) id[i] = (int64_t)((i * 7919) % n) * 3 + 11;
    }
    if (with_padded) {
        padded = malloc((size_t)n);
        for (int64_t i = 0; i < n; i++) padded[i] = (uint8_t)(pos[3 * i] < (1u << (GRID_BITS - 3)));
    }
    outputs a, b, c;
    alloc_out(&a, n, k_store);
    alloc_out(&b, n, k_store);
    alloc_out(&c, n, 16);
    int bad = 0, rc;
    rc = orc_run(n, pos, id, padded, periodic, GRID_BITS, n_dens, n_hop, n_merge, k_store, 80.0,
                 200.0, 240.0, mean_density, with_padded, 1, a.dens, a.nbr, a.hop, a.root,
                 a.chain_of, a.group, a.g_count, a.g_peak, a.g_peak_dens, a.counts);
    if (rc) bad |= fail("orc_run (kd-tree)", rc);
    rc = orc_run(n, pos, id, padded, periodic, GRID_BITS, n_dens, n_hop, n_merge, k_store, 80.0,
                 200.0, 240.0, mean_density, with_padded, 0, b.dens, b.nbr, b.hop, b.root,
                 b.chain_of, b.group, b.g_count, b.g_peak, b.g_peak_dens, b.counts);
    if (rc) bad |= fail("orc_run (brute force)", rc);
    if (!bad && (memcmp(a.nbr, b.nbr, sizeof(int32_t) * (size_t)n * (size_t)k_store) ||
                 memcmp(a.dens, b.dens, sizeof(double) * (size_t)n) ||
                 memcmp(a.group, b.group, sizeof(int32_t) * (size_t)n))) {
        fprintf(stderr, "asan driver: kd-tree and brute force differ\n");
        bad = 1;
    }
    /* the bounded-memory pipeline in pieces of 97 particles, 16 columns kept */
    uint64_t *row_hash = malloc(sizeof(uint64_t) * (size_t)n);
    int64_t *r2max = malloc(sizeof(int64_t) * (size_t)n);
    rc = orc_run_lite(n, pos, id, padded, periodic, GRID_BITS, n_dens, n_hop, n_merge, k_store, 16,
                      80.0, 200.0, 240.0, mean_density, with_padded, 97, c.dens, c.nbr, row_hash,
                      r2max, c.hop, c.root, c.chain_of, c.group, c.g_count, c.g_peak,
                      c.g_peak_dens, c.counts);
    if (rc) bad |= fail("orc_run_lite", rc);
    if (!bad && (memcmp(a.group, c.group, sizeof(int32_t) * (size_t)n) ||
                 memcmp(a.dens, c.dens, sizeof(double) * (size_t)n))) {
        fprintf(stderr, "asan driver: bounded-memory pipeline differs\n");
        bad = 1;
    }
    if (!bad) {
        const double levels[3] = {80.0, 400.0, 2000.0};
        const int64_t cap = 3 * (a.counts[0] > 0 ? a.counts[0] : 1);
        int32_t *sub = malloc(sizeof(int32_t) * 3 * (size_t)n);
        int64_t t_off[4], n_sym = 0;
        int64_t *t_count = malloc(sizeof(int64_t) * (size_t)cap);
        int32_t *t_peak = malloc(sizeof(int32_t) * (size_t)cap);
        double *t_pd = malloc(sizeof(double) * (size_t)cap);
        int32_t *t_par = malloc(sizeof(int32_t) * (size_t)cap);
        rc = orc_subhalos(n, k_store, n_merge, a.nbr, a.dens, a.chain_of, a.counts[0], id, levels,
                          3, 1.0, sub, t_off, t_count, t_peak, t_pd, t_par, &n_sym);
        if (rc) bad |= fail("orc_subhalos", rc);
        free(sub);
        free(t_count);
        free(t_peak);
        free(t_pd);
        free(t_par);
    }
    printf("case n=%lld periodic=%d n_dens=%d ids=%d padded=%d: chains %lld, groups %lld\n",
           (long long)n, periodic, n_dens, with_ids, with_padded, (long long)a.counts[0],
           (long long)a.counts[2]);
    free(row_hash);
    free(r2max);
    free_out(&a);
    free_out(&b);
    free_out(&c);
    free(pos);
    free(id);
    free(padded);
    return bad;
}

int main(void)
{
    int bad = 0;
    bad |= run_case(3000, 1, 64, 64, 0, 0, 1);
    bad |= run_case(2500, 0, 64, 32, 1, 1, 2);
    bad |= run_case(1500, 1, 128, 100, 1, 0, 3);
    bad |= run_case(129, 1, 128, 128, 0, 0, 4); /* barely more particles than N_dens */
    /* argument checks: fewer particles than N_dens, misordered sizes */
    {
        uint32_t pos[3 * 8] = {0};
        double dens[8];
        int32_t i32[8 * 64];
        int64_t i64[8], counts[3];
        if (orc_run(8, pos, NULL, NULL, 1, GRID_BITS, 64, 16, 4, 64, 80.0, 200.0, 240.0, 1.0, 0, 1,
                    dens, i32, i32, i32, i32, i32, i64, i32, dens, counts) == 0) {
            fprintf(stderr, "asan driver: n < n_dens accepted\n");
            bad = 1;
        }
        if (orc_run(8, pos, NULL, NULL, 1, GRID_BITS, 4, 4, 8, 4, 80.0, 200.0, 240.0, 1.0, 0, 1,
                    dens, i32, i32, i32, i32, i32, i64, i32, dens, counts) == 0) {
            fprintf(stderr, "asan driver: n_merge > n_hop accepted\n");
            bad = 1;
        }
    }
    if (!bad) printf("asan driver: ok\n");
    return bad;
}
