/*
 * Drives every entry point of the CPU oracle over small lattices of each
 * model (odd sizes, so the four-row column blocks of the random stream have
 * ragged ends; q at its limits; beta at 0 and far above the transition) so
 * that a build with AddressSanitizer and UndefinedBehaviorSanitizer sees
 * every array access and every integer operation the oracle makes.
 * Also checks that the two labellers agree on the last sweep's bonds.
 * Exit status 0 and the line "oracle sanitize: ok" on success.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/sw_oracle.h"

static int64_t sites(int dim, int L) { return dim == 2 ? (int64_t)L * L : (int64_t)L * L * L; }

static size_t state_bytes(int model) { return model == SWO_ISING || model == SWO_POTTS ? 1 : (model == SWO_XY ? 4 : 2); }

static int run_case(int model, int dim, int L, int q, double beta, uint64_t seed)
{
    const int64_t N = sites(dim, L);
    const int64_t ns = 4;
    /* exact-size heap blocks: any access past an end is a sanitizer report */
    void *state = malloc((size_t)N * state_bytes(model));
    uint8_t *bonds = malloc((size_t)N);
    int32_t *labels = malloc((size_t)N * 4);
    int32_t *labels2 = malloc((size_t)N * 4);
    double *re = malloc(ns * 8), *rx = malloc(ns * 8), *ry = malloc(ns * 8);
    int64_t *ra = malloc(ns * 8);
    const int nq = model == SWO_POTTS ? q : 1;
    int64_t *rc = malloc((size_t)(ns * nq) * 8);
    int64_t *counts = malloc((size_t)nq * 8);
    swo_init_state(model, dim, L, q, seed, 1u, state);
    swo_sweeps(model, dim, L, q, beta, seed, 1u, 0u, ns, state, re, rx, ry, ra, model == SWO_POTTS ? rc : NULL,
               bonds, labels);
    swo_labels_bfs(dim, L, bonds, labels2);
    int bad = memcmp(labels, labels2, (size_t)N * 4) != 0;
    swo_labels_uf(dim, L, bonds, labels2);
    bad |= memcmp(labels, labels2, (size_t)N * 4) != 0;
    int64_t cs[3];
    swo_cluster_stats(N, labels, cs);
    double e, mx, my;
    int64_t al;
    swo_measure(model, dim, L, q, state, &e, &mx, &my, &al, model == SWO_POTTS ? counts : NULL);
    /* a lone step of each kind, on the evolved state */
    (void)swo_bonds(model, dim, L, q, beta, seed, 1u, ns, state, bonds);
    swo_labels_uf(dim, L, bonds, labels);
    swo_set_clusters(model, dim, L, q, seed, 1u, ns, labels, state);
    for (int64_t g = 0; g < N; ++g)
        (void)swo_cluster_decision(model, q, seed, 1u, ns, dim, L, (uint64_t)g);
    if (bad) fprintf(stderr, "labellers disagree: model %d dim %d L %d q %d\n", model, dim, L, q);
    free(state), free(bonds), free(labels), free(labels2), free(re), free(rx), free(ry), free(ra), free(rc),
        free(counts);
    return bad;
}

int main(void)
{
    int bad = 0;
    const double betas[3] = {0.0, 0.6, 30.0};
    for (int b = 0; b < 3; ++b) {
        const double be = betas[b];
        bad |= run_case(SWO_ISING, 2, 3, 2, be, 1);
        bad |= run_case(SWO_ISING, 2, 7, 2, be, 2);
        bad |= run_case(SWO_ISING, 3, 3, 2, be, 3);
        bad |= run_case(SWO_ISING, 3, 5, 2, be, 4);
        bad |= run_case(SWO_POTTS, 2, 5, 2, be, 5);
        bad |= run_case(SWO_POTTS, 2, 6, 3, be, 6);
        bad |= run_case(SWO_POTTS, 2, 5, 256, be, 7);
        bad |= run_case(SWO_POTTS, 3, 4, 3, be, 8);
        bad |= run_case(SWO_XY, 2, 5, 0, be, 9);
        bad |= run_case(SWO_XY, 3, 3, 0, be, 10);
        bad |= run_case(SWO_CLOCK, 2, 6, 2, be, 11);
        bad |= run_case(SWO_CLOCK, 2, 5, 4, be, 12);
        bad |= run_case(SWO_CLOCK, 2, 7, 512, be, 13);
        bad |= run_case(SWO_CLOCK, 3, 4, 512, be, 14);
    }
    /* the clock tables over their whole index range */
    for (int q = 2; q <= 512; q += q < 16 ? 2 : 62) {
        for (uint32_t r = 0; r < (uint32_t)q; ++r)
            for (uint32_t p = 0; p < (uint32_t)q; ++p) {
                int m, sg;
                swo_clock_projection(q, p, r, &m, &sg);
                if (m < 0 || m > q / 2) bad = 1;
                if (swo_clock_mirror(q, swo_clock_mirror(q, p, r), r) != p) bad = 1;
            }
        for (int m1 = 0; m1 <= q / 2; ++m1) (void)swo_clock_threshold(q, 30.0, m1, q / 2 - m1);
        (void)swo_clock_axis(7, 0, 3, q);
    }
    (void)swo_threshold(0, 0.0), (void)swo_threshold(0, 1e6), (void)swo_threshold(1, 1e6);
    (void)swo_xy_phi(~0ull, ~0u, ~0u);
    (void)swo_bond_uniform(~0ull, ~0u, ~0u, 3, 3, 26, 2);
    if (bad) return 1;
    printf("oracle sanitize: ok\n");
    return 0;
}
