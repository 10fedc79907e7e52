/*
 * sw_oracle.h -- plain, single-threaded CPU oracle for the Swendsen-Wang
 * multi-cluster sweep (Komura & Okabe, "CUDA programs for GPU computing of
 * Swendsen-Wang multi-cluster spin flip algorithm: 2D and 3D Ising, Potts,
 * and XY models").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this code; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code with the HIP path.
 *
 * Conventions (the readings of the paper are listed beside each function in
 * sw_oracle.c):
 *   lattice  d in {2,3}, linear size L >= 3, periodic, N = L^d sites,
 *            site index i = x + L*(y + L*z), x fastest.
 *   bonds    bonds[i] bit mu = bond between i and its +mu neighbour.
 *   states   Ising: int8 +1/-1.  Potts: uint8 in [0,q).  XY: float angle in
 *            [0, (float)2pi).  Clock (q even, <= 512): uint16 p in [0,q),
 *            angle 2 pi p / q.
 *   labels   int32, label[i] = minimum site index of i's cluster.
 */
#ifndef SW_ORACLE_H
#define SW_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { SWO_ISING = 0, SWO_POTTS = 1, SWO_XY = 2, SWO_CLOCK = 3 };
enum {
    SWO_TAG_BOND = 0, SWO_TAG_BOND_Z = 1, SWO_TAG_BOND_TIE = 2,
    SWO_TAG_CLUSTER = 3, SWO_TAG_GLOBAL = 4, SWO_TAG_INIT = 5
};

/* Philox4x32-10 block function (Salmon et al., SC'11). */
void swo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Word w of the random stream (tag, sweep) of replica `rep` under `seed`. */
uint32_t swo_word(uint64_t seed, uint32_t rep, uint32_t tag, uint32_t sweep, uint64_t w);

/* The 32-bit uniform of bond (g, mu) of an L^dim lattice at sweep n:
 * (P << 16) | S with the 16-bit primary P and the 16-bit secondary S (see
 * sw_oracle.c, R7). */
uint32_t swo_bond_uniform(uint64_t seed, uint32_t rep, uint32_t sweep, int dim, int L, uint64_t g,
                          int mu);

/* Random decision of the cluster whose label is g: Ising/XY/Potts(q=2) use
 * one bit, Potts q >= 3 a new state in [0,q). */
uint32_t swo_cluster_decision(int model, int q, uint64_t seed, uint32_t rep, uint32_t sweep,
                              int dim, int L, uint64_t g);

/* Bond threshold for Ising (model 0) and Potts (model 1): floor(p * 2^32). */
uint64_t swo_threshold(int model, double beta);

/* Hot start: every state drawn from the INIT stream. */
void swo_init_state(int model, int dim, int L, int q, uint64_t seed, uint32_t rep,
                    void *state);

/* Embedding direction of the XY update at sweep n. */
double swo_xy_phi(uint64_t seed, uint32_t rep, uint32_t sweep);

/* Clock model: mirror axis index r of sweep n, the folded projection of
 * state p on it (index m into cos(pi m / q) and its sign), the integer bond
 * threshold of two projections, and the mirror image of p. */
uint32_t swo_clock_axis(uint64_t seed, uint32_t rep, uint32_t sweep, int q);
void swo_clock_projection(int q, uint32_t p, uint32_t r, int *m, int *sign);
uint64_t swo_clock_threshold(int q, double beta, int m1, int m2);
uint16_t swo_clock_mirror(int q, uint32_t p, uint32_t r);

/* Step (1): bond lattice for sweep n from `state`; returns #active bonds. */
int64_t swo_bonds(int model, int dim, int L, int q, double beta, uint64_t seed,
                  uint32_t rep, uint32_t sweep, const void *state, uint8_t *bonds);

/* Step (2): minimum-index cluster labels, two independent methods. */
void swo_labels_uf(int dim, int L, const uint8_t *bonds, int32_t *labels);
void swo_labels_bfs(int dim, int L, const uint8_t *bonds, int32_t *labels);

/* Step (3): every cluster takes a new random state (in place). */
void swo_set_clusters(int model, int dim, int L, int q, uint64_t seed, uint32_t rep,
                      uint32_t sweep, const int32_t *labels, void *state);

/* Observables of one configuration.
 *   energy : H with J = 1 (Ising -sum s s; Potts sum (1 - delta); XY and
 *            clock -sum cos)
 *   mx, my : Ising (sum s, 0); Potts (M^2 of the Potts definition, 0);
 *            XY and clock (sum cos, sum sin)
 *   aligned: number of bonds joining equal states (Ising/Potts), else 0
 *   counts : Potts only, q entries n[k] (may be NULL) */
void swo_measure(int model, int dim, int L, int q, const void *state, double *energy,
                 double *mx, double *my, int64_t *aligned, int64_t *counts);

/* Cluster statistics of a label array: #clusters, largest size, sum of sizes^2. */
void swo_cluster_stats(int64_t N, const int32_t *labels, int64_t out[3]);

/* `nsweeps` whole sweeps n0 .. n0+nsweeps-1 in place on `state`.  Before
 * sweep n0+k the configuration is measured into rec_*[k] (any may be NULL;
 * rec_counts holds q entries per sweep).  bonds_last / labels_last (may be
 * NULL) receive the bonds and labels of the last sweep. */
void swo_sweeps(int model, int dim, int L, int q, double beta, uint64_t seed, uint32_t rep,
                uint32_t n0, int64_t nsweeps, void *state, double *rec_energy,
                double *rec_mx, double *rec_my, int64_t *rec_aligned, int64_t *rec_counts,
                uint8_t *bonds_last, int32_t *labels_last);

#ifdef __cplusplus
}
#endif
#endif
