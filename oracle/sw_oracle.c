/*
 * sw_oracle.c -- plain, single-threaded CPU oracle of the Swendsen-Wang sweep.
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark.  The product library never includes,
 * links or calls it, and it shares no code with the HIP path.
 *
 * It follows the three steps of the SW update as the paper lists them in
 * Sec. 2: (1) active-bond generation, (2) cluster labelling, (3) a random new
 * state for every cluster, for the Hamiltonians of Sec. 1: Eq. (1) Ising,
 * Eq. (2) q-state Potts, Eq. (3) classical XY (embedded-cluster projection).
 * Written for clarity, not speed; double precision throughout except where
 * the state itself is stored (FP32 XY angles).
 *
 * Readings where the paper is silent or garbled (each is also recorded in the
 * design notes of the repository):
 *   R1  bond probability: the printed exponent has lost its minus sign;
 *       Ising uses p = 1 - exp(-2J/T).
 *   R2  Potts: with H = -J sum (delta - 1) the energy gap between an unlike and
 *       a like pair is J, so the Fortuin-Kasteleyn probability is
 *       p = 1 - exp(-J/T).  This is the reading under which the Potts critical
 *       point sits at T = 1/ln(1 + sqrt q); it is pinned by exact enumeration.
 *   R3  Potts states are stored as 0..q-1 instead of 1..q.
 *   R4  XY is the continuous model (FP32 angles), not the 512-state clock; the
 *       mirror direction is a random angle phi, drawn once per sweep, the
 *       same for every site (Sec. 2, the "ispr" paragraph).
 *   R5  "set randomly" (step 3): the new state of a cluster is drawn
 *       independently of its old state; XY reflects a cluster with
 *       probability 1/2.
 *   R6  labels: the fixed point of label equivalence, i.e. the minimum site
 *       index of the cluster.
 *   R7  random numbers: Philox4x32-10 in place of the paper's LCG (the paper
 *       allows any generator).  Word w of stream (tag, n) for replica r and
 *       seed s is output lane (w mod 4) of Philox(counter = (w div 4, n, tag,
 *       r), key = (s mod 2^32, s div 2^32)).  n is the 0-based sweep index,
 *       cumulative over calls.  Tags: BOND 0, BOND_Z 1, BOND_TIE 2,
 *       CLUSTER 3, GLOBAL 4, INIT 5.  Site (x, y, z) of an L^d lattice has
 *       row-major index g = x + L (y + L z).  Bond and Potts words are laid
 *       out by columns: the Philox block with counter word
 *       b = x + L (floor(y/4) + ceil(L/4) z) holds, in lanes 0..3, the words
 *       of the sites (x, 4 floor(y/4) + 0..3, z).  The uniform of bond
 *       (g, mu) is the 32-bit number U = P * 2^16 + S: the primary P is the
 *       high (x) or low (y) half of that BOND word; for z it is the high (y
 *       even) or low (y odd) half of lane floor((y mod 8)/2) of the BOND_Z
 *       block b = x + L (floor(y/8) + ceil(L/8) z); the secondary S is the
 *       high half of word d*g + mu of BOND_TIE.  Cluster decisions: Ising,
 *       XY and Potts with q = 2 take bit (g mod 32) of word g/32 of CLUSTER
 *       for the cluster labelled g; Potts with q >= 3 takes the CLUSTER word
 *       of site g in the column layout of the bond words.
 *   R8  a bond is active iff the pair is aligned and u < p with strict <;
 *       u = word * 2^-32, compared exactly as the integer test word < thr
 *       with thr = floor(p * 2^32).
 *   R9  J = k_B = 1, beta = 1/T; any L >= 3 (the paper's multiple of 32 is a
 *       constraint of its kernels, not of the method).
 *   R13 the q-state clock model, the paper's own XY path (Sec. 2, XY
 *       paragraph; Sec. 3 uses q = 512): integer states p in [0, q), spin
 *       angle 2 pi p / q, q even and at most 512 (the paper's table limit),
 *       H = -J sum cos(2 pi (p_i - p_j) / q) (Eq. (3) on the clock angles).
 *       The random mirror direction `ispr` is the axis index
 *       r = floor(w q / 2^32) of word 0 of GLOBAL at the sweep, the axis at
 *       angle phi = pi r / q (the q axes that map the clock onto itself; the
 *       half-step axes are needed, else the parity of p would never change).
 *       Projection sigma = cos(theta - phi) = cos(pi a / q) with
 *       a = (2 p - r) mod 2q, taken from one table c[m] = cos(pi m / q),
 *       0 <= m < q/2: fold a to a1 = min(a, 2q - a); sigma = c[a1] for
 *       a1 < q/2, 0 for a1 = q/2, -c[q - a1] beyond.  A bond is active iff
 *       both projections are nonzero with equal signs and U < thr(m_i, m_j),
 *       thr = floor(p 2^32) (capped at 2^32 - 1) with
 *       p = -expm1(-(2 beta) (c[m_i] c[m_j])): an integer test, like Ising's.
 *       A cluster is mirrored with probability 1/2 (decision bit as XY):
 *       p -> (q/2 + r - p) mod q, the image of theta -> pi + 2 phi - theta.
 *       Measured: E with the paper's energy table rule[k] = cos(2 pi k / q)
 *       over k = (p_i - p_j) mod q, and Mx, My from cos, sin of 2 pi p / q.
 */
#include "sw_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static const double TWO_PI_D = 6.283185307179586476925286766559;
static const double PI_D = 3.141592653589793238462643383279;

/* ------------------------------------------------------------------------ */
/* Random numbers (R7).  Philox4x32-10 as published by Salmon, Moraes, Dror  */
/* and Shaw (SC'11): ten rounds of two 32x32->64 multiplications, with the   */
/* Weyl key schedule between rounds.                                          */
/* ------------------------------------------------------------------------ */
void swo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

uint32_t swo_word(uint64_t seed, uint32_t rep, uint32_t tag, uint32_t sweep, uint64_t w)
{
    uint32_t ctr[4] = {(uint32_t)(w >> 2), sweep, tag, rep};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t out[4];
    swo_philox4x32_10(ctr, key, out);
    return out[w & 3u];
}

/* Word of site (x, y, z) in the column layout of R7: lane (y mod 4) of the
 * block x + L (floor(y/4) + ceil(L/4) z) of stream (tag, sweep). */
static uint32_t column_word(uint64_t seed, uint32_t rep, uint32_t tag, uint32_t sweep, int L,
                            uint64_t x, uint64_t y, uint64_t z)
{
    uint64_t q4 = ((uint64_t)L + 3) / 4;
    uint64_t block = x + (uint64_t)L * (y / 4 + q4 * z);
    return swo_word(seed, rep, tag, sweep, 4 * block + (y % 4));
}

uint32_t swo_bond_uniform(uint64_t seed, uint32_t rep, uint32_t sweep, int dim, int L, uint64_t g,
                          int mu)
{
    uint64_t x = g % (uint64_t)L, y = (g / (uint64_t)L) % (uint64_t)L;
    uint64_t z = (dim == 3) ? g / ((uint64_t)L * (uint64_t)L) : 0;
    uint32_t p;
    if (mu < 2) {
        uint32_t w = column_word(seed, rep, SWO_TAG_BOND, sweep, L, x, y, z);
        p = (mu == 0) ? (w >> 16) : (w & 0xffffu);
    } else {
        uint64_t q8 = ((uint64_t)L + 7) / 8;
        uint64_t block = x + (uint64_t)L * (y / 8 + q8 * z);
        uint32_t w = swo_word(seed, rep, SWO_TAG_BOND_Z, sweep, 4 * block + (y % 8) / 2);
        p = (y % 2) ? (w & 0xffffu) : (w >> 16);
    }
    uint32_t s = swo_word(seed, rep, SWO_TAG_BOND_TIE, sweep, (uint64_t)dim * g + (uint64_t)mu) >> 16;
    return (p << 16) | s;
}

uint32_t swo_cluster_decision(int model, int q, uint64_t seed, uint32_t rep, uint32_t sweep,
                              int dim, int L, uint64_t g)
{
    if (model == SWO_POTTS && q > 2) {
        uint64_t x = g % (uint64_t)L, y = (g / (uint64_t)L) % (uint64_t)L;
        uint64_t z = (dim == 3) ? g / ((uint64_t)L * (uint64_t)L) : 0;
        uint32_t w = column_word(seed, rep, SWO_TAG_CLUSTER, sweep, L, x, y, z);
        return (uint32_t)(((uint64_t)w * (uint64_t)q) >> 32);
    }
    uint32_t w = swo_word(seed, rep, SWO_TAG_CLUSTER, sweep, g >> 5);
    return (w >> (g & 31u)) & 1u;
}

/* ------------------------------------------------------------------------ */
/* Lattice helpers.                                                           */
/* ------------------------------------------------------------------------ */
static int64_t num_sites(int dim, int L)
{
    int64_t n = 1;
    for (int k = 0; k < dim; ++k) n *= L;
    return n;
}

/* +mu neighbour of site i with periodic boundaries (Sec. 1). */
static int64_t neighbour(int dim, int L, int64_t i, int mu)
{
    int64_t x = i % L;
    int64_t y = (i / L) % L;
    int64_t z = (dim == 3) ? i / ((int64_t)L * L) : 0;
    if (mu == 0) x = (x + 1) % L;
    else if (mu == 1) y = (y + 1) % L;
    else z = (z + 1) % L;
    return x + (int64_t)L * (y + (int64_t)L * z);
}

/* ------------------------------------------------------------------------ */
/* Bond probability (R1, R2, R8).                                             */
/* ------------------------------------------------------------------------ */
uint64_t swo_threshold(int model, double beta)
{
    double p = (model == SWO_ISING) ? -expm1(-2.0 * beta) : -expm1(-beta);
    if (!(p > 0.0)) return 0;
    return (uint64_t)floor(ldexp(p, 32));
}

/* ------------------------------------------------------------------------ */
/* Hot start (the paper's spinset kernel: a random initial configuration).    */
/* ------------------------------------------------------------------------ */
static float xy_angle_from_unit(double u01)
{
    /* u01 in [0,1); one rounding to double, one to float; the float image
     * of 2pi wraps to 0 so that every stored angle is in [0, (float)2pi). */
    double t = u01 * TWO_PI_D;
    float f = (float)t;
    if (f >= (float)TWO_PI_D) f = 0.0f;
    return f;
}

void swo_init_state(int model, int dim, int L, int q, uint64_t seed, uint32_t rep, void *state)
{
    int64_t N = num_sites(dim, L);
    for (int64_t i = 0; i < N; ++i) {
        uint32_t w = swo_word(seed, rep, SWO_TAG_INIT, 0, (uint64_t)i);
        if (model == SWO_ISING) {
            ((int8_t *)state)[i] = (w >> 31) ? (int8_t)-1 : (int8_t)1;
        } else if (model == SWO_POTTS) {
            ((uint8_t *)state)[i] = (uint8_t)(((uint64_t)w * (uint64_t)q) >> 32);
        } else if (model == SWO_CLOCK) {
            ((uint16_t *)state)[i] = (uint16_t)(((uint64_t)w * (uint64_t)q) >> 32);
        } else {
            ((float *)state)[i] = xy_angle_from_unit((double)w * 0x1p-32);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* XY embedding direction (R4): a uniform angle from 53 random bits.          */
/* ------------------------------------------------------------------------ */
double swo_xy_phi(uint64_t seed, uint32_t rep, uint32_t sweep)
{
    uint32_t w0 = swo_word(seed, rep, SWO_TAG_GLOBAL, sweep, 0);
    uint32_t w1 = swo_word(seed, rep, SWO_TAG_GLOBAL, sweep, 1);
    double u = ((double)(w0 >> 5) * 67108864.0 + (double)(w1 >> 6)) * 0x1p-53;
    return TWO_PI_D * u;
}

/* ------------------------------------------------------------------------ */
/* Clock model (R13): mirror axis, projections, bond thresholds, mirror.      */
/* ------------------------------------------------------------------------ */
uint32_t swo_clock_axis(uint64_t seed, uint32_t rep, uint32_t sweep, int q)
{
    uint32_t w = swo_word(seed, rep, SWO_TAG_GLOBAL, sweep, 0);
    return (uint32_t)(((uint64_t)w * (uint64_t)q) >> 32);
}

/* cos(pi m / q), the projection of a clock spin at angular distance m pi / q
 * from the axis, 0 <= m < q/2. */
static double clock_c(int q, int m)
{
    return cos((PI_D * (double)m) / (double)q);
}

/* Fold the projection index a = (2p - r) mod 2q: *m in [0, q/2] and the sign
 * of sigma (+1, -1, or 0 when the spin is perpendicular to the axis). */
void swo_clock_projection(int q, uint32_t p, uint32_t r, int *m, int *sign)
{
    int a = (int)((2u * p + 2u * (uint32_t)q - r) % (2u * (uint32_t)q));
    int a1 = a <= q ? a : 2 * q - a;
    if (2 * a1 < q) {
        *m = a1;
        *sign = 1;
    } else if (2 * a1 == q) {
        *m = q / 2;
        *sign = 0;
    } else {
        *m = q - a1;
        *sign = -1;
    }
}

uint64_t swo_clock_threshold(int q, double beta, int m1, int m2)
{
    double x = (2.0 * beta) * (clock_c(q, m1) * clock_c(q, m2));
    double p = -expm1(-x);
    if (!(p > 0.0)) return 0;
    double t = floor(ldexp(p, 32));
    return t >= 4294967295.0 ? 4294967295ull : (uint64_t)t;
}

uint16_t swo_clock_mirror(int q, uint32_t p, uint32_t r)
{
    return (uint16_t)(((uint32_t)(q / 2) + r + (uint32_t)q - p) % (uint32_t)q);
}

/* ------------------------------------------------------------------------ */
/* Step (1): active-bond generation (Sec. 2).                                 */
/*   Ising/Potts: aligned pair and u < p.                                     */
/*   XY: project on the mirror direction, sigma = cos(theta - phi); the       */
/*   embedded Ising coupling is J sigma_i sigma_j, so the bond is active with */
/*   probability 1 - exp(-2 beta sigma_i sigma_j) when that product is        */
/*   positive (Wolff's embedded cluster).  Evaluated as                       */
/*   u < -expm1(-((2 beta sigma_i) sigma_j)) in that order.                   */
/* ------------------------------------------------------------------------ */
int64_t swo_bonds(int model, int dim, int L, int q, double beta, uint64_t seed, uint32_t rep,
                  uint32_t sweep, const void *state, uint8_t *bonds)
{
    int64_t N = num_sites(dim, L);
    int64_t active = 0;
    double *sigma = NULL;
    double two_beta = 2.0 * beta;
    uint64_t thr = 0;
    uint32_t axis = 0;
    if (model == SWO_CLOCK) {
        axis = swo_clock_axis(seed, rep, sweep, q);
    } else if (model == SWO_XY) {
        double phi = swo_xy_phi(seed, rep, sweep);
        const float *th = (const float *)state;
        sigma = (double *)malloc(sizeof(double) * (size_t)N);
        for (int64_t i = 0; i < N; ++i) sigma[i] = cos((double)th[i] - phi);
    } else {
        thr = swo_threshold(model, beta);
    }
    for (int64_t i = 0; i < N; ++i) {
        uint8_t b = 0;
        for (int mu = 0; mu < dim; ++mu) {
            int64_t j = neighbour(dim, L, i, mu);
            uint32_t w = swo_bond_uniform(seed, rep, sweep, dim, L, (uint64_t)i, mu);
            int on;
            if (model == SWO_ISING) {
                const int8_t *s = (const int8_t *)state;
                on = (s[i] == s[j]) && ((uint64_t)w < thr);
            } else if (model == SWO_POTTS) {
                const uint8_t *s = (const uint8_t *)state;
                on = (s[i] == s[j]) && ((uint64_t)w < thr);
            } else if (model == SWO_CLOCK) {
                const uint16_t *s = (const uint16_t *)state;
                int mi, si, mj, sj;
                swo_clock_projection(q, s[i], axis, &mi, &si);
                swo_clock_projection(q, s[j], axis, &mj, &sj);
                on = si != 0 && si == sj && (uint64_t)w < swo_clock_threshold(q, beta, mi, mj);
            } else {
                double x = (two_beta * sigma[i]) * sigma[j];
                double p = -expm1(-x);
                double u = (double)w * 0x1p-32;
                on = u < p;
            }
            if (on) {
                b |= (uint8_t)(1u << mu);
                ++active;
            }
        }
        bonds[i] = b;
    }
    free(sigma);
    return active;
}

/* ------------------------------------------------------------------------ */
/* Step (2): cluster labelling (R6).                                          */
/* Method A: union-find (the Hoshen-Kopelman family the paper cites for the   */
/* CPU), linking the larger root under the smaller so that every root is the */
/* minimum of its set.                                                        */
/* ------------------------------------------------------------------------ */
static int64_t uf_find(int32_t *par, int64_t a)
{
    while (par[a] != a) {
        par[a] = par[par[a]]; /* path halving */
        a = par[a];
    }
    return a;
}

void swo_labels_uf(int dim, int L, const uint8_t *bonds, int32_t *labels)
{
    int64_t N = num_sites(dim, L);
    for (int64_t i = 0; i < N; ++i) labels[i] = (int32_t)i;
    for (int64_t i = 0; i < N; ++i) {
        for (int mu = 0; mu < dim; ++mu) {
            if (!(bonds[i] >> mu & 1u)) continue;
            int64_t j = neighbour(dim, L, i, mu);
            int64_t a = uf_find(labels, i), b = uf_find(labels, j);
            if (a == b) continue;
            if (a < b) labels[b] = (int32_t)a;
            else labels[a] = (int32_t)b;
        }
    }
    for (int64_t i = 0; i < N; ++i) labels[i] = (int32_t)uf_find(labels, i);
}

/* Method B: breadth-first search from every unvisited site in increasing
 * index order, so the seed of each search is its cluster's minimum index. */
void swo_labels_bfs(int dim, int L, const uint8_t *bonds, int32_t *labels)
{
    int64_t N = num_sites(dim, L);
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    for (int64_t i = 0; i < N; ++i) labels[i] = -1;
    for (int64_t s = 0; s < N; ++s) {
        if (labels[s] >= 0) continue;
        int64_t head = 0, tail = 0;
        labels[s] = (int32_t)s;
        queue[tail++] = s;
        while (head < tail) {
            int64_t i = queue[head++];
            int64_t x = i % L, y = (i / L) % L, z = (dim == 3) ? i / ((int64_t)L * L) : 0;
            for (int mu = 0; mu < dim; ++mu) {
                /* +mu neighbour through bonds[i] */
                int64_t jp = neighbour(dim, L, i, mu);
                if ((bonds[i] >> mu & 1u) && labels[jp] < 0) {
                    labels[jp] = (int32_t)s;
                    queue[tail++] = jp;
                }
                /* -mu neighbour through its own +mu bond */
                int64_t xm = x, ym = y, zm = z;
                if (mu == 0) xm = (x + L - 1) % L;
                else if (mu == 1) ym = (y + L - 1) % L;
                else zm = (z + L - 1) % L;
                int64_t jm = xm + (int64_t)L * (ym + (int64_t)L * zm);
                if ((bonds[jm] >> mu & 1u) && labels[jm] < 0) {
                    labels[jm] = (int32_t)s;
                    queue[tail++] = jm;
                }
            }
        }
    }
    free(queue);
}

/* ------------------------------------------------------------------------ */
/* Step (3): every cluster is set to a random state (R5).  The decision of a */
/* cluster is drawn from the CLUSTER stream at its label (its minimum site    */
/* index, R7), so all sites of the cluster see the same outcome.              */
/*   Ising: +1 or -1.  Potts: uniform in [0,q).                               */
/*   XY: with probability 1/2 the cluster is reflected in the line normal to  */
/*   the direction phi, s -> s - 2 (s.r) r, i.e. theta -> pi + 2 phi - theta, */
/*   wrapped into [0, 2pi) in double and then rounded to float.               */
/* ------------------------------------------------------------------------ */
static float xy_reflect(float theta, double phi)
{
    double v = (PI_D + 2.0 * phi) - (double)theta;
    if (v >= TWO_PI_D) v -= TWO_PI_D;
    if (v >= TWO_PI_D) v -= TWO_PI_D;
    if (v < 0.0) v += TWO_PI_D;
    float f = (float)v;
    if (f >= (float)TWO_PI_D) f = 0.0f;
    return f;
}

void swo_set_clusters(int model, int dim, int L, int q, uint64_t seed, uint32_t rep,
                      uint32_t sweep, const int32_t *labels, void *state)
{
    int64_t N = num_sites(dim, L);
    double phi = (model == SWO_XY) ? swo_xy_phi(seed, rep, sweep) : 0.0;
    uint32_t axis = (model == SWO_CLOCK) ? swo_clock_axis(seed, rep, sweep, q) : 0u;
    for (int64_t i = 0; i < N; ++i) {
        uint32_t dec = swo_cluster_decision(model, q, seed, rep, sweep, dim, L, (uint64_t)labels[i]);
        if (model == SWO_ISING) {
            ((int8_t *)state)[i] = dec ? (int8_t)-1 : (int8_t)1;
        } else if (model == SWO_POTTS) {
            ((uint8_t *)state)[i] = (uint8_t)dec;
        } else if (model == SWO_CLOCK) {
            uint16_t *p = (uint16_t *)state;
            if (dec) p[i] = swo_clock_mirror(q, p[i], axis);
        } else if (dec) {
            float *th = (float *)state;
            th[i] = xy_reflect(th[i], phi);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Measurement (Sec. 2: M = sum s and the energy of Eq. (1); Eq. (5) for the */
/* Potts M^2; Eq. (3) for XY).                                                */
/* ------------------------------------------------------------------------ */
void swo_measure(int model, int dim, int L, int q, const void *state, double *energy,
                 double *mx, double *my, int64_t *aligned, int64_t *counts)
{
    int64_t N = num_sites(dim, L);
    double e = 0.0, sx = 0.0, sy = 0.0;
    int64_t al = 0;
    if (model == SWO_ISING) {
        const int8_t *s = (const int8_t *)state;
        int64_t m = 0, pair_sum = 0;
        for (int64_t i = 0; i < N; ++i) {
            m += s[i];
            for (int mu = 0; mu < dim; ++mu) {
                int64_t j = neighbour(dim, L, i, mu);
                pair_sum += (int64_t)s[i] * (int64_t)s[j];
                if (s[i] == s[j]) ++al;
            }
        }
        e = -(double)pair_sum;
        sx = (double)m;
    } else if (model == SWO_POTTS) {
        const uint8_t *s = (const uint8_t *)state;
        int64_t *n = (int64_t *)calloc((size_t)q, sizeof(int64_t));
        int64_t unlike = 0;
        for (int64_t i = 0; i < N; ++i) {
            n[s[i]] += 1;
            for (int mu = 0; mu < dim; ++mu) {
                int64_t j = neighbour(dim, L, i, mu);
                if (s[i] == s[j]) ++al;
                else ++unlike;
            }
        }
        e = (double)unlike; /* H = -J sum (delta - 1) */
        double sum_sq = 0.0;
        for (int k = 0; k < q; ++k) sum_sq += (double)n[k] * (double)n[k];
        sx = ((double)q * sum_sq - (double)N * (double)N) / (double)(q - 1);
        if (counts)
            for (int k = 0; k < q; ++k) counts[k] = n[k];
        free(n);
    } else if (model == SWO_CLOCK) {
        const uint16_t *p = (const uint16_t *)state;
        double *rule = (double *)malloc(sizeof(double) * (size_t)q);
        double *sn = (double *)malloc(sizeof(double) * (size_t)q);
        for (int k = 0; k < q; ++k) {
            rule[k] = cos((TWO_PI_D * (double)k) / (double)q);
            sn[k] = sin((TWO_PI_D * (double)k) / (double)q);
        }
        for (int64_t i = 0; i < N; ++i) {
            sx += rule[p[i]];
            sy += sn[p[i]];
            for (int mu = 0; mu < dim; ++mu) {
                int64_t j = neighbour(dim, L, i, mu);
                e -= rule[((int)p[i] - (int)p[j] + q) % q];
            }
        }
        free(rule);
        free(sn);
    } else {
        const float *th = (const float *)state;
        for (int64_t i = 0; i < N; ++i) {
            sx += cos((double)th[i]);
            sy += sin((double)th[i]);
            for (int mu = 0; mu < dim; ++mu) {
                int64_t j = neighbour(dim, L, i, mu);
                e -= cos((double)th[i] - (double)th[j]);
            }
        }
    }
    if (energy) *energy = e;
    if (mx) *mx = sx;
    if (my) *my = sy;
    if (aligned) *aligned = al;
}

void swo_cluster_stats(int64_t N, const int32_t *labels, int64_t out[3])
{
    int64_t *size = (int64_t *)calloc((size_t)N, sizeof(int64_t));
    for (int64_t i = 0; i < N; ++i) size[labels[i]] += 1;
    int64_t nc = 0, mx = 0, s2 = 0;
    for (int64_t i = 0; i < N; ++i) {
        if (size[i] == 0) continue;
        ++nc;
        if (size[i] > mx) mx = size[i];
        s2 += size[i] * size[i];
    }
    free(size);
    out[0] = nc;
    out[1] = mx;
    out[2] = s2;
}

/* ------------------------------------------------------------------------ */
/* Whole sweeps: measure, (1) bonds, (2) labels, (3) new cluster states.      */
/* ------------------------------------------------------------------------ */
void swo_sweeps(int model, int dim, int L, int q, double beta, uint64_t seed, uint32_t rep,
                uint32_t n0, int64_t nsweeps, void *state, double *rec_energy, double *rec_mx,
                double *rec_my, int64_t *rec_aligned, int64_t *rec_counts, uint8_t *bonds_last,
                int32_t *labels_last)
{
    int64_t N = num_sites(dim, L);
    uint8_t *bonds = (uint8_t *)malloc((size_t)N);
    int32_t *labels = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    for (int64_t k = 0; k < nsweeps; ++k) {
        uint32_t n = n0 + (uint32_t)k;
        if (rec_energy || rec_mx || rec_my || rec_aligned || rec_counts) {
            double e, x, y;
            int64_t al;
            swo_measure(model, dim, L, q, state, &e, &x, &y, &al,
                        (rec_counts && model == SWO_POTTS) ? rec_counts + k * q : NULL);
            if (rec_energy) rec_energy[k] = e;
            if (rec_mx) rec_mx[k] = x;
            if (rec_my) rec_my[k] = y;
            if (rec_aligned) rec_aligned[k] = al;
        }
        swo_bonds(model, dim, L, q, beta, seed, rep, n, state, bonds);
        swo_labels_uf(dim, L, bonds, labels);
        swo_set_clusters(model, dim, L, q, seed, rep, n, labels, state);
    }
    if (bonds_last && nsweeps > 0) memcpy(bonds_last, bonds, (size_t)N);
    if (labels_last && nsweeps > 0) memcpy(labels_last, labels, sizeof(int32_t) * (size_t)N);
    free(bonds);
    free(labels);
}
