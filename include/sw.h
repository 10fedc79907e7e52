/*
 * sw.h -- C ABI of the MI355X Swendsen-Wang engine (libswmc.so).
 *
 * The engine runs the Swendsen-Wang multi-cluster update of Komura & Okabe,
 * "CUDA programs for GPU computing of Swendsen-Wang multi-cluster spin flip
 * algorithm: 2D and 3D Ising, Potts, and XY models", for
 *   Ising   (Sec. 1, Eq. (1)),  states int8 +1/-1,
 *   Potts   (Sec. 1, Eq. (2)),  states uint8 in [0,q)  (paper: 1..q),
 *   XY      (Sec. 1, Eq. (3)),  states float angles in [0, (float)2pi),
 *   clock   (the paper's XY path: Sec. 2, XY paragraph; Sec. 3 uses q = 512),
 *           states uint16 p in [0, q), angle 2 pi p / q, q even, <= 512,
 * on 2D square and 3D simple-cubic lattices of linear size L with periodic
 * boundaries.  One sweep is the three steps of Sec. 2: (1) active-bond
 * generation, (2) cluster labelling (label equivalence, fixed point = minimum
 * site index), (3) every cluster set to a random state.  Every step runs in
 * HIP kernels on one GPU.
 *
 * Conventions shared by every call:
 *   site index  i = x + L*(y + L*z), x fastest; N = L^dim.
 *   bond byte   bit mu (0=x,1=y,2=z) = bond between i and its +mu neighbour.
 *   labels      int32, minimum site index of the cluster.
 *   random      Philox4x32-10 (Salmon et al., SC'11; the paper's program
 *               notes in Sec. 2 allow any generator).  Word w of stream
 *               (tag, sweep n) of replica r is lane w%4 of
 *               Philox(counter=(w/4, n, tag, r), key=(seed mod 2^32,
 *               seed div 2^32)); tags: bond 0, bond z 1, bond tie 2,
 *               cluster 3, global 4, init 5.  The sweep index n is 0-based
 *               and cumulative over calls.
 *               Column blocks: for site (x, y, z) the block with counter
 *               word b4 = x + L*(floor(y/4) + ceil(L/4)*z) holds in its lanes
 *               0..3 the words of sites (x, 4*floor(y/4) + 0..3, z).
 *               The 32-bit uniform of bond (i, mu), i = (x, y, z), is
 *               P*2^16 + S.  Primary P: for x the high half, for y the low
 *               half, of lane y%4 of the tag-0 block b4; for z the high
 *               (y even) or low (y odd) half of lane floor((y%8)/2) of the
 *               tag-1 block b8 = x + L*(floor(y/8) + ceil(L/8)*z).
 *               Secondary S: high half of word dim*i+mu of tag 2 (row-major
 *               i; it decides only when P equals the threshold's high half).
 *               A cluster labelled g takes bit g%32 of word g/32 of tag 3
 *               (Ising, XY, Potts q=2: bit set = flip / mirror / state 1),
 *               or, for Potts q>=3, the state floor(w*q/2^32) from the tag-3
 *               word w of site g in the column blocks (lane y%4 of block b4).
 *               The hot start takes word i of tag 5 at n = 0; the XY mirror
 *               angle phi of sweep n takes words 0 and 1 of tag 4 (53 bits).
 *   couplings   J = k_B = 1, beta = 1/T.  Bond probability: Ising
 *               1-exp(-2 beta) (Sec. 2, step (1)), Potts 1-exp(-beta), XY
 *               1-exp(-2 beta sigma_i sigma_j) on the projections
 *               sigma = cos(theta - phi) onto a random direction phi drawn
 *               once per sweep (Sec. 2, embedded-cluster paragraph).
 *   clock       the mirror axis (the paper's `ispr`) of sweep n is
 *               r = floor(w q / 2^32), w = word 0 of tag 4, at angle pi r / q;
 *               sigma = cos(pi a / q), a = (2p - r) mod 2q, folded to
 *               m in [0, q/2] with a sign; a bond needs equal nonzero signs
 *               and U < thr(m_i, m_j) = floor(2^32 (1 - exp(-2 beta
 *               cos(pi m_i/q) cos(pi m_j/q)))) (capped at 2^32 - 1): an
 *               integer test.  A cluster whose decision bit is set is
 *               mirrored, p -> (q/2 + r - p) mod q.  Records hold E (the
 *               paper's rule table cos(2 pi k / q)), sum cos and sum sin.
 *
 * Errors: every int-returning call returns 0 (or a count) on success and a
 * negative SW_E_* code on failure; sw_last_error() gives a message for the
 * calling thread.  Label walks and unions on the device are bounded (by
 * N + 1 steps, which a valid label forest never needs); an iterative
 * labeller is bounded by its iteration cap.  A call whose sweeps hit either
 * bound returns SW_E_NOCONV and that sweep's labels and states are not
 * trustworthy.  Handles are not thread-safe: one thread per handle.
 * All host pointers are owned by the caller and must hold the stated number
 * of elements; calls that take them are synchronous.  Device memory is owned
 * by the library and freed by sw_destroy / sw_batch_destroy.
 */
#ifndef SW_H
#define SW_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum sw_model { SW_ISING = 0, SW_POTTS = 1, SW_XY = 2, SW_CLOCK = 3 };

enum sw_status {
    SW_OK = 0,
    SW_E_INVALID = -1, /* bad argument (model, dim, L, q, beta, sizes, NULL) */
    SW_E_NOMEM = -2,   /* device or host allocation failed */
    SW_E_DEVICE = -3,  /* HIP runtime error (message in sw_last_error) */
    SW_E_NOCONV = -4,  /* labelling did not reach its fixed point within the cap */
    SW_E_BUSY = -5,    /* serving queue full / slot budget exhausted */
    SW_E_NOTFOUND = -6, /* unknown job id */
    SW_E_CANCELLED = -7 /* status of a served job cancelled before its end */
};

typedef struct sw_ctx *sw_handle;

/* Cluster statistics of the last labelling (Sec. 2, step (2)). */
typedef struct {
    int64_t n_clusters;  /* number of clusters */
    int64_t max_cluster; /* size of the largest cluster */
    int64_t sum_c2;      /* sum over clusters of size^2 (improved estimator of M^2) */
} sw_cluster_stats;

/* Observables of one configuration (Sec. 2: M = sum s, energy of Eq. (1);
 * Eq. (5) for the Potts M^2).  `sweep` = number of sweeps done before the
 * configuration was measured (the configuration entering that sweep). */
typedef struct {
    int64_t sweep;
    double energy; /* H with J = 1 */
    double mag;    /* Ising: M = sum s; Potts: sqrt(M^2); XY: |(sum cos, sum sin)| */
    double mag2;   /* M^2 (Potts: Eq. (5)) */
    double mx, my; /* Ising: (M, 0); Potts: (0, 0); XY: (sum cos, sum sin) */
} sw_record;

/* --- plain form: one lattice per handle, one launch per kernel ------------ */

/* Create a lattice and give it a hot start (every state drawn from the INIT
 * stream; the paper's spinset kernel).  model: SW_ISING (q ignored, use 2),
 * SW_POTTS (2 <= q <= 256), SW_XY (q ignored, use 0), SW_CLOCK (even q,
 * 2 <= q <= 512); dim 2 or 3; L >= 3 and
 * L^dim <= 2^31 - 1; beta >= 0 and finite.  Replica 0.  NULL on error. */
sw_handle sw_create(int model, int dim, int L, int q, double beta, uint64_t seed);

/* As sw_create with an explicit replica index (fourth Philox counter word). */
sw_handle sw_create_replica(int model, int dim, int L, int q, double beta, uint64_t seed,
                            uint32_t replica);

/* As sw_create_replica on an explicit tile shape: tile in [0, sw_tile_count)
 * picks the shape of the labelling tiles (Sec. 2, step (2): the local pass
 * works on one tile in on-chip memory), -1 the shape sw_tune recorded for
 * (model, dim, L), else shape 0 (the fastest on large lattices) unless
 * another shape pads the lattice to whole tiles by more than a quarter less
 * (then the one that pads least).  The shape changes the speed, never the
 * trajectory.  NULL on error. */
sw_handle sw_create_tiled(int model, int dim, int L, int q, double beta, uint64_t seed,
                          uint32_t replica, int tile);

/* Number of tile shapes for (model, dim), and the extent (tx, ty, tz) of
 * shape `tile` (tz = 1 in 2D).  Host-only; SW_E_INVALID on bad arguments. */
int sw_tile_count(int model, int dim);
int sw_tile_shape(int model, int dim, int tile, int *tx, int *ty, int *tz);

/* Tile shape index of a handle. */
int sw_get_tile(sw_handle h);

/* Tuner: for every tile shape, create a scratch lattice (model, dim, L, q,
 * beta), run 2 warm-up and `sweeps` timed sweeps (1 .. 100000, HIP events)
 * and record the fastest shape for (model, dim, L) in a process-wide table
 * that later sw_create / sw_create_replica / batch / server lattices of that
 * (model, dim, L) use.  *best receives the shape, ms_per_sweep (if not NULL,
 * sw_tile_count entries) each shape's time.  Synchronous; allocates and frees
 * the scratch lattices.  Thread-safe table; SW_E_* on error. */
int sw_tune(int model, int dim, int L, int q, double beta, int sweeps, int *best,
            double *ms_per_sweep);

/* Run n >= 0 sweeps.  Before each sweep the configuration is measured into
 * the record series (when measuring is on, the default).  Synchronous. */
int sw_sweep(sw_handle h, int64_t n);

/* Averages over the recorded series since the last sw_reset_measure:
 * m2 = <(M/N)^2>, m4 = <(M/N)^4>, energy = <E>/N (any pointer may be NULL),
 * and the cluster statistics of the last labelling (zeros before any sweep).
 * With no records the current configuration alone is measured. */
int sw_measure(sw_handle h, double *m2, double *m4, double *energy, sw_cluster_stats *cs);

/* Moments of the recorded series since the last sw_reset_measure (the
 * current configuration alone when nothing is recorded): the outputs of the
 * paper's program (Sec. 2: <m^2>, <m^4>, energy and specific heat per spin),
 * <|m|>, and the moment ratio of Sec. 3, Eq. (6).  m = M/N with M of Eq. (4)
 * (Ising), sqrt of Eq. (5) (Potts) or |(sum cos, sum sin)| (XY). */
typedef struct {
    int64_t n;            /* records averaged */
    double abs_m;         /* <|m|> */
    double m2, m4;        /* <m^2>, <m^4> */
    double energy;        /* <E>/N */
    double energy2;       /* <(E/N)^2> */
    double specific_heat; /* beta^2 (<E^2> - <E>^2) / N */
    double binder;        /* <m^4> / <m^2>^2 (0 when <m^2> = 0) */
} sw_moments;
int sw_get_moments(sw_handle h, sw_moments *out);

/* Global phase of step (2), the label equivalence across tiles (the bond
 * kernel labels every tile itself).  SW_LABEL_UNION (default): one pass that
 * links tile roots with device-scope atomicMin, reaching the fixed point
 * directly.  The paper's two iterative labellers, chosen like its program's
 * `algorithm` parameter (Sec. 2, program notes; label-equivalence
 * paragraphs): SW_LABEL_HAWICK (0; scanning with atomicMin on a temporary R,
 * analysis of R chains, labeling label <- R[label]) and SW_LABEL_KALENTEV
 * (1; one label variable, scanning and analysis, no atomic operation), each
 * iterated inside one launch per sweep until a scan changes nothing, at most
 * max_iterations (1 .. 4096) scans; reaching the cap without convergence
 * makes the call return SW_E_NOCONV.  Every labeller yields the same labels
 * and so the same trajectory.  Plain form only: batched and served lattices
 * use SW_LABEL_UNION.  Resets the labelling statistics. */
enum sw_labeller { SW_LABEL_HAWICK = 0, SW_LABEL_KALENTEV = 1, SW_LABEL_UNION = 2 };
int sw_set_labeller(sw_handle h, int algorithm, int max_iterations);

/* Labelling statistics since the last sw_set_labeller: sweeps labelled by an
 * iterative labeller, the scans they ran in total and the most any one ran
 * (any pointer may be NULL; all zero under SW_LABEL_UNION). */
int sw_get_label_stats(sw_handle h, int64_t *labellings, int64_t *scans, int64_t *max_scans);

/* Test hook: bound every device label walk and union retry of this handle by
 * `cap` steps (1 .. 2^32-1; default N + 1, never reached on a valid forest).
 * A tiny cap makes the kernels stop early, flag the sweep and return
 * SW_E_NOCONV, which is how the error path is exercised. */
int sw_set_walk_cap(sw_handle h, int64_t cap);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * cluster statistics of sw_measure's last argument, computed without any
 * allocation.  The per-root sizes live in a fixed device array of at most
 * 2^22 sites (16 MiB, held by each GPU the library runs on until the process
 * ends): lattices with more sites are rejected with SW_E_INVALID.  All calls
 * on one GPU share that array, so calls that overlap on a GPU race; each
 * call clears what it uses.  Synchronous on the handle's stream. */
int sw_cluster_stats_noalloc(sw_handle h, sw_cluster_stats *cs);

/* Drop the recorded series (the paper's discarded MCS). */
int sw_reset_measure(sw_handle h);

/* Copy up to `max` records (oldest first) into `out`; returns the count. */
int64_t sw_series(sw_handle h, sw_record *out, int64_t max);

/* Turn per-sweep measurement on (1, default) or off (0). */
int sw_set_measure(sw_handle h, int on);

/* Release all device memory of the handle.  NULL is ignored. */
void sw_destroy(sw_handle h);

/* Message of the last error on the calling thread ("" if none). */
const char *sw_last_error(void);

/* Per-kernel device time of plain sweeps.  Level 1 brackets the bond kernel
 * (bond generation + tile labelling; it also applies the previous sweep's
 * cluster decisions) of every sweep whose index is a multiple of 16 with HIP
 * events on the handle's stream and accumulates its duration and the number
 * of launches timed; level 2 also times those sweeps' global labelling phase
 * (the label merge across tiles, or the iterative labeller) and the flip
 * that ends each sw_sweep call; 0 turns it off.  Any level > 0 clears the
 * totals.  SW_E_INVALID for other levels. */
int sw_profile(sw_handle h, int on);
/* Accumulated milliseconds and launch counts per kernel (3 entries each:
 * 0 = bond, 1 = global labelling phase, 2 = flip). */
int sw_profile_read(sw_handle h, double *ms, int64_t *launches);

/* --- state access (checkpoint / parity hooks) ----------------------------- */

/* Number of sweeps done so far (the next sweep's index n). */
int64_t sw_sweep_index(sw_handle h);
/* Set the next sweep's index (resume a stream position; 0 <= n < 2^32). */
int sw_set_sweep_index(sw_handle h, int64_t n);
/* Copy the N states out / in (int8, uint8 or float by model).  sw_set_state
 * rejects out-of-range states (Ising not +1/-1, Potts >= q, XY outside
 * [0, (float)2pi) or NaN) with SW_E_INVALID. */
int sw_get_state(sw_handle h, void *host_state);
int sw_set_state(sw_handle h, const void *host_state);
/* Minimum-index labels (N int32) and bond bytes (N uint8) of the last sweep
 * run (whatever sw_set_sweep_index or sw_set_state did since); identity
 * labels and zero bonds before any sweep. */
int sw_get_labels(sw_handle h, int32_t *host_labels);
int sw_get_bonds(sw_handle h, uint8_t *host_bonds);
/* Lattice parameters of a handle (any pointer may be NULL). */
int sw_info(sw_handle h, int *model, int *dim, int *L, int *q, double *beta, uint64_t *seed,
            uint32_t *replica);

/* --- batched form: many lattices of uneven size in one launch ------------- */

typedef struct sw_batch_s *sw_batch;

/* One lattice of a batch (same rules as sw_create_replica). */
typedef struct {
    int model, dim, L, q;
    double beta;
    uint64_t seed;
    uint32_t replica;
} sw_job_desc;

/* Create n >= 1 lattices that sweep together: every kernel launch covers the
 * tiles of all lattices of one (model, dim) group, and chunks of sweeps are
 * replayed from a captured HIP graph.  NULL on error. */
sw_batch sw_batch_create(const sw_job_desc *jobs, int n);

/* Run n sweeps on every member.  Each member's trajectory is identical to a
 * plain handle with the same parameters. */
int sw_batch_sweep(sw_batch b, int64_t n);

/* Run counts[j] sweeps on member j (0 = idle) in the same batched launches. */
int sw_batch_sweep_counts(sw_batch b, const int64_t *counts);

/* Number of members; a handle that views member j (state access, measure,
 * series; do not sw_destroy it, and sw_sweep on it runs that member alone). */
int sw_batch_size(sw_batch b);
sw_handle sw_batch_member(sw_batch b, int j);

/* Sweeps replayed per captured graph (default chosen by the tuner). */
int sw_batch_set_chunk(sw_batch b, int sweeps_per_graph);

/* Streams the batch's launches use (1 .. 8, default 2 when the batch has two
 * lattices or more): the members are dealt to that many parts by site count,
 * each part replaying its own graph on its own stream, so that the parts'
 * kernels can run side by side.  The trajectories do not depend on it. */
int sw_batch_set_streams(sw_batch b, int n);

void sw_batch_destroy(sw_batch b);

/* --- served form: continuous batching of submitted jobs ------------------- */

typedef struct sw_server_s *sw_server;

/* A job: lattice parameters plus the number of sweeps to run. */
typedef struct {
    sw_job_desc lattice;
    int64_t sweeps;
} sw_job;

/* Result of a finished job. */
typedef struct {
    int64_t id;
    int status;          /* 0 = done, SW_E_* on failure */
    int64_t sweeps;      /* sweeps run */
    double submit_s;     /* server clock at submission, seconds */
    double start_s;      /* admitted to the device */
    double finish_s;     /* last sweep completed */
    double m2, m4, energy; /* averages over all sweeps of the job */
} sw_job_result;

/* Start a server whose resident lattices may use at most hbm_budget_bytes of
 * device memory and at most max_active jobs at once; chunk = sweeps per
 * scheduling tick.  The device buffers of finished jobs are kept for the
 * next admissions (no allocation or free per job), at most
 * min(hbm_budget_bytes / 4, 4 GiB) of them beyond the budget; they are
 * released by sw_server_destroy.  NULL on error. */
sw_server sw_server_create(int64_t hbm_budget_bytes, int max_active, int chunk);

/* Queue a job; returns its id (>= 0) or SW_E_*.  Jobs whose footprint exceeds
 * the whole budget are rejected with SW_E_INVALID. */
int64_t sw_server_submit(sw_server s, const sw_job *job);

/* One scheduling tick: admit queued jobs that fit, run one chunk of sweeps
 * on every active job in batched launches, retire finished jobs.  Returns
 * the number of jobs still queued or active. */
int64_t sw_server_step(sw_server s);

/* Copy the result of finished job `id` (SW_E_NOTFOUND if unknown, 1 if not
 * finished yet, 0 when copied).  With state != NULL the final configuration
 * is copied too (N states). */
int sw_server_poll(sw_server s, int64_t id, sw_job_result *out, void *state);

/* Cancel job `id` between ticks.  A queued job leaves the queue; a running
 * one leaves the device at once and its memory returns to the budget.  Its
 * result (sw_server_poll) then has status SW_E_CANCELLED, the sweeps it ran,
 * the averages over them (0 when none ran) and the state after them (a job
 * cancelled in the queue has no state: poll leaves the buffer untouched).
 * Returns 0 when cancelled, 1 if the job had already finished (its result
 * stays), SW_E_NOTFOUND for an unknown id. */
int sw_server_cancel(sw_server s, int64_t id);

/* Device bytes one job of this shape needs while resident. */
int64_t sw_footprint(int model, int dim, int L, int q);

/* Streams a server deals each tick's (model, dim, tile shape) groups to
 * (1 .. 8, default 4), by site count: the groups' launches run side by side.
 * Jobs are admitted (their lattices created) on a stream of their own while
 * a tick runs.  Results do not depend on it. */
int sw_server_set_streams(sw_server s, int n);

void sw_server_destroy(sw_server s);

#ifdef __cplusplus
}
#endif
#endif
