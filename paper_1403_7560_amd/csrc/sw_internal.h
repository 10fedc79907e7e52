// sw_internal.h -- layout shared by the HIP kernels and the host runtime of
// libswmc (product code; the oracle does not use it).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swmc {

enum { ISING = 0, POTTS = 1, XY = 2, CLOCK = 3 };
// Clock model: the largest q (the paper's shared-memory table limit).
constexpr int CLOCK_QMAX = 512;
enum { TAG_BOND = 0, TAG_BOND_Z = 1, TAG_BOND_TIE = 2, TAG_CLUSTER = 3, TAG_GLOBAL = 4,
       TAG_INIT = 5 };

// A label word is either the global index of the site's parent (< 2^31) or,
// for a cluster root, ROOT_FLAG | the cluster's random decision (Sec. 2,
// step (3)), so the flip needs no separate per-root array.
constexpr uint32_t ROOT_FLAG = 0x80000000u;

// k_flip's sweep argument that means "the last sweep of the launch chain"
// (sweep0 + count - 1), used once per chain for Ising and Potts.
constexpr uint32_t FLIP_LAST = 0xFFFFFFFFu;

// Per-lattice descriptor read by every kernel (one per lattice in a batch).
struct InstDesc {
    int32_t model, dim, L, q;
    int32_t tiles[3];     // tiles along x, y, z (z = 1 in 2D)
    int32_t ntiles;
    int32_t nslots;       // measurement slots per record
    int64_t N;
    uint64_t thr;         // Ising / Potts bond threshold floor(p 2^32)
    uint32_t thr_hi;      // thr >> 16 (0 .. 65536), compared with the 16-bit primaries
    uint32_t thr_lo;      // thr & 0xffff, compared with the secondary on a tie
    double two_beta;      // XY: 2 beta
    uint32_t key0, key1, rep;
    // schedule of the current launch chain: sweep sweep0 + k runs while k < count
    uint32_t sweep0, count;
    uint32_t remaining;   // sweeps left in a batched call (advanced on the device)
    uint32_t chunk;       // sweeps per graph replay
    int32_t measure;      // write a record per sweep
    int32_t store_bonds;  // keep the bond bytes in HBM
    int64_t rec_row0;     // record row of sweep0 (-1: no recording)
    int64_t rec_cap;      // rows in rec (one extra scratch row follows)
    void *state;
    uint32_t *label;      // label words of even sweeps
    uint32_t *label2;     // label words of odd sweeps
    float *theta_w[2];    // XY: angles entering even / odd sweeps of a launch chain
    uint8_t *bond;
    int32_t *face;        // per direction mu: [tile][out|in][F_mu]
    int64_t face_off[3];
    int32_t face_len[3];
    int64_t *part;        // [ntiles][nslots] per-tile partial sums
    int64_t *rec;         // [rec_cap + 1][nslots]
    // Bounded walks: a label chain or union retry longer than walk_cap steps
    // (never reached on a valid forest, whose chains strictly decrease and so
    // end within N steps) stops, sets ERR_WALK in *err and the host call
    // reports SW_E_NOCONV.
    uint32_t *err;
    uint32_t walk_cap;
    // Iterative labellers (Hawick 0 / Kalentev 1): per tile up to edge_cap
    // unique (out root, in root) pairs and their count; Hawick's temporary
    // label R (N words); labelling statistics {labellings, scans, max scans}.
    uint64_t *edges;
    int32_t *ecount;
    int32_t edge_cap;
    uint32_t *rbuf;
    uint64_t *lstats;
    // Clock model: integer bond thresholds of two projection indices,
    // [(q/2 + 1)^2], and cos, sin of 2 pi k / q, k < q ([2q]).
    uint32_t *clock_thr;
    double *clock_trig;
};

// Bits of a lattice's device error word.
constexpr uint32_t ERR_WALK = 1u;   // a label walk or union hit walk_cap
constexpr uint32_t ERR_ITER = 2u;   // iterative labelling hit its iteration cap

// Tile shape of a kernel variant.
struct TileShape {
    int tx, ty, tz;
};

// Launchers (defined in sw_kernels.hip).  `variant` picks a tile shape from
// the table tile_shapes(model, dim).
int num_tile_variants(int model, int dim);
TileShape tile_shape(int model, int dim, int variant);
int slots_for(int model, int q);
// Tile t of an L^dim lattice cut into tiles of shape ts lies wholly inside it.
bool tile_interior(int dim, int L, const TileShape &ts, int t);

hipError_t launch_init(const InstDesc *d_desc, int inst, const InstDesc &h, hipStream_t s);
// The first `nfull` entries of the tile map are tiles wholly inside their
// lattice (see append_tiles); they run the bond kernel without edge tests.
// `t0`/`t1` (may be null) are recorded by the launches themselves: t0 when
// the first bond launch starts executing, t1 when the last one ends, so their
// elapsed time is the kernel's own duration without the gaps around it.
hipError_t launch_bond(int model, int dim, int variant, const InstDesc *d_desc,
                       const int2 *d_tmap, int ntiles, int nfull, uint32_t k, int mode, hipStream_t s,
                       hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
hipError_t launch_merge(int dim, int model, int variant, const InstDesc *d_desc, const int2 *d_tmap,
                        int ntiles, uint32_t k, hipStream_t s);
hipError_t launch_reduce(int model, const InstDesc *d_desc, const int2 *d_tmap, int ntiles, hipStream_t s);
hipError_t launch_flip(int model, int dim, int variant, const InstDesc *d_desc,
                       const int2 *d_tmap, int ntiles, uint32_t k, hipStream_t s);
hipError_t launch_canon(const InstDesc *d_desc, int inst, int64_t N, int32_t *d_out,
                        hipStream_t s);
hipError_t launch_advance(InstDesc *d_desc, int ninst, hipStream_t s);
// Per-model instantiations behind launch_bond / launch_flip (one translation
// unit each).
hipError_t launch_bond_ising(int dim, int v, const InstDesc *dd, const int2 *tm, int nt, int nf, uint32_t k,
                             int mode, hipStream_t s, hipEvent_t t0, hipEvent_t t1);
hipError_t launch_bond_potts(int dim, int v, const InstDesc *dd, const int2 *tm, int nt, int nf, uint32_t k,
                             int mode, hipStream_t s, hipEvent_t t0, hipEvent_t t1);
hipError_t launch_bond_xy(int dim, int v, const InstDesc *dd, const int2 *tm, int nt, int nf, uint32_t k,
                          int mode, hipStream_t s, hipEvent_t t0, hipEvent_t t1);
hipError_t launch_flip_ising(int dim, int v, const InstDesc *dd, const int2 *tm, int nt, uint32_t k, hipStream_t s);
hipError_t launch_flip_potts(int dim, int v, const InstDesc *dd, const int2 *tm, int nt, uint32_t k, hipStream_t s);
hipError_t launch_flip_xy(int dim, int v, const InstDesc *dd, const int2 *tm, int nt, uint32_t k, hipStream_t s);
hipError_t launch_bond_clock(int dim, int v, const InstDesc *dd, const int2 *tm, int nt, int nf, uint32_t k,
                             int mode, hipStream_t s, hipEvent_t t0, hipEvent_t t1);
hipError_t launch_flip_clock(int dim, int v, const InstDesc *dd, const int2 *tm, int nt, uint32_t k, hipStream_t s);

// The paper's iterative labellers for the global phase (alg 0 Hawick, 1
// Kalentev; defined in sw_label.hip): one cooperative launch per sweep that
// iterates until a scan changes nothing or `cap` scans ran.  `ctl` must hold
// label_ctl_words(cap) words; it is cleared by the launch itself.
hipError_t launch_label_iter(int dim, int model, int variant, int alg, const InstDesc *d_desc, const int2 *d_tmap,
                             int ntiles, uint32_t k, uint32_t *ctl, int cap, hipStream_t s);
int label_ctl_words(int cap);

}  // namespace swmc

namespace swmc {
// out3 = {#clusters, max size, sum size^2}; must be zeroed by the caller.
hipError_t launch_cluster_stats(const InstDesc *d_desc, int inst, int64_t N, int32_t *scratch,
                                unsigned long long *out3, hipStream_t s);
// The same without allocating: the scratch is a file-scope device array of
// STATIC_STATS_SITES sites (hipErrorInvalidValue beyond); synchronous, the
// three sums land in host_out.
constexpr int64_t STATIC_STATS_SITES = (int64_t)1 << 22;
constexpr int MAX_DEVICES = 64;
hipError_t cluster_stats_static(const InstDesc *d_desc, int inst, int64_t N, unsigned long long host_out[3],
                                hipStream_t s);
}  // namespace swmc
