// sw_bond.h -- the bond kernel (bond generation + tile labelling +
// measurement) and the flip kernel, as templates over (model, dim, tile
// shape).  Each model's instantiations are compiled in a translation unit of
// their own (sw_bond_ising.hip, sw_bond_potts.hip, sw_bond_xy.hip).
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sw_device.h"

namespace swmc {

// ---- union-find in LDS (tile-local indices) --------------------------------
// The parent table is addressed through an LDS (address space 3) pointer so
// that every access is a ds_* instruction.  Loads are volatile: other lanes
// and wavefronts link roots concurrently.
typedef __attribute__((address_space(3))) int lds_int;

// Root of a with path halving: a non-root's parent may be replaced by any
// ancestor (every pointer goes to a smaller index of the same cluster), so
// the plain store is safe against concurrent unions.
__device__ __forceinline__ int lds_find(volatile lds_int *par, int a)
{
    while (true) {
        const int p = par[a];
        if (p == a) return a;
        const int g = par[p];
        if (g == p) return p;
        par[a] = g;
        a = g;
    }
}

__device__ __forceinline__ void lds_union(lds_int *par, int a, int b)
{
    volatile lds_int *vp = par;
    while (true) {
        a = lds_find(vp, a);
        b = lds_find(vp, b);
        if (a == b) return;
        if (a < b) {
            const int t = a;
            a = b;
            b = t;
        }
        const int old = __hip_atomic_fetch_min(&par[a], b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old == a) return;  // a was still a root: now linked under b
        a = old;               // a was linked meanwhile: merge its parent instead
    }
}

// Apply a wavefront's queued equivalences (a << 16 | b) to the LDS table;
// called with the whole wavefront, lane l takes entries l, l + 64, ...
typedef __attribute__((address_space(3))) uint32_t lds_u32;
static __device__ __noinline__ void flush_queue(lds_int *par, const lds_u32 *q, int qn, int lane)
{
    for (int e = lane; e < qn; e += 64) {
        const uint32_t pr = q[e];
        lds_union(par, (int)(pr >> 16), (int)(pr & 0xffffu));
    }
}

// ---------------------------------------------------------------------------
// Helpers of the bond kernel.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double from_right_d(double v)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const uint32_t lo = from_right((uint32_t)u), hi = from_right((uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ double readlane_d(double v, int l)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The 16-bit secondary of bond (g, mu): high half of word d*g+mu of the tie
// stream; consulted only when the primary equals the threshold's high half.
__device__ __noinline__ uint32_t bond_secondary(uint32_t key0, uint32_t key1, uint32_t rep, uint32_t n,
                                                int dim, uint32_t g, int mu)
{
    const uint32_t w = (uint32_t)dim * g + (uint32_t)mu;
    const uint4 b = philox(make_uint4(w >> 2, n, (uint32_t)TAG_BOND_TIE, rep), key0, key1);
    return lane_of(b, w & 3u) >> 16;
}

// (cos theta, sin theta) in FP64 for a float angle in [0, 2pi], from a table
// of cos/sin(k 2pi/128) and short polynomials in r = theta - k 2pi/128,
// |r| <= pi/128: the truncated Taylor terms are below 1e-20 and the rounding
// a few ulps, ample for the measurement sums and the fast bond test (the
// exact bond test uses the library cos).
#define XY_TAB 128
__device__ __forceinline__ void xy_sincos(float th, const double2 *tab, double &c, double &s)
{
    const double DHI = TWO_PI_D / XY_TAB;                   // exact: 2pi_d / 2^7
    const double DLO = 2.4492935982947064e-16 / XY_TAB;     // 2pi - 2pi_d, scaled
    const int k = (int)((float)th * (float)(XY_TAB / TWO_PI_D) + 0.5f);
    double r = fma(-(double)k, DHI, (double)th);
    r = fma(-(double)k, DLO, r);
    const double r2 = r * r;
    const double cr = fma(r2, fma(r2, fma(r2, fma(r2, 1.0 / 40320.0, -1.0 / 720.0), 1.0 / 24.0), -0.5), 1.0);
    const double sr = r * fma(r2, fma(r2, fma(r2, fma(r2, 1.0 / 362880.0, -1.0 / 5040.0), 1.0 / 120.0), -1.0 / 6.0), 1.0);
    const double2 t = tab[k & (XY_TAB - 1)];
    c = fma(t.x, cr, -(t.y * sr));
    s = fma(t.y, cr, t.x * sr);
}

// XY bond test, exact form: u = (P 2^16 + S) 2^-32 < -expm1(-(2 beta s_i) s_j)
// with s = cos(theta - phi) in FP64, decided from the 16-bit primary alone
// unless u's interval straddles p.  Runs only when the fast test below cannot
// decide.
__device__ __noinline__ uint32_t xy_bond_exact(float ti, float tj, uint32_t gi, double phi, double two_beta,
                                               uint32_t p, uint32_t key0, uint32_t key1, uint32_t rep, uint32_t n,
                                               int dim, int mu)
{
    const double si = cos((double)ti - phi), sj = cos((double)tj - phi);
    const double x = (two_beta * si) * sj;
    const double pr = -expm1(-x);
    const double lo = (double)p * 0x1p-16, hi = (double)(p + 1u) * 0x1p-16;
    if (hi <= pr) return 1u;
    if (lo >= pr) return 0u;
    const uint32_t sec = bond_secondary(key0, key1, rep, n, dim, gi, mu);
    return (double)((p << 16) | sec) * 0x1p-32 < pr ? 1u : 0u;
}

// XY bond test, fast form: p = 1 - e^-x in FP32 from x = (2 beta s_i) s_j,
// the projections taken as cos(theta) cos(phi) + sin(theta) sin(phi) in FP64.
// |p_fast - p_exact| stays below 3e-7 (FP64 projections ~1e-15, the float
// rounding of x and of x log2(e), the exp2 instruction and the subtraction a
// few float ulps each), so a primary interval that clears p_fast by
// XY_MARGIN = 2^-18 decides the bond exactly as the FP64 rule would.
// Returns 1 / 0, or 2 when undecided.
#define XY_MARGIN 0x1p-18f
__device__ __forceinline__ uint32_t xy_bond_fast(double two_beta, double si, double sj, uint32_t p)
{
    const float x = (float)((two_beta * si) * sj);
    const float pf = 1.0f - __builtin_amdgcn_exp2f(x * -1.44269504088896340736f);
    const float lo = (float)p * 0x1p-16f, hi = (float)(p + 1u) * 0x1p-16f;
    if (hi <= pf - XY_MARGIN) return 1u;
    if (lo >= pf + XY_MARGIN) return 0u;
    return 2u;
}

// ---------------------------------------------------------------------------
// Bond generation + tile-local labelling + measurement.
// mode 0: full sweep step; mode 1: measurement of the configuration only.
//
// Lane c of every wavefront owns column c of the tile; wavefront w owns the
// tile rows [w R, (w+1) R) (row r = y + TY z), kept in registers.  The x
// neighbour comes from lane c+1 by a DPP shift (the tile's last column from a
// halo column), the y and z neighbours from the same lane's other rows or a
// halo row.  The bond words are the column blocks of the random layout: one
// Philox call per lane gives the words of four consecutive rows.
//
// Labelling scans the rows in order: the x bonds of a row form runs (ballot
// and bit tricks); a run takes the smallest label among its sites bonded to the
// row above (3D: or the plane behind), otherwise its own start.  Only run
// starts are union-find nodes: s_par[start] links to the inherited label.  A
// bonded neighbour whose label differs is an equivalence, queued and resolved
// in s_par (larger root under smaller) together with the bonds that cross
// wavefront blocks and the periodic bonds of a tile that spans the lattice.
// After path compression the root of a site is s_par[its run start].
// ---------------------------------------------------------------------------
template <int MODEL> struct LaneValue { typedef uint32_t type; };
template <> struct LaneValue<XY> { typedef double type; };
// What the working buffers hold between the sweeps of a chain: XY angles,
// clock state indices (unused by Ising / Potts).
template <int MODEL> struct WorkOf { typedef uint32_t type; };
template <> struct WorkOf<XY> { typedef float type; };

// Clock model: fold the projection index a = (2p - r) mod 2q of state p on
// the mirror axis r to m in [0, q/2] and the projection's sign (+1, -1, 0
// for a spin perpendicular to the axis): sigma = sign cos(pi m / q).
__device__ __forceinline__ uint32_t clock_fold(uint32_t p, uint32_t r, uint32_t q, int &sgn)
{
    uint32_t a = 2u * p + 2u * q - r;  // in (0, 4q)
    if (a >= 2u * q) a -= 2u * q;
    const uint32_t a1 = a <= q ? a : 2u * q - a;
    if (2u * a1 < q) {
        sgn = 1;
        return a1;
    }
    if (2u * a1 == q) {
        sgn = 0;
        return q >> 1;
    }
    sgn = -1;
    return q - a1;
}

// Clock mirror of state p on axis r: (q/2 + r - p) mod q.
__device__ __forceinline__ uint32_t clock_mirror(uint32_t p, uint32_t r, uint32_t q)
{
    uint32_t v = (q >> 1) + r + q - p;  // in (0, 2.5q)
    if (v >= q) v -= q;
    if (v >= q) v -= q;
    return v;
}

// Mirror axis of sweep n: floor(w q / 2^32) of word 0 of the GLOBAL stream.
__device__ __forceinline__ uint32_t clock_axis(const InstDesc &d, uint32_t n)
{
    const uint4 w = philox(make_uint4(0u, n, (uint32_t)TAG_GLOBAL, d.rep), d.key0, d.key1);
    return (uint32_t)(((uint64_t)w.x * (uint64_t)(uint32_t)d.q) >> 32);
}

// Clock bond test: both projections nonzero with one sign, and the 32-bit
// uniform (primary P, secondary on a tie) below the integer threshold of the
// two projection indices (a table the host builds per (q, beta)).
__device__ __forceinline__ uint32_t clock_bond(uint32_t pi, uint32_t pj, uint32_t r, const InstDesc &d,
                                               uint32_t P, uint32_t gi, int mu, uint32_t key0, uint32_t key1,
                                               uint32_t rep, uint32_t n, int dim)
{
    const uint32_t q = (uint32_t)d.q;
    int si, sj;
    const uint32_t mi = clock_fold(pi, r, q, si), mj = clock_fold(pj, r, q, sj);
    if (si == 0 || si != sj) return 0u;
    const uint32_t thr = d.clock_thr[mi * ((q >> 1) + 1u) + mj];
    const uint32_t th = thr >> 16;
    if (P != th) return P < th ? 1u : 0u;
    return bond_secondary(key0, key1, rep, n, dim, gi, mu) < (thr & 0xffffu) ? 1u : 0u;
}

// Wavefronts per SIMD the bond kernel's registers are sized for: Ising /
// Potts the hardware's 8 while a wavefront holds at most 16 rows (the LDS
// of 8 such wavefronts per SIMD fits the CU's 160 KB), else 3; XY keeps its
// FP64 projections in registers and runs 4.
template <int MODEL, int T, int NW> struct BondOccupancy {
    static constexpr int value = (MODEL == XY) ? 4 : ((T / NW <= 1024) ? 8 : 3);
};
// (the clock model keeps integer states and runs 8, like Ising)

template <int MODEL, int DIM, int TX, int TY, int TZ, int NW, bool FULL>
__global__ void __launch_bounds__(64 * NW, (BondOccupancy<MODEL, TX * TY * TZ, NW>::value))
k_bond(const InstDesc *__restrict__ descs,
                                              const int2 *__restrict__ tmap, uint32_t k, int mode)
{
    typedef typename StateOf<MODEL>::type S;
    constexpr int T = TX * TY * TZ;
    constexpr int ROWS = TY * TZ;
    constexpr int NT = 64 * NW;  // threads per workgroup (NW wavefronts)
    constexpr int R = ROWS / NW; // rows per wavefront
    constexpr int NG = R / 4;    // groups of four rows per wavefront
    constexpr bool IS_XY = (MODEL == XY);
    constexpr bool IS_CK = (MODEL == CLOCK);
    // XY and clock hold one value per row (no packed bytes of four rows)
    constexpr bool VEC = IS_XY || IS_CK;
    constexpr int QCAP = 128;    // per-wave queue of deferred equivalences
    constexpr int NONE = 0x7fffffff;
    static_assert(TX == 64, "a tile row is one wavefront (lane = column)");
    static_assert(ROWS % NW == 0 && R % 4 == 0 && R <= 32, "whole row groups, one bond bit per row");
    static_assert(TY % 4 == 0, "row groups of the column random layout stay in a plane");
    static_assert(DIM == 2 ? TZ == 1 : R % TY == 0, "3D: whole planes per wavefront");

    __shared__ int s_par[T];
    __shared__ unsigned long long s_xm[ROWS];  // in-tile x-bond mask of every row
    __shared__ uint32_t s_rowg[ROWS];          // global index of every row's first site
    __shared__ unsigned long long s_dm[ROWS];  // cluster decision bit of every site, one word per row
    __shared__ uint32_t s_q[NW][QCAP];
    // Potts histogram of the measurement: it is done before the scan fills the
    // equivalence queues, so it shares their memory
    int *s_hist = (int *)&s_q[0][0];
    static_assert(NW * QCAP >= 256, "histogram fits the queues");
    __shared__ double s_red[NW][3];
    __shared__ double s_phi[4];  // XY: phi, cos phi, sin phi, previous sweep's phi
    __shared__ double2 s_cs[IS_XY ? XY_TAB : 1];  // XY: cos/sin(k 2pi/128)
    // clock: the paper's tables, cos (= the pair energy rule) and sin of 2 pi k / q
    __shared__ double s_trig[IS_CK ? 2 * CLOCK_QMAX : 1];
    __shared__ uint32_t s_axis[2];  // clock: this sweep's and the previous sweep's mirror axis
    // 3D XY after the first sweep of a chain: the incoming angles of the sites
    // outside a wavefront's rows that its bond tests read (slot j < R: +z of
    // row j where the next plane is not the wavefront's; R + p: +y of plane
    // p's last row; last: the halo column, lane c < R for row c), resolved
    // in one batch before the wavefront's own rows
    constexpr bool NBX = IS_XY && DIM == 3;
    constexpr int NBS = R + R / TY + 1;
    __shared__ float s_nth[NBX ? NW * NBS * 64 : 1];

    const int2 tm = tmap[tile_slot()];
    if (tm.x < 0) return;
    // a reference: fields load from the (read-only) descriptor when used,
    // instead of a copy that would hold them all in scalar registers
    const InstDesc &d = descs[tm.x];
    if (k >= d.count) return;
    const uint32_t n = d.sweep0 + k;
    const int L = d.L;
    const int t = tm.y;
    const int tx = t % d.tiles[0];
    const int ty = (t / d.tiles[0]) % d.tiles[1];
    const int tz = (DIM == 3) ? t / (d.tiles[0] * d.tiles[1]) : 0;
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
    const int tid = threadIdx.x;
    // the wavefront index is uniform: readfirstlane lets everything derived
    // from it (rows, global addresses) live in scalar registers
    const int c = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r0 = wv * R;
    // FULL: the tile lies wholly inside the lattice (every tile when the side
    // is a multiple of the tile's); its extents are constants and no row or
    // column needs a range test.  The host lists such tiles apart.
    if (FULL && !((x0 + TX <= L) && (y0 + TY <= L) && (DIM == 2 || z0 + TZ <= L))) return;
    const int ex = FULL ? TX : min(TX, L - x0);
    const int ey = FULL ? TY : min(TY, L - y0);
    const int ez = (DIM == 3) ? (FULL ? TZ : min(TZ, L - z0)) : 1;
    const bool vc = FULL || c < ex;
    const bool full = (mode == 0);
    const bool meas = (mode == 1) || d.measure;
    const bool bits_dec = (MODEL != POTTS) || d.q == 2;
    const uint32_t key0 = d.key0, key1 = d.key1, rep = d.rep;
    const GLOBAL S *g_st = (const GLOBAL S *)d.state;
    GLOBAL uint32_t *g_label = (GLOBAL uint32_t *)labels_of(d, n);
    // After the first sweep of a launch chain the states in HBM are stale: a
    // site's incoming state is its cluster's decision in the previous sweep's
    // labels (step (3) of that sweep, done here) -- Ising / Potts the decision
    // itself, XY the previous sweep's angle mirrored or kept.
    const bool from_labels = full && k > 0;
    GLOBAL uint32_t *lab_prev = (GLOBAL uint32_t *)labels_of(d, n - 1u);
    const uint32_t uL = (uint32_t)L;
    const uint32_t gx = (uint32_t)(x0 + c);
    const uint32_t gxr = (x0 + ex == L) ? 0u : (uint32_t)(x0 + ex);  // column right of the tile

    // tile row j of this wavefront -> local y, z (2D: the wave holds part of
    // the plane; 3D: whole planes)
    auto row_y = [&](int j) -> int { return DIM == 2 ? r0 + j : j % TY; };
    auto row_z = [&](int j) -> int { return DIM == 2 ? 0 : r0 / TY + j / TY; };
    auto row_ok = [&](int j) -> bool { return FULL || (row_y(j) < ey && row_z(j) < ez); };
    // global index of (x, y0 + ly, z0 + lz), ly <= ey and lz <= ez wrapping
    auto gat = [&](uint32_t x, int ly, int lz) -> uint32_t {
        uint32_t y = (uint32_t)(y0 + ly), z = (uint32_t)(z0 + lz);
        if (y >= uL) y -= uL;
        if (DIM == 3 && z >= uL) z -= uL;
        return x + uL * (y + uL * z);
    };
    // the same for a site of the tile (ly < ey, lz < ez): nothing wraps
    auto gin = [&](uint32_t x, int ly, int lz) -> uint32_t {
        return x + uL * ((uint32_t)(y0 + ly) + uL * (uint32_t)(z0 + lz));
    };
    auto gidx = [&](int l) -> uint32_t {  // tile-local index -> global index
        return s_rowg[l >> 6] + (uint32_t)(l & 63);
    };

    if (IS_XY && tid < XY_TAB) {
        double sk, ck;
        sincos((double)tid * (TWO_PI_D / XY_TAB), &sk, &ck);
        s_cs[tid] = make_double2(ck, sk);
    }
    if (IS_XY && tid == 0) {
        const double ph = xy_phi(d, n);
        double sp, cp;
        sincos(ph, &sp, &cp);
        s_phi[0] = ph;
        s_phi[1] = cp;
        s_phi[2] = sp;
        s_phi[3] = from_labels ? xy_phi(d, n - 1u) : 0.0;
    }
    if (IS_CK) {
        for (int i = tid; i < 2 * d.q; i += NT) s_trig[i] = d.clock_trig[i];
        if (tid == 0) {
            s_axis[0] = clock_axis(d, n);
            s_axis[1] = from_labels ? clock_axis(d, n - 1u) : 0u;
        }
    }
    if (MODEL == POTTS && meas)
        for (int q = tid; q < d.q; q += NT) s_hist[q] = 0;
    for (int r = tid; r < ROWS; r += NT) s_rowg[r] = gat((uint32_t)x0, r % TY, r / TY);
    // Cluster decision bits of every tile row (one bit per possible root): bit
    // c of s_dm[r] is bit g mod 32 of word g/32 of the cluster stream, g the
    // global index of site (x0 + c, row r).  The row's 64 bits lie in three
    // consecutive words, in Philox block g_r/128 and possibly the next one.
    if (full && bits_dec && tid < ROWS) {
        const int r = tid, ly = r % TY, lz = r / TY;
        if (ly < ey && lz < ez) {
            const uint32_t gr = gin((uint32_t)x0, ly, lz);
            const uint32_t blk = gr >> 7, wo = (gr >> 5) & 3u;
            const uint4 w0 = philox(make_uint4(blk, n, (uint32_t)TAG_CLUSTER, rep), key0, key1);
            uint4 w1 = make_uint4(0u, 0u, 0u, 0u);
            if (wo >= 2u) w1 = philox(make_uint4(blk + 1u, n, (uint32_t)TAG_CLUSTER, rep), key0, key1);
            // words wo, wo + 1, wo + 2 of the sequence w0, w1
            const uint32_t a = wo == 0u ? w0.x : wo == 1u ? w0.y : wo == 2u ? w0.z : w0.w;
            const uint32_t b = wo == 0u ? w0.y : wo == 1u ? w0.z : wo == 2u ? w0.w : w1.x;
            const uint32_t e = wo == 0u ? w0.z : wo == 1u ? w0.w : wo == 2u ? w1.x : w1.y;
            const uint32_t sh = gr & 31u;
            const uint32_t lo = __builtin_amdgcn_alignbit(b, a, sh), hi = __builtin_amdgcn_alignbit(e, b, sh);
            s_dm[r] = ((unsigned long long)hi << 32) | lo;
        }
    }
    if (VEC || (MODEL == POTTS && meas)) __syncthreads();
    const double phi = IS_XY ? s_phi[0] : 0.0, cphi = IS_XY ? s_phi[1] : 0.0, sphi = IS_XY ? s_phi[2] : 0.0;
    const double phi_prev = IS_XY ? s_phi[3] : 0.0;
    const uint32_t axis = IS_CK ? s_axis[0] : 0u, axis_prev = IS_CK ? s_axis[1] : 0u;
    const uint32_t uq = (uint32_t)d.q;

    // ---- states of the wave's rows, their +y/+z rows and the +x halo column --
    // Ising / Potts keep the states; XY keeps (cos theta, sin theta) in FP64.
    typedef typename LaneValue<MODEL>::type V;
    V own[R], ownS[R];
    // XY: the angles entering the previous sweep of the chain, and this sweep's
    const GLOBAL float *th_prev = IS_XY ? (const GLOBAL float *)(((n - 1u) & 1u) ? d.theta_w[1] : d.theta_w[0]) : nullptr;
    GLOBAL float *th_cur = IS_XY ? (GLOBAL float *)((n & 1u) ? d.theta_w[1] : d.theta_w[0]) : nullptr;
    // clock: the same for the state indices
    const GLOBAL uint16_t *ck_prev =
        IS_CK ? (const GLOBAL uint16_t *)(((n - 1u) & 1u) ? d.theta_w[1] : d.theta_w[0]) : nullptr;
    GLOBAL uint16_t *ck_cur = IS_CK ? (GLOBAL uint16_t *)((n & 1u) ? d.theta_w[1] : d.theta_w[0]) : nullptr;
    typedef typename WorkOf<MODEL>::type W;
    // clock: incoming state index of site g
    auto clock_in = [&](uint32_t g) -> uint32_t {
        if (!from_labels) return (uint32_t)((const GLOBAL uint16_t *)d.state)[g];
        const uint32_t w = root_word(lab_prev, lab_prev[g], d);
        const uint32_t p = ck_prev[g];
        return (w & 1u) ? clock_mirror(p, axis_prev, uq) : p;
    };
    // XY: incoming angle of site g
    auto theta_in = [&](uint32_t g) -> float {
        if (!from_labels) return ((const GLOBAL float *)d.state)[g];
        const uint32_t w = root_word(lab_prev, lab_prev[g], d);
        const float t = th_prev[g];
        return (w & 1u) ? xy_reflect(t, phi_prev) : t;
    };
    auto value_at = [&](uint32_t g, V &vs) -> V {
        if constexpr (IS_XY) {
            double sv, cv;
            xy_sincos(theta_in(g), s_cs, cv, sv);
            vs = sv;
            return cv;
        } else if constexpr (IS_CK) {
            vs = 0;
            return (V)clock_in(g);
        } else {
            vs = 0;
            if (from_labels) {
                const uint32_t w = root_word(lab_prev, lab_prev[g], d);
                return (V)state_of_decision<MODEL>(w & 0xffu);
            }
            return (V)(uint8_t)g_st[g];
        }
    };
    // the wavefront's own rows; XY stores the incoming angles for the next sweep
    auto set_own = [&](int j, uint32_t g, uint32_t dec, W th_old) {
        if constexpr (IS_XY) {
            const float th = from_labels ? ((dec & 1u) ? xy_reflect(th_old, phi_prev) : th_old) : th_old;
            if (full) th_cur[g] = th;
            double sv, cv;
            xy_sincos(th, s_cs, cv, sv);
            own[j] = cv;
            ownS[j] = sv;
        } else if constexpr (IS_CK) {
            const uint32_t p = from_labels ? ((dec & 1u) ? clock_mirror(th_old, axis_prev, uq) : th_old) : th_old;
            if (full) ck_cur[g] = (uint16_t)p;
            own[j] = p;
            ownS[j] = 0;
        } else {
            own[j] = from_labels ? (V)state_of_decision<MODEL>(dec & 0xffu) : (V)(uint8_t)g_st[g];
            ownS[j] = 0;
        }
    };
    // 2D: the merge may have chained this tile's roots of the previous sweep
    // through other tiles.  Every root of the tile that a face link can have
    // touched is in the tile's own face slots (the out side's roots with a
    // bond across, all of the in side's roots); the workgroup first points
    // each of them at its final root, so that the chase below ends in two
    // loads for every site.  Only the tile's own slots are read: this launch
    // overwrites them at its end, while neighbours may already have rewritten
    // theirs.
    if (DIM == 2 && from_labels && (d.tiles[0] > 1 || d.tiles[1] > 1)) {
        // both faces' slots in one pass (the x face's, then the y face's): a
        // 64x64 tile's 256 slots are one per thread, walked side by side
        const int E0 = d.tiles[0] > 1 ? 2 * d.face_len[0] : 0;
        const int E = E0 + (d.tiles[1] > 1 ? 2 * d.face_len[1] : 0);
        const GLOBAL int32_t *fs0 = (const GLOBAL int32_t *)d.face + d.face_off[0] + (int64_t)t * 2 * d.face_len[0];
        const GLOBAL int32_t *fs1 = (const GLOBAL int32_t *)d.face + d.face_off[1] + (int64_t)t * 2 * d.face_len[1];
        for (int e0 = 0; e0 < E; e0 += NT) {
            const int e = e0 + tid;
            const int32_t x = e < E0 ? fs0[e] : (e < E ? fs1[e - E0] : -1);
            const int32_t xl = (int32_t)from_left((uint32_t)x);
            if (x < 0 || (c != 0 && xl == x)) continue;  // no root, or the lane before has it
            // path halving: each node passed is pointed at its grandparent,
            // shortening the chains later workgroups and the chase walk
            uint32_t r = (uint32_t)x, w = lab_prev[r], steps = 0;
            while (!(w & ROOT_FLAG)) {
                if (++steps > d.walk_cap) break;
                const uint32_t w2 = lab_prev[w];
                if (w2 & ROOT_FLAG) {
                    r = w;
                    w = w2;
                    break;
                }
                lab_prev[r] = w2;
                r = w2;
                w = lab_prev[r];
            }
            if (!(w & ROOT_FLAG)) flag_error(d, ERR_WALK);
            else if (r != (uint32_t)x) lab_prev[x] = r;
        }
        __syncthreads();
    }
    if constexpr (NBX) {
        if (from_labels) {
            // one batch: every slot's label word and angle, then their roots'
            // words, chains walked in lock-step rounds, as for the own rows
            uint32_t g[NBS], w[NBS], val[NBS];
            float th[NBS];
            bool use[NBS];
            const int eyl = min(TY, ey) - 1;  // local y of a plane's last row
#pragma unroll
            for (int i = 0; i < NBS; ++i) {
                use[i] = false;
                g[i] = 0u;
                if (i < R) {
                    const int jf = i & ~3;
                    if (!(jf + TY < R && row_z(jf) + 1 < ez) && vc && row_ok(i)) {
                        use[i] = true;
                        g[i] = gat(gx, row_y(i), row_z(i) + 1);
                    }
                } else if (i < R + R / TY) {
                    const int j = (i - R) * TY + eyl;
                    if (vc && row_ok(j)) {
                        use[i] = true;
                        g[i] = gat(gx, row_y(j) + 1, row_z(j));
                    }
                } else {
                    const int ly = c % TY, lz = r0 / TY + c / TY;
                    if (c < R && ly < ey && lz < ez) {
                        use[i] = true;
                        g[i] = gin(gxr, ly, lz);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < NBS; ++i) {
                w[i] = use[i] ? lab_prev[g[i]] : ROOT_FLAG;
                th[i] = use[i] ? th_prev[g[i]] : 0.0f;
            }
#pragma unroll
            for (int i = 0; i < NBS; ++i) val[i] = (w[i] & ROOT_FLAG) ? w[i] : lab_prev[w[i]];
            bool more = false;
#pragma unroll
            for (int i = 0; i < NBS; ++i) more |= !(val[i] & ROOT_FLAG);
            uint32_t rounds = 0;
            while (more) {
                if (++rounds > d.walk_cap) {
                    flag_error(d, ERR_WALK);
#pragma unroll
                    for (int i = 0; i < NBS; ++i)
                        if (!(val[i] & ROOT_FLAG)) val[i] = ROOT_FLAG;
                    break;
                }
                more = false;
#pragma unroll
                for (int i = 0; i < NBS; ++i)
                    if (!(val[i] & ROOT_FLAG)) {
                        val[i] = lab_prev[val[i]];
                        more |= !(val[i] & ROOT_FLAG);
                    }
            }
#pragma unroll
            for (int i = 0; i < NBS; ++i)
                if (use[i]) s_nth[(wv * NBS + i) * 64 + c] = (val[i] & 1u) ? xy_reflect(th[i], phi_prev) : th[i];
        }
    }
    if (from_labels) {
        // per half of the rows (3D XY: all of them, its neighbour batch has
        // freed its registers): every row's label word, then all their tile
        // roots' words, in flight together; chains the merge made longer walked
        // in lock-step rounds; the tile root pointed at the final root
        constexpr int RH = (R >= 8 && !NBX) ? R / 2 : R;
#pragma unroll
        for (int h = 0; h < R; h += RH) {
            uint32_t w[RH], cur[RH], val[RH];
            W tho[RH];
#pragma unroll
            for (int i = 0; i < RH; ++i) {
                w[i] = ROOT_FLAG;
                tho[i] = 0;
                if (vc && row_ok(h + i)) {
                    const uint32_t g0 = gin((uint32_t)x0, row_y(h + i), row_z(h + i));
                    w[i] = (lab_prev + g0)[c];
                    if constexpr (IS_XY) tho[i] = (th_prev + g0)[c];
                    if constexpr (IS_CK) tho[i] = (ck_prev + g0)[c];
                }
            }
#pragma unroll
            for (int i = 0; i < RH; ++i) {
                cur[i] = w[i];
                // a root word loads the lattice's first word instead (no branch
                // around the load; the value is dropped)
                const uint32_t ld = lab_prev[(w[i] & ROOT_FLAG) ? 0u : w[i]];
                val[i] = (w[i] & ROOT_FLAG) ? w[i] : ld;
            }
            bool more = false;
#pragma unroll
            for (int i = 0; i < RH; ++i) more |= !(val[i] & ROOT_FLAG);
            uint32_t rounds = 0;
            while (__any(more)) {
                if (++rounds > d.walk_cap) {  // uniform
                    if (more) flag_error(d, ERR_WALK);
#pragma unroll
                    for (int i = 0; i < RH; ++i) {
                        cur[i] = w[i];
                        if (!(val[i] & ROOT_FLAG)) val[i] = ROOT_FLAG;
                    }
                    break;
                }
                more = false;
#pragma unroll
                for (int i = 0; i < RH; ++i) {
                    if (!(val[i] & ROOT_FLAG)) {
                        cur[i] = val[i];
                        val[i] = lab_prev[cur[i]];
                        more |= !(val[i] & ROOT_FLAG);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < RH; ++i) {
                if (!(w[i] & ROOT_FLAG) && cur[i] != w[i]) lab_prev[w[i]] = cur[i];
                own[h + i] = 0;
                ownS[h + i] = 0;
                if (vc && row_ok(h + i)) set_own(h + i, gin(gx, row_y(h + i), row_z(h + i)), val[i], tho[i]);
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < R; ++j) {
            own[j] = 0;
            ownS[j] = 0;
            if (vc && row_ok(j)) {
                const uint32_t g = gin(gx, row_y(j), row_z(j));
                W th0 = 0;
                if constexpr (IS_XY) th0 = ((const GLOBAL float *)d.state)[g];
                if constexpr (IS_CK) th0 = ((const GLOBAL uint16_t *)d.state)[g];
                set_own(j, g, 0u, th0);
            }
        }
    }
    // state byte of a site outside this wavefront's rows (halo, next block)
    auto state_byte = [&](uint32_t g) -> uint32_t {
        V unused;
        return (uint32_t)value_at(g, unused);
    };
    // incoming values of up to four sites outside this wavefront's rows (those
    // with use[i]): their previous labels are resolved in lock-step, the first
    // loads of all four and then their roots' words in flight together, where
    // value_at walks one chain after the other
    auto values4 = [&](const uint32_t *g, const bool *use, V *v, V *vs) {
        if (!from_labels) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                v[i] = 0;
                vs[i] = 0;
                if (use[i]) v[i] = value_at(g[i], vs[i]);
            }
            return;
        }
        uint32_t w[4], val[4];
        W th[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            w[i] = use[i] ? lab_prev[g[i]] : ROOT_FLAG;
            th[i] = 0;
            if constexpr (IS_XY) th[i] = use[i] ? th_prev[g[i]] : 0.0f;
            if constexpr (IS_CK) th[i] = use[i] ? (uint32_t)ck_prev[g[i]] : 0u;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) val[i] = (w[i] & ROOT_FLAG) ? w[i] : lab_prev[w[i]];
        bool more = false;
#pragma unroll
        for (int i = 0; i < 4; ++i) more |= !(val[i] & ROOT_FLAG);
        uint32_t rounds = 0;
        while (more) {
            if (++rounds > d.walk_cap) {
                flag_error(d, ERR_WALK);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (!(val[i] & ROOT_FLAG)) val[i] = ROOT_FLAG;
                break;
            }
            more = false;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (!(val[i] & ROOT_FLAG)) {
                    val[i] = lab_prev[val[i]];
                    more |= !(val[i] & ROOT_FLAG);
                }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            v[i] = 0;
            vs[i] = 0;
            if (!use[i]) continue;
            if constexpr (IS_XY) {
                xy_sincos((val[i] & 1u) ? xy_reflect(th[i], phi_prev) : th[i], s_cs, v[i], vs[i]);
            } else if constexpr (IS_CK) {
                v[i] = (val[i] & 1u) ? clock_mirror(th[i], axis_prev, uq) : th[i];
            } else {
                v[i] = (V)state_of_decision<MODEL>(val[i] & 0xffu);
            }
        }
    };
    // halo column: XY: lane j < R holds the site right of the tile in row j;
    // Ising / Potts: lane g < NG holds that column's four rows of group g
    V hx = 0, hxS = 0;
    uint32_t hxg = 0;
    if (VEC && c < R) {
        const int ly = DIM == 2 ? r0 + c : c % TY, lz = DIM == 2 ? 0 : r0 / TY + c / TY;
        if (ly < ey && lz < ez) {
            if constexpr (NBX) {
                if (from_labels) xy_sincos(s_nth[(wv * NBS + NBS - 1) * 64 + c], s_cs, hx, hxS);
                else hx = value_at(gin(gxr, ly, lz), hxS);
            } else {
                hx = value_at(gin(gxr, ly, lz), hxS);
            }
        }
    }
    if (!VEC && c < NG) {
        uint32_t hg[4];
        bool hu[4];
        V hv[4], hvs[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int j = 4 * c + m;
            const int ly = DIM == 2 ? r0 + j : j % TY, lz = DIM == 2 ? 0 : r0 / TY + j / TY;
            hu[m] = ly < ey && lz < ez;
            hg[m] = hu[m] ? gin(gxr, ly, lz) : 0u;
        }
        values4(hg, hu, hv, hvs);
#pragma unroll
        for (int m = 0; m < 4; ++m) hxg |= (uint32_t)hv[m] << (8 * m);
    }

    // ---- (1) bonds and measurement --------------------------------------------
    // Bond bits of row j = 4 g + m sit at bit 8 m + 7 of bxg[g] / byg[g] / bzg[g]
    // (+x, +y, +z): the byte layout of the four-rows-at-once tests below.
    uint32_t bxg[NG], byg[NG], bzg[NG];
    int cnt_al = 0, cnt_m = 0;
    // Potts, q <= HPACK_Q: this lane's count of every state, 6 bits a state
    // (a lane holds R < 64 rows), summed over the wavefront at the end
    constexpr int HPACK_Q = 10;
    static_assert(R < 64, "state counts are packed in 6-bit fields");
    unsigned long long hpack = 0ull;
    double e_acc = 0.0, sx_acc = 0.0, sy_acc = 0.0;
    const uint32_t thr_hi = d.thr_hi;
    const uint32_t q4 = (uL + 3u) >> 2;  // column blocks per plane row
    uint4 zw = make_uint4(0u, 0u, 0u, 0u);
    // Ising / Potts: the states of a group's four rows packed one per byte
    uint32_t P[NG];
    // The first rows of wavefront w + 1 (2D: one row; 3D: one plane) are the
    // +y / +z neighbours of wavefront w's last rows.  Wavefront w + 1 hands
    // them over through LDS, in wavefront w's part of s_par (nodes
    // [64 r0, 64 (r0 + R)), which w writes only once its own scan starts), so
    // that w neither loads nor resolves them again (3D Ising / Potts: the
    // packed states of those row groups).  2D (one row per wavefront) and XY
    // (fewer wavefronts per SIMD) do not: there the barrier cost more than
    // the loads it saved.
    constexpr int HG = (DIM == 2) ? 1 : TY / 4;  // row groups handed over
    constexpr bool HAND = !VEC && DIM == 3;
    static_assert(HG <= NG, "the handed-over rows fit the receiving wavefront's nodes");
    if constexpr (!VEC) {
#pragma unroll
        for (int gi = 0; gi < NG; ++gi)
            P[gi] = own[4 * gi] | (own[4 * gi + 1] << 8) | (own[4 * gi + 2] << 16) | (own[4 * gi + 3] << 24);
        if (HAND && wv > 0) {
#pragma unroll
            for (int gi = 0; gi < HG; ++gi) s_par[TX * (r0 - R) + TX * gi + c] = (int)P[gi];
        }
        // a tile with all TZ planes: the last wavefront's +z plane is the next
        // tile's first plane; every wavefront resolves rows of it (ly = wv,
        // wv + NW, ...) into the last wavefront's hand-over slots, byte ly % 4
        // of word ly / 4, instead of the last wavefront loading them all while
        // the others wait for it at the next barrier
        if constexpr (HAND) {
            if (ez == TZ) {  // uniform
                typedef __attribute__((address_space(3))) uint8_t lds_u8;
                lds_u8 *last = (lds_u8 *)&s_par[TX * (R * (NW - 1))];
                for (int ly = wv; ly < TY; ly += NW)
                    last[4 * (TX * (ly / 4) + c) + (ly % 4)] =
                        (vc && ly < ey) ? (uint8_t)state_byte(gat(gx, ly, TZ)) : (uint8_t)0;
            }
        }
        if (HAND) __syncthreads();
    }
    // packed states of row group i of the first rows of wavefront wv + 1
    auto handed = [&](int i) -> uint32_t { return (uint32_t)s_par[TX * r0 + TX * i + c]; };
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
        const int jf = 4 * gi;
        bxg[gi] = byg[gi] = bzg[gi] = 0;
        if (!row_ok(jf)) continue;  // uniform: the group's first row is outside the lattice
        const uint32_t gyf = (uint32_t)(y0 + row_y(jf)), gzf = (uint32_t)(z0 + row_z(jf));
        uint4 w = make_uint4(0u, 0u, 0u, 0u);
        if (full) {
            w = philox(make_uint4(gx + uL * ((gyf >> 2) + q4 * gzf), n, (uint32_t)TAG_BOND, rep), key0, key1);
            if (DIM == 3 && ((TY % 8) != 0 || (row_y(jf) % 8) == 0))
                zw = philox(make_uint4(gx + uL * ((gyf >> 3) + ((uL + 7u) >> 3) * gzf), n, (uint32_t)TAG_BOND_Z, rep),
                            key0, key1);
        }
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
        // z primaries of the group: lanes 0,1 of the BOND_Z block for y mod 8 < 4, else lanes 2,3
        const bool zhi = (gyf & 4u) != 0;
        const uint32_t zwa = zhi ? zw.z : zw.x, zwb = zhi ? zw.w : zw.y;
        const uint32_t zs[4] = {zwa >> 16, zwa & 0xffffu, zwb >> 16, zwb & 0xffffu};
        if constexpr (!VEC) {
            // rows of the group inside the lattice, bit 7 of their byte
            uint32_t vb = 0;
#pragma unroll
            for (int m = 0; m < 4; ++m)
                if (row_ok(jf + m)) vb |= 0x80u << (8 * m);
            if (!vc) vb = 0;
            // +y neighbours: the group shifted by one row, the fifth row from the
            // next group, a load across the wave block, or the wrapped row
            uint32_t PU = 0;
            const int l3 = row_y(jf + 3), z3 = row_z(jf + 3);
            if (row_ok(jf + 3)) {
                uint32_t nb;
                const bool nb_own = DIM == 2 ? (jf + 4 < R && l3 + 1 < ey) : (l3 + 1 < TY && l3 + 1 < ey);
                if (nb_own) nb = P[gi + 1 < NG ? gi + 1 : gi] & 0xffu;
                else nb = vc ? state_byte(gat(gx, l3 + 1, z3)) : 0u;
                PU = __builtin_amdgcn_alignbyte(nb, P[gi], 1);
            } else {
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int j = jf + m;
                    if (!row_ok(j)) continue;
                    uint32_t ub;
                    if (row_y(j) + 1 < ey && m < 3) ub = (P[gi] >> (8 * (m + 1))) & 0xffu;
                    else ub = vc ? state_byte(gat(gx, row_y(j) + 1, row_z(j))) : 0u;
                    PU |= ub << (8 * m);
                }
            }
            // +z neighbours: the group one plane ahead in this wave, else loads
            uint32_t PZ = 0;
            if (DIM == 3) {
                const int lz = row_z(jf);
                if (jf + TY < R && lz + 1 < ez) {
                    PZ = P[gi + TY / 4 < NG ? gi + TY / 4 : gi];
                } else if (HAND && lz + 1 < TZ && lz + 1 < ez) {
                    PZ = handed((jf % TY) / 4);  // the first plane of wavefront wv + 1
                } else if (HAND && lz + 1 == TZ && ez == TZ) {
                    PZ = handed((jf % TY) / 4);  // the next tile's first plane, resolved by every wavefront
                } else if (vc) {
                    uint32_t zg[4];
                    bool zu[4];
                    V zv[4], zvs[4];
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        zu[m] = row_ok(jf + m);
                        zg[m] = zu[m] ? gat(gx, row_y(jf + m), lz + 1) : 0u;
                    }
                    values4(zg, zu, zv, zvs);
#pragma unroll
                    for (int m = 0; m < 4; ++m) PZ |= (uint32_t)zv[m] << (8 * m);
                }
            }
            // +x neighbours: lane c + 1, the last column from the halo
            uint32_t PR = from_right(P[gi]);
            if (c == ex - 1) PR = (uint32_t)__builtin_amdgcn_readlane((int)hxg, gi);
            const uint32_t EQX = zero_bytes(P[gi] ^ PR) & vb;
            const uint32_t EQY = zero_bytes(P[gi] ^ PU) & vb;
            const uint32_t EQZ = (DIM == 3) ? (zero_bytes(P[gi] ^ PZ) & vb) : 0u;
            if (meas) {
                cnt_al += __popc(EQX) + __popc(EQY) + __popc(EQZ);
                if (MODEL == ISING) {
                    cnt_m += __popc(vb) - 2 * __popc(P[gi] & vb);
                } else if (d.q <= HPACK_Q) {
                    // one count per state and group instead of an LDS atomic per
                    // site: those serialise when a wavefront holds few states
                    for (int st = 0; st < d.q; ++st)
                        hpack += (unsigned long long)__popc(zero_bytes(P[gi] ^ (0x01010101u * (uint32_t)st)) & vb)
                                 << (6 * st);
                } else {
#pragma unroll
                    for (int m = 0; m < 4; ++m)
                        if (vb & (0x80u << (8 * m))) atomicAdd(&s_hist[(P[gi] >> (8 * m)) & 0xffu], 1);
                }
            }
            if (full) {
                // primary < threshold high half, per row, moved to bit 7 of the row's byte
                uint32_t tx[4], ty_[4], tz_[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    tx[m] = (ws[m] >> 16) - thr_hi;
                    ty_[m] = (ws[m] & 0xffffu) - thr_hi;
                    tz_[m] = zs[m] - thr_hi;
                }
                const uint32_t LTX = __builtin_amdgcn_perm(tx[1], tx[0], 0x0c0c0703u) |
                                     __builtin_amdgcn_perm(tx[3], tx[2], 0x07030c0cu);
                const uint32_t LTY = __builtin_amdgcn_perm(ty_[1], ty_[0], 0x0c0c0703u) |
                                     __builtin_amdgcn_perm(ty_[3], ty_[2], 0x07030c0cu);
                bxg[gi] = LTX & EQX;
                byg[gi] = LTY & EQY;
                if (DIM == 3) {
                    const uint32_t LTZ = __builtin_amdgcn_perm(tz_[1], tz_[0], 0x0c0c0703u) |
                                         __builtin_amdgcn_perm(tz_[3], tz_[2], 0x07030c0cu);
                    bzg[gi] = LTZ & EQZ;
                }
                // a primary equal to the threshold's high half needs the secondary (rare)
                uint32_t tmin = min(min(min(tx[0], tx[1]), min(tx[2], tx[3])), min(min(ty_[0], ty_[1]), min(ty_[2], ty_[3])));
                if (DIM == 3) tmin = min(tmin, min(min(tz_[0], tz_[1]), min(tz_[2], tz_[3])));
                if (tmin == 0u) {
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const uint32_t bit = 0x80u << (8 * m);
                        const uint32_t g = gin(gx, row_y(jf + m), row_z(jf + m));
                        if ((EQX & bit) && tx[m] == 0u && bond_secondary(key0, key1, rep, n, DIM, g, 0) < d.thr_lo)
                            bxg[gi] |= bit;
                        if ((EQY & bit) && ty_[m] == 0u && bond_secondary(key0, key1, rep, n, DIM, g, 1) < d.thr_lo)
                            byg[gi] |= bit;
                        if (DIM == 3 && (EQZ & bit) && tz_[m] == 0u &&
                            bond_secondary(key0, key1, rep, n, DIM, g, 2) < d.thr_lo)
                            bzg[gi] |= bit;
                    }
                }
            }
        } else {
            // +z neighbours outside this wavefront's rows, the group's four at once
            V zbuf[4] = {0, 0, 0, 0}, zbufS[4] = {0, 0, 0, 0};
            if (DIM == 3 && !(jf + TY < R && row_z(jf) + 1 < ez)) {
                uint32_t zg[4];
                bool zu[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    zu[m] = vc && row_ok(jf + m);
                    zg[m] = zu[m] ? gat(gx, row_y(jf + m), row_z(jf + m) + 1) : 0u;
                }
                if constexpr (NBX) {
                    if (from_labels) {
#pragma unroll
                        for (int m = 0; m < 4; ++m)
                            if (zu[m]) xy_sincos(s_nth[(wv * NBS + jf + m) * 64 + c], s_cs, zbuf[m], zbufS[m]);
                    } else {
                        values4(zg, zu, zbuf, zbufS);
                    }
                } else {
                    values4(zg, zu, zbuf, zbufS);
                }
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int j = jf + m;
                if (!row_ok(j)) continue;
                const int ly = row_y(j), lz = row_z(j);
                // +y neighbour: the next row of this wave, else a load (halo or next wave)
                V up, upS;
                if (DIM == 2 ? (j + 1 < R && ly + 1 < ey) : (ly + 1 < min(TY, ey))) {
                    up = own[j + 1 < R ? j + 1 : j];
                    upS = ownS[j + 1 < R ? j + 1 : j];
                } else {
                    up = 0;
                    upS = 0;
                    if (vc) {
                        if constexpr (NBX) {
                            if (from_labels) xy_sincos(s_nth[(wv * NBS + R + j / TY) * 64 + c], s_cs, up, upS);
                            else up = value_at(gat(gx, ly + 1, lz), upS);
                        } else {
                            up = value_at(gat(gx, ly + 1, lz), upS);
                        }
                    }
                }
                V zn = 0, znS = 0;
                if (DIM == 3) {
                    if (j + TY < R && lz + 1 < ez) {
                        zn = own[j + TY < R ? j + TY : j];
                        znS = ownS[j + TY < R ? j + TY : j];
                    } else {
                        zn = zbuf[m];
                        znS = zbufS[m];
                    }
                }
                const uint32_t g = gin(gx, ly, lz);
                if constexpr (IS_CK) {
                    // clock: integer states; measurement from the paper's tables
                    uint32_t rt = from_right((uint32_t)own[j]);
                    if (c == ex - 1) rt = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)hx, j);
                    const uint32_t pi = own[j];
                    if (meas && vc) {
                        sx_acc += s_trig[pi];
                        sy_acc += s_trig[uq + pi];
                        // pair energy -cos(2 pi (p_i - p_j) / q) = -rule[(p_i - p_j) mod q]
                        e_acc -= s_trig[(pi + uq - rt) % uq];
                        e_acc -= s_trig[(pi + uq - (uint32_t)up) % uq];
                        if (DIM == 3) e_acc -= s_trig[(pi + uq - (uint32_t)zn) % uq];
                    }
                    if (full && vc) {
                        const uint32_t px = ws[m] >> 16, py = ws[m] & 0xffffu, pz = zs[m];
                        const uint32_t onx = clock_bond(pi, rt, axis, d, px, g, 0, key0, key1, rep, n, DIM);
                        const uint32_t ony = clock_bond(pi, up, axis, d, py, g, 1, key0, key1, rep, n, DIM);
                        const uint32_t onz = DIM == 3 ? clock_bond(pi, zn, axis, d, pz, g, 2, key0, key1, rep, n, DIM) : 0u;
                        bxg[gi] |= onx << (8 * m + 7);
                        byg[gi] |= ony << (8 * m + 7);
                        bzg[gi] |= onz << (8 * m + 7);
                    }
                    continue;
                }
                V rt = from_right_d(own[j]), rtS = from_right_d(ownS[j]);
                if (c == ex - 1) {
                    rt = readlane_d(hx, j);
                    rtS = readlane_d(hxS, j);
                }
                if (meas && vc) {
                    sx_acc += own[j];
                    sy_acc += ownS[j];
                    e_acc -= own[j] * rt + ownS[j] * rtS;
                    e_acc -= own[j] * up + ownS[j] * upS;
                    if (DIM == 3) e_acc -= own[j] * zn + ownS[j] * znS;
                }
                if (full && vc) {
                    const uint32_t px = ws[m] >> 16, py = ws[m] & 0xffffu, pz = zs[m];
                    const double si = own[j] * cphi + ownS[j] * sphi;
                    uint32_t onx = xy_bond_fast(d.two_beta, si, rt * cphi + rtS * sphi, px);
                    uint32_t ony = xy_bond_fast(d.two_beta, si, up * cphi + upS * sphi, py);
                    uint32_t onz = 0;
                    if (DIM == 3) onz = xy_bond_fast(d.two_beta, si, zn * cphi + znS * sphi, pz);
                    if ((onx | ony | onz) & 2u) {  // rare: p within the margin of the primary interval
                        const float ti = theta_in(g);
                        if (onx == 2u)
                            onx = xy_bond_exact(ti, theta_in((c == ex - 1) ? gin(gxr, ly, lz) : g + 1u), g, phi,
                                                d.two_beta, px, key0, key1, rep, n, DIM, 0);
                        if (ony == 2u)
                            ony = xy_bond_exact(ti, theta_in(gat(gx, ly + 1, lz)), g, phi, d.two_beta, py, key0,
                                                key1, rep, n, DIM, 1);
                        if (DIM == 3 && onz == 2u)
                            onz = xy_bond_exact(ti, theta_in(gat(gx, ly, lz + 1)), g, phi, d.two_beta, pz, key0,
                                                key1, rep, n, DIM, 2);
                    }
                    bxg[gi] |= onx << (8 * m + 7);
                    byg[gi] |= ony << (8 * m + 7);
                    bzg[gi] |= onz << (8 * m + 7);
                }
            }
        }
        if (full && d.store_bonds && vc) {
            // bond byte of each row: bit mu = bond to the +mu neighbour
            const uint32_t B = (bxg[gi] >> 7) | (byg[gi] >> 6) | (bzg[gi] >> 5);
#pragma unroll
            for (int m = 0; m < 4; ++m)
                if (row_ok(jf + m))
                    ((GLOBAL uint8_t *)d.bond)[gin(gx, row_y(jf + m), row_z(jf + m))] = (uint8_t)(B >> (8 * m));
        }
    }
    auto bit_of = [&](const uint32_t *arr, int j) -> uint32_t { return (arr[j >> 2] >> (8 * (j & 3) + 7)) & 1u; };

    // ---- measurement partials of this tile -----------------------------------
    if (meas) {
        GLOBAL int64_t *part = (GLOBAL int64_t *)d.part + (int64_t)t * d.nslots;
        // a lattice of one tile has no faces and the plain form launches no
        // merge for it: the workgroup writes the sweep's record itself (the
        // merge's reduction of one tile's partials gives the same values)
        const bool own_rec = full && d.ntiles == 1 && d.rec_row0 >= 0 && d.rec_row0 + (int64_t)k < d.rec_cap;
        GLOBAL int64_t *rec = (GLOBAL int64_t *)d.rec + (own_rec ? (d.rec_row0 + (int64_t)k) * d.nslots : 0);
        if (VEC) {
            const double a = wave_sum_d(e_acc), b = wave_sum_d(sx_acc), cc = wave_sum_d(sy_acc);
            if (c == 0) {
                s_red[wv][0] = a;
                s_red[wv][1] = b;
                s_red[wv][2] = cc;
            }
        } else {
            const int a = wave_sum_i(cnt_al), b = wave_sum_i(cnt_m);
            if (MODEL == POTTS && d.q <= HPACK_Q)
                for (int st = 0; st < d.q; ++st) {
                    const int v = wave_sum_i((int)((hpack >> (6 * st)) & 63ull));
                    if (c == 0) atomicAdd(&s_hist[st], v);
                }
            if (c == 0) {
                s_red[wv][0] = (double)a;
                s_red[wv][1] = (double)b;
            }
        }
        __syncthreads();
        if (tid == 0) {
            // wavefronts in order (a fixed order: deterministic XY sums)
            double v[3] = {0.0, 0.0, 0.0};
            for (int w = 0; w < NW; ++w)
                for (int q = 0; q < 3; ++q) v[q] += s_red[w][q];
            if (VEC) {
                for (int q = 0; q < 3; ++q) part[q] = __double_as_longlong(v[q]);
                if (own_rec)
                    for (int q = 0; q < 3; ++q) rec[q] = __double_as_longlong(v[q]);
            } else {
                part[0] = (int64_t)v[0];
                if (MODEL == ISING) part[1] = (int64_t)v[1];
                if (own_rec) {
                    rec[0] = (int64_t)v[0];
                    if (MODEL == ISING) rec[1] = (int64_t)v[1];
                }
            }
        }
        if (MODEL == POTTS) {
            for (int q = tid; q < d.q; q += NT) {
                part[1 + q] = s_hist[q];
                if (own_rec) rec[1 + q] = s_hist[q];
            }
            // the counts share memory with the equivalence queues: for q > 64
            // wavefronts 1.. read slots of wavefront 0's queue (and 2, 3 of 1's),
            // so every read completes before any wavefront starts queueing
            if (d.q > 64) __syncthreads();  // uniform condition
        }
    }
    if (!full) return;

    // ---- (2) local labelling ---------------------------------------------------
    const unsigned long long upto = (c == 63) ? ~0ull : ((2ull << c) - 1ull);
    int qn = 0;  // entries in this wave's queue (uniform)
    auto flush = [&]() {
        if (qn) flush_queue((lds_int *)s_par, (const lds_u32 *)s_q[wv], qn, c);
        qn = 0;
    };
    // a ballot of one comparison is that comparison's lane mask (a compound
    // condition is rebuilt lane by lane first)
    auto ballot = [](bool p) -> unsigned long long { return __builtin_amdgcn_ballot_w64(p); };
    const unsigned long long vmask = (ex >= 64) ? ~0ull : ((1ull << ex) - 1ull);  // lanes c < ex
    // queue (a, b) from the lanes where `want` holds
    auto push = [&](bool want, int a, int b) {
        const unsigned long long m = ballot(want);
        if (!m) return;
        if (qn > QCAP - 64) flush();
        if (want) {
            const int pos = qn + __popcll(m & ((1ull << c) - 1ull));
            s_q[wv][pos] = ((uint32_t)a << 16) | (uint32_t)b;
        }
        qn += __popcll(m);
    };
    int labr[R];  // label of the run of (c, row j): a union-find node of this tile
    {
        int prevlab = NONE;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            labr[j] = NONE;
            if (!row_ok(j)) {  // ragged tile: rows past the lattice edge
                prevlab = NONE;
                continue;
            }
            const int rr = r0 + j;
            // x bonds to lane c + 1 < ex
            const unsigned long long xb = ballot(bit_of(bxg, j) != 0u) & (vmask >> 1);
            // the masks the cross-block and periodic links read (node_of):
            // full 2D tiles need only each wavefront's first and last row
            constexpr int HR = (DIM == 2) ? 1 : TY;
            const bool need_xm = !FULL || j < HR || j >= R - HR || (DIM == 3 && (j % TY == 0 || j % TY == TY - 1));
            if (need_xm && c == 0) s_xm[rr] = xb;
            const int rs = 63 - __clzll((long long)(~(xb << 1) & upto));
            const int node = rs + TX * rr;
            // bonded to the row above / the plane behind (inside the wavefront's rows)
            const bool up_in = j > 0 && row_y(j) > 0, back_in = DIM == 3 && j >= TY;
            const bool ya = up_in && vc && bit_of(byg, j > 0 ? j - 1 : 0);
            const bool zb = back_in && vc && bit_of(bzg, j >= TY ? j - TY : 0);
            const int ca = ya ? prevlab : NONE;
            const int cb = zb ? labr[j >= TY ? j - TY : 0] : NONE;
            const int cand = min(ca, cb);
            // the run's label: the smallest label its sites inherit, else its own
            // start (every inherited label is a smaller node, so s_par stays a
            // forest pointing downwards).  The run start seeds the slot, the
            // bonded sites lower it, all read it back: the wavefront's LDS
            // operations complete in order.
            if (vc && c == rs) s_par[node] = node;
            if (ya || zb)
                __hip_atomic_fetch_min((lds_int *)&s_par[node], cand, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            const int lab = vc ? __hip_atomic_load((lds_int *)&s_par[node], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)
                               : NONE;
            // a bonded neighbour with another label: one entry per stretch of equal labels
            const int cal = (int)from_left((uint32_t)ca);
            push(ya && ca != lab && (c == rs || cal != ca), ca, lab);
            if (DIM == 3) {
                const int cbl = (int)from_left((uint32_t)cb);
                push(zb && cb != lab && (c == rs || cbl != cb), cb, lab);
            }
            // periodic x bond of a tile that spans the lattice: to (0, row)
            if (d.tiles[0] == 1) push(c == ex - 1 && bit_of(bxg, j), TX * rr, lab);
            prevlab = lab;
            labr[j] = lab;
        }
    }
    __syncthreads();  // every row's x mask and run-start links written
    // run-start node of site (c, tile row r)
    auto node_of = [&](int r) -> int {
        const unsigned long long xm = s_xm[r];
        return (63 - __clzll((long long)(~(xm << 1) & upto))) + TX * r;
    };
#pragma unroll
    for (int j = 0; j < R; ++j) {
        if (!row_ok(j)) continue;
        const int rr = r0 + j, ly = row_y(j), lz = row_z(j);
        const bool oy = vc && bit_of(byg, j), oz = vc && bit_of(bzg, j);
        // +y bond into the next wavefront's block (2D)
        if (DIM == 2 && j == R - 1 && ly + 1 < ey) push(oy, node_of(rr + 1), node_of(rr));
        // +z bond into the next wavefront's block (3D)
        if (DIM == 3 && j + TY >= R && lz + 1 < ez) push(oz, node_of(rr + TY < ROWS ? rr + TY : rr), node_of(rr));
        // periodic bonds of a tile that spans the lattice
        if (ly == ey - 1 && d.tiles[1] == 1) push(oy, node_of(TY * lz), node_of(rr));
        if (DIM == 3 && lz == ez - 1 && d.tiles[2] == 1) push(oz, node_of(ly), node_of(rr));
    }
    flush();
    __syncthreads();
    // root of every row's label: pointer jumping on all rows at once (the
    // parents only ever point to smaller nodes, so this ends)
    // (two jumps per pass, alternating between two arrays: no copies)
    int root[R], nxt[R];
#pragma unroll
    for (int j = 0; j < R; ++j) root[j] = (vc && row_ok(j)) ? labr[j] : -1;
    while (true) {
        bool moving = false;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            nxt[j] = (FULL || root[j] >= 0) ? s_par[FULL ? root[j] : max(root[j], 0)] : -1;
            moving |= nxt[j] != root[j];
        }
        if (!__any(moving)) break;  // root[] final
        moving = false;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            root[j] = (FULL || nxt[j] >= 0) ? s_par[FULL ? nxt[j] : max(nxt[j], 0)] : -1;
            moving |= root[j] != nxt[j];
        }
        if (!__any(moving)) break;  // root[] == nxt[], final
    }

    // ---- local roots draw the cluster decision; labels and faces to HBM -------
    const int F0 = d.face_len[0], F1 = d.face_len[1], F2 = (DIM == 3) ? d.face_len[2] : 0;
    GLOBAL int32_t *fo0 = (GLOBAL int32_t *)d.face + d.face_off[0] + (int64_t)t * 2 * F0;
    GLOBAL int32_t *fo1 = (GLOBAL int32_t *)d.face + d.face_off[1] + (int64_t)t * 2 * F1;
    GLOBAL int32_t *fo2 = (GLOBAL int32_t *)d.face + d.face_off[DIM == 3 ? 2 : 0] + (int64_t)t * 2 * F2;
    const bool fx = d.tiles[0] > 1, fy = d.tiles[1] > 1, fz = (DIM == 3) && d.tiles[2] > 1;
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
        const int jf = 4 * gi;
        if (!row_ok(jf)) continue;
        bool isr[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int j = jf + m, rr = r0 + j;
            isr[m] = row_ok(j) && vc && root[j] == c + TX * rr;
        }
        uint32_t dec[4] = {0u, 0u, 0u, 0u};  // Potts q > 2: the decisions of the group
        if (!bits_dec && __ballot(isr[0] || isr[1] || isr[2] || isr[3])) {
            const uint32_t gyf = (uint32_t)(y0 + row_y(jf)), gzf = (uint32_t)(z0 + row_z(jf));
            const uint4 w = philox(make_uint4(gx + uL * ((gyf >> 2) + q4 * gzf), n, (uint32_t)TAG_CLUSTER, rep), key0, key1);
            const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int m = 0; m < 4; ++m) dec[m] = (uint32_t)(((uint64_t)ws[m] * (uint64_t)d.q) >> 32);
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int j = jf + m, rr = r0 + j;
            if (!row_ok(j)) continue;
            const int ly = row_y(j), lz = row_z(j);
            const int32_t rg = (int32_t)gidx(FULL ? root[j] : max(root[j], 0));
            const uint32_t dm = bits_dec ? (uint32_t)(s_dm[rr] >> c) & 1u : dec[m];
            if (vc) (g_label + gin((uint32_t)x0, ly, lz))[c] = isr[m] ? (ROOT_FLAG | dm) : (uint32_t)rg;
            // faces for the global merge: the out side marks a bond across the face
            if (fx) {
                if (c == ex - 1) fo0[rr] = bit_of(bxg, j) ? rg : -1;
                if (c == 0) fo0[F0 + rr] = rg;
            }
            if (fy && vc) {
                if (ly == ey - 1) fo1[c + TX * lz] = bit_of(byg, j) ? rg : -1;
                if (ly == 0) fo1[F1 + c + TX * lz] = rg;
            }
            if (DIM == 3 && fz && vc) {
                if (lz == ez - 1) fo2[c + TX * ly] = bit_of(bzg, j) ? rg : -1;
                if (lz == 0) fo2[F2 + c + TX * ly] = rg;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// (3) every site takes its cluster root's decision -- once per launch chain,
// for its last sweep (the bond kernel applies the earlier sweeps' decisions).
//
// A site's label word is its tile root's global index (or, for a root, ROOT
// | decision); the merge may have linked tile roots to roots elsewhere.  Lane
// = column, wavefront w owns rows [w R, (w+1) R) as in k_bond.  All rows'
// words are loaded first, then all their roots' words, so the dependent
// loads of a lane overlap; the few chains the merge made longer are walked in
// lock-step rounds, and the final root is written back into the tile root
// so that later workgroups take one hop.
// ---------------------------------------------------------------------------
template <int MODEL, int DIM, int TX, int TY, int TZ, int NW>
__global__ void __launch_bounds__(64 * NW, (MODEL == XY) ? 4 : 8) k_flip(const InstDesc *__restrict__ descs,
                                              const int2 *__restrict__ tmap, uint32_t k)
{
    constexpr int ROWS = TY * TZ;
    constexpr int R = ROWS / NW;
    static_assert(TX == 64 && ROWS % NW == 0, "lane = column, whole rows per wavefront");
    __shared__ double s_phi;
    __shared__ uint32_t s_axis;
    const int2 tm = tmap[tile_slot()];
    if (tm.x < 0) return;
    // a reference: fields load from the (read-only) descriptor when used,
    // instead of a copy that would hold them all in scalar registers
    const InstDesc &d = descs[tm.x];
    if (k == FLIP_LAST) {
        if (d.count == 0) return;
        k = d.count - 1u;  // the chain's last sweep
    }
    if (k >= d.count) return;
    const uint32_t n = d.sweep0 + k;
    const int L = d.L;
    const uint32_t uL = (uint32_t)L;
    const int t = tm.y;
    const int tx = t % d.tiles[0];
    const int ty = (t / d.tiles[0]) % d.tiles[1];
    const int tz = (DIM == 3) ? t / (d.tiles[0] * d.tiles[1]) : 0;
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
    const int ex = min(TX, L - x0), ey = min(TY, L - y0), ez = (DIM == 3) ? min(TZ, L - z0) : 1;
    const int tid = threadIdx.x;
    // the wavefront index is uniform: readfirstlane lets everything derived
    // from it (rows, global addresses) live in scalar registers
    const int c = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r0 = wv * R;
    const bool vc = c < ex;
    if (MODEL == XY) {
        if (tid == 0) s_phi = xy_phi(d, n);
        __syncthreads();
    }
    if (MODEL == CLOCK) {
        if (tid == 0) s_axis = clock_axis(d, n);
        __syncthreads();
    }
    GLOBAL uint32_t *g_label = (GLOBAL uint32_t *)labels_of(d, n);
    auto row_ok = [&](int j) -> bool {
        const int rr = r0 + j;
        return (rr % TY) < ey && (rr / TY) < ez;
    };
    auto gsite = [&](int j) -> uint32_t {
        const int rr = r0 + j;
        return (uint32_t)(x0 + c) + uL * ((uint32_t)(y0 + rr % TY) + uL * (uint32_t)(z0 + rr / TY));
    };

    // the rows' loads in flight together, in two batches from 16 rows per
    // wavefront on (registers for 8 wavefronts per SIMD)
    constexpr int RH = (R >= 16) ? R / 2 : R;
    const double phi = (MODEL == XY) ? s_phi : 0.0;
    const uint32_t axis = (MODEL == CLOCK) ? s_axis : 0u;
#pragma unroll 1
    for (int h = 0; h < R; h += RH) {
        uint32_t w[RH], cur[RH], val[RH];
#pragma unroll
        for (int i = 0; i < RH; ++i) {
            w[i] = ROOT_FLAG;
            if (vc && row_ok(h + i)) w[i] = g_label[gsite(h + i)];
        }
        // cur: the tile root (or the site itself); val: its word
#pragma unroll
        for (int i = 0; i < RH; ++i) {
            cur[i] = w[i];
            val[i] = (w[i] & ROOT_FLAG) ? w[i] : g_label[w[i]];
        }
        // chains the merge made longer, walked in lock-step rounds
        bool more = false;
#pragma unroll
        for (int i = 0; i < RH; ++i) more |= !(val[i] & ROOT_FLAG);
        uint32_t rounds = 0;
        while (__any(more)) {
            if (++rounds > d.walk_cap) {  // uniform
                if (more) flag_error(d, ERR_WALK);
#pragma unroll
                for (int i = 0; i < RH; ++i) {
                    cur[i] = w[i];
                    if (!(val[i] & ROOT_FLAG)) val[i] = ROOT_FLAG;
                }
                break;
            }
            more = false;
#pragma unroll
            for (int i = 0; i < RH; ++i) {
                if (!(val[i] & ROOT_FLAG)) {
                    cur[i] = val[i];
                    val[i] = g_label[cur[i]];
                    more |= !(val[i] & ROOT_FLAG);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < RH; ++i) {
            // point the tile root straight at the final root
            if (!(w[i] & ROOT_FLAG) && cur[i] != w[i]) g_label[w[i]] = cur[i];
            if (!vc || !row_ok(h + i)) continue;
            const uint32_t dec = val[i] & 0xffu;
            const uint32_t g = gsite(h + i);
            if (MODEL == ISING) {
                ((GLOBAL int8_t *)d.state)[g] = dec ? (int8_t)-1 : (int8_t)1;
            } else if (MODEL == POTTS) {
                ((GLOBAL uint8_t *)d.state)[g] = (uint8_t)dec;
            } else if (MODEL == CLOCK) {
                // the state that entered the sweep, mirrored or kept
                const uint32_t p = ((const GLOBAL uint16_t *)((n & 1u) ? d.theta_w[1] : d.theta_w[0]))[g];
                ((GLOBAL uint16_t *)d.state)[g] = (uint16_t)(dec ? clock_mirror(p, axis, (uint32_t)d.q) : p);
            } else {
                // the angle that entered the sweep, mirrored or kept
                const float t = ((const GLOBAL float *)((n & 1u) ? d.theta_w[1] : d.theta_w[0]))[g];
                ((GLOBAL float *)d.state)[g] = dec ? xy_reflect(t, phi) : t;
            }
        }
    }
}

template <int MODEL, int DIM>
static hipError_t bond_dispatch(int v, const InstDesc *dd, const int2 *tm, int nt, int nf, uint32_t k, int mode,
                                hipStream_t s, hipEvent_t t0, hipEvent_t t1)
{
    // Full tiles first, then the tiles cut by the lattice edge. Timing events
    // ride on the first and the last launch; untimed launches (and those a
    // graph captures) take the plain launch path.
    const bool timed = t0 != nullptr || t1 != nullptr;
    const bool split = nf > 0 && nt > nf;
#define LAUNCH(kern, grid, block, e0, e1, ...)                                                                 \
    do {                                                                                                       \
        if (timed)                                                                                             \
            hipExtLaunchKernelGGL(kern, grid, block, 0, s, e0, e1, 0, __VA_ARGS__);                            \
        else                                                                                                   \
            hipLaunchKernelGGL(kern, grid, block, 0, s, __VA_ARGS__);                                          \
    } while (0)
#define X(i, a, b, c, w)                                                                                       \
    if (v == i) {                                                                                              \
        if (nf > 0)                                                                                            \
            LAUNCH((k_bond<MODEL, DIM, a, b, c, w, true>), dim3(nf), dim3(64 * w), t0, split ? nullptr : t1,     \
                   dd, tm, k, mode);                                                                           \
        if (nt > nf)                                                                                           \
            LAUNCH((k_bond<MODEL, DIM, a, b, c, w, false>), dim3(nt - nf), dim3(64 * w), split ? nullptr : t0,   \
                   t1, dd, tm + nf, k, mode);                                                                  \
        return hipGetLastError();                                                                              \
    }
    if constexpr (MODEL < XY && DIM == 2) { SW_VARIANTS_ISING2 }
    if constexpr (MODEL < XY && DIM == 3) { SW_VARIANTS_ISING3 }
    if constexpr (MODEL >= XY && DIM == 2) { SW_VARIANTS_XY2 }
    if constexpr (MODEL >= XY && DIM == 3) { SW_VARIANTS_XY3 }
#undef X
#undef LAUNCH
    return hipErrorInvalidValue;
}

template <int MODEL, int DIM>
static hipError_t flip_dispatch(int v, const InstDesc *dd, const int2 *tm, int nt, uint32_t k, hipStream_t s)
{
#define X(i, a, b, c, w)                                                                             \
    if (v == i) {                                                                                    \
        hipLaunchKernelGGL((k_flip<MODEL, DIM, a, b, c, w>), dim3(nt), dim3(64 * w), 0, s, dd, tm, k); \
        return hipGetLastError();                                                                    \
    }
    if constexpr (MODEL < XY && DIM == 2) { SW_VARIANTS_ISING2 }
    if constexpr (MODEL < XY && DIM == 3) { SW_VARIANTS_ISING3 }
    if constexpr (MODEL >= XY && DIM == 2) { SW_VARIANTS_XY2 }
    if constexpr (MODEL >= XY && DIM == 3) { SW_VARIANTS_XY3 }
#undef X
    return hipErrorInvalidValue;
}

}  // namespace swmc
