// sw_kernels.hip -- gfx950 kernels of the Swendsen-Wang sweep.
//
// One sweep (Sec. 2 of the paper: (1) active bonds, (2) cluster labelling,
// (3) random state per cluster) is three launches per (model, dim) group:
//
//   k_bond   one workgroup per lattice tile.  Stages the tile and its +1 halo
//            in LDS, draws the bond words (Philox4x32-10, one block per
//            4 aligned sites and direction), forms the bonds, measures the
//            incoming configuration, then labels the tile's clusters with a
//            union-find in LDS (label equivalence resolved by atomicMin on
//            roots, fixed point = minimum index).  Local roots receive their
//            cluster decision; labels and the tile's two faces per direction
//            go to HBM.
//   k_merge  global label equivalence across tiles: for every active bond
//            that crosses a tile face, link the larger root under the smaller
//            with device-scope atomicMin (Hawick's atomicMin on R[label],
//            retried until linked, so one pass reaches the fixed point).
//            An extra grid slice reduces the per-tile measurement partials.
//   k_flip   every site follows its label chain to the root and takes the
//            root's decision (Ising +-1, Potts state, XY mirror).
//
// Kernels read a per-lattice descriptor and a tile map, so one launch covers
// any number of lattices of one (model, dim) group (the batched form).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sw_internal.h"

namespace swmc {

#define TWO_PI_D 6.283185307179586476925286766559
#define PI_D 3.141592653589793238462643383279

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64-bit products with the Weyl key schedule.  The key is uniform per
// launch, so it lives in scalar registers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Component `lane` (0..3) of v with mask arithmetic (a plain ternary chain is
// lowered to an indexed private-memory load).
__device__ __forceinline__ uint32_t lane_of(const uint4 &v, uint32_t lane)
{
    const uint32_t m1 = 0u - (lane & 1u), m2 = 0u - ((lane >> 1) & 1u);
    const uint32_t lo = v.x ^ ((v.x ^ v.y) & m1);
    const uint32_t hi = v.z ^ ((v.z ^ v.w) & m1);
    return lo ^ ((lo ^ hi) & m2);
}

__device__ __forceinline__ uint32_t comp(const uint4 &v, int c)
{
    return c == 0 ? v.x : (c == 1 ? v.y : (c == 2 ? v.z : v.w));
}

// The four words of sites gi0 .. gi0+3 from the Philox blocks gi0/4 (a) and
// gi0/4 + 1 (b).  Aligned quads take the components in place.
__device__ __forceinline__ void quad_words(uint32_t gi0, const uint4 &a, const uint4 &b, uint32_t w[4])
{
    const uint32_t off = gi0 & 3u;
    if (off == 0) {
        w[0] = a.x;
        w[1] = a.y;
        w[2] = a.z;
        w[3] = a.w;
    } else {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const uint32_t p = off + (uint32_t)m;
            w[m] = (p < 4u) ? lane_of(a, p) : lane_of(b, p - 4u);
        }
    }
}

// Direction of the XY embedding at sweep n: a uniform angle from 53 bits of
// the GLOBAL stream (words 0 and 1).
__device__ __forceinline__ double xy_phi(const InstDesc &d, uint32_t n)
{
    const uint4 w = philox(make_uint4(0u, n, (uint32_t)TAG_GLOBAL, d.rep), d.key0, d.key1);
    const double u = ((double)(w.x >> 5) * 67108864.0 + (double)(w.y >> 6)) * 0x1p-53;
    return TWO_PI_D * u;
}

// Mirror of an XY spin in the line normal to phi: theta -> pi + 2 phi - theta,
// wrapped into [0, 2pi) in double, then rounded to float.
__device__ __forceinline__ float xy_reflect(float th, double phi)
{
    double v = (PI_D + 2.0 * phi) - (double)th;
    if (v >= TWO_PI_D) v -= TWO_PI_D;
    if (v >= TWO_PI_D) v -= TWO_PI_D;
    if (v < 0.0) v += TWO_PI_D;
    float f = (float)v;
    if (f >= (float)TWO_PI_D) f = 0.0f;
    return f;
}

template <int MODEL> struct StateOf;
template <> struct StateOf<ISING> { typedef int8_t type; };
template <> struct StateOf<POTTS> { typedef uint8_t type; };
template <> struct StateOf<XY> { typedef float type; };

__device__ __forceinline__ int wave_sum_i(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---- union-find in LDS (tile-local indices) --------------------------------
// Root of a with path halving: a non-root's parent may be replaced by any
// ancestor (every pointer goes to a smaller index of the same cluster), so
// the plain store is safe against concurrent unions.
__device__ __forceinline__ int lds_find(volatile int *par, int a)
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

__device__ __forceinline__ void lds_union(int *par, int a, int b)
{
    volatile int *vp = par;
    while (true) {
        a = lds_find(vp, a);
        b = lds_find(vp, b);
        if (a == b) return;
        if (a < b) {
            const int t = a;
            a = b;
            b = t;
        }
        const int old = atomicMin(&par[a], b);
        if (old == a) return;  // a was still a root: now linked under b
        a = old;               // a was linked meanwhile: merge its parent instead
    }
}

// ---- union-find on the global label words -----------------------------------
__device__ __forceinline__ uint32_t glabel_load(uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void glabel_store(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of a on the global label words, with path halving (see lds_find).
__device__ __forceinline__ uint32_t gfind(uint32_t *lab, uint32_t a)
{
    while (true) {
        const uint32_t p = glabel_load(lab + a);
        if (p & ROOT_FLAG) return a;
        const uint32_t g = glabel_load(lab + p);
        if (g & ROOT_FLAG) return p;
        glabel_store(lab + a, g);
        a = g;
    }
}

__device__ __forceinline__ void gunion(uint32_t *lab, uint32_t a, uint32_t b)
{
    while (true) {
        a = gfind(lab, a);
        b = gfind(lab, b);
        if (a == b) return;
        if (a < b) {
            const uint32_t t = a;
            a = b;
            b = t;
        }
        // roots hold ROOT_FLAG|decision > any index, so atomicMin links a root
        const uint32_t old = atomicMin(lab + a, b);
        if (old & ROOT_FLAG) return;
        a = old;
    }
}

// ---------------------------------------------------------------------------
// Hot start: word i of the INIT stream (sweep 0) gives the state of site i.
// One thread per aligned block of four sites.
// ---------------------------------------------------------------------------
template <int MODEL>
__global__ void __launch_bounds__(256) k_init(const InstDesc *__restrict__ descs, int inst)
{
    const InstDesc &d = descs[inst];
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b * 4 >= d.N) return;
    const uint4 w = philox(make_uint4((uint32_t)b, 0u, (uint32_t)TAG_INIT, d.rep), d.key0, d.key1);
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
    for (int m = 0; m < 4; ++m) {
        const int64_t i = b * 4 + m;
        if (i >= d.N) break;
        if (MODEL == ISING) {
            ((int8_t *)d.state)[i] = (ws[m] >> 31) ? (int8_t)-1 : (int8_t)1;
        } else if (MODEL == POTTS) {
            ((uint8_t *)d.state)[i] = (uint8_t)(((uint64_t)ws[m] * (uint64_t)d.q) >> 32);
        } else {
            const double t = ((double)ws[m] * 0x1p-32) * TWO_PI_D;
            float f = (float)t;
            if (f >= (float)TWO_PI_D) f = 0.0f;
            ((float *)d.state)[i] = f;
        }
    }
}

// ---------------------------------------------------------------------------
// Helpers of the bond kernel.
// ---------------------------------------------------------------------------
#define GLOBAL __attribute__((address_space(1)))
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Tile handled by this workgroup.  Workgroups are dealt to the 8 XCDs in
// turn, so slot b's neighbour b+1 runs on another XCD; this ordering keeps
// consecutive tiles (whose halos overlap) on one XCD and its L2.
__device__ __forceinline__ int tile_slot()
{
    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    if (nb & 7) return b;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

// Bytes of t that are zero -> bit 7 of that byte set (exact per byte).
__device__ __forceinline__ uint32_t zero_bytes(uint32_t t)
{
    return ~(((t & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | t) & 0x80808080u;
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

// Primaries (16 bits) of the bonds of sites gi0 .. gi0+3: x and y come from
// word g of BOND (high and low half), z from word g/2 of BOND_Z (high half for
// even g, low half for odd g).
template <int DIM>
__device__ __forceinline__ void quad_primaries(const InstDesc &d, uint32_t n, uint32_t gi0, int nv,
                                               uint32_t px[4], uint32_t py[4], uint32_t pz[4])
{
    const uint32_t b0 = gi0 >> 2;
    const uint4 a = philox(make_uint4(b0, n, (uint32_t)TAG_BOND, d.rep), d.key0, d.key1);
    uint32_t w[4];
    if ((gi0 & 3u) == 0) {
        w[0] = a.x;
        w[1] = a.y;
        w[2] = a.z;
        w[3] = a.w;
    } else {
        uint4 b = a;
        if ((gi0 & 3u) + (uint32_t)nv > 4u)
            b = philox(make_uint4(b0 + 1u, n, (uint32_t)TAG_BOND, d.rep), d.key0, d.key1);
        quad_words(gi0, a, b, w);
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        px[m] = w[m] >> 16;
        py[m] = w[m] & 0xffffu;
    }
    if (DIM == 3) {
        // z words g/2 for g = gi0 .. gi0+3 lie in blocks gi0/8 and possibly gi0/8 + 1
        const uint32_t zb0 = gi0 >> 3;
        const uint4 za = philox(make_uint4(zb0, n, (uint32_t)TAG_BOND_Z, d.rep), d.key0, d.key1);
        uint4 zb = za;
        if (((gi0 + (uint32_t)nv - 1u) >> 3) != zb0)
            zb = philox(make_uint4(zb0 + 1u, n, (uint32_t)TAG_BOND_Z, d.rep), d.key0, d.key1);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const uint32_t g = gi0 + (uint32_t)m;
            const uint32_t idx = (g >> 1) - (zb0 << 2);  // 0 .. 5
            const uint32_t word = (idx < 4u) ? lane_of(za, idx) : lane_of(zb, idx - 4u);
            pz[m] = (g & 1u) ? (word & 0xffffu) : (word >> 16);
        }
    } else {
#pragma unroll
        for (int m = 0; m < 4; ++m) pz[m] = 0;
    }
}

// ---------------------------------------------------------------------------
// Bond generation + tile-local labelling + measurement.
// mode 0: full sweep step; mode 1: measurement of the configuration only.
// ---------------------------------------------------------------------------
template <int MODEL, int DIM, int TX, int TY, int TZ>
__global__ void __launch_bounds__(256) k_bond(const InstDesc *__restrict__ descs,
                                              const int2 *__restrict__ tmap, uint32_t k, int mode)
{
    typedef typename StateOf<MODEL>::type S;
    constexpr int T = TX * TY * TZ;
    constexpr int SX = TX + 4, SY = TY + 1, SZ = (DIM == 3) ? TZ + 1 : 1;  // rows padded to 4 bytes
    constexpr int NH = SX * SY * SZ;
    constexpr int QX = TX / 4;
    constexpr int NQ = T / 4;
    constexpr int QPT = NQ / 256;
    constexpr int ROWS = TY * TZ;
    constexpr int R = ROWS / 4;  // rows scanned by each wavefront
    constexpr bool IS_XY = (MODEL == XY);
    constexpr int QCAP = 256;    // per-wave queue of deferred equivalences
    static_assert(TX == 64, "a tile row is one wavefront (lane = column) in the labelling scan");
    static_assert(T <= 32768, "provisional labels are 16-bit");
    static_assert(ROWS % 4 == 0, "whole rows per wavefront");
    static_assert(NQ % 256 == 0, "whole quads per thread");
    static_assert(DIM == 3 || TZ == 1, "2D tiles have TZ = 1");

    // LDS: the staged states (or XY projections) are dead once the bonds are
    // known, so the labelling arrays reuse that space.
    constexpr int STAGE_BYTES = IS_XY ? NH * 16 : ((NH + 15) / 16) * 16;
    constexpr int LABEL_BYTES = T * 4 + T * 2;
    constexpr int REGION = STAGE_BYTES > LABEL_BYTES ? STAGE_BYTES : LABEL_BYTES;
    __shared__ __align__(16) uint8_t s_mem[REGION];
    __shared__ __align__(16) uint8_t s_bond[T];
    __shared__ uint32_t s_cw[ROWS * 8];  // cluster decision words, 8 per tile row
    __shared__ uint32_t s_q[4][QCAP];
    __shared__ int s_hist[MODEL == POTTS ? 256 : 1];
    __shared__ double s_red[4][3];
    __shared__ double s_phi;
    S *s_st = (S *)s_mem;
    double2 *s_sig = (double2 *)s_mem;
    int *s_par = (int *)s_mem;
    int16_t *s_plab = (int16_t *)(s_mem + T * 4);

    const int2 tm = tmap[tile_slot()];
    if (tm.x < 0) return;
    const InstDesc d = descs[tm.x];
    if (k >= d.count) return;
    const uint32_t n = d.sweep0 + k;
    const int L = d.L;
    const int t = tm.y;
    const int tx = t % d.tiles[0];
    const int ty = (t / d.tiles[0]) % d.tiles[1];
    const int tz = (DIM == 3) ? t / (d.tiles[0] * d.tiles[1]) : 0;
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
    const int ex = min(TX, L - x0), ey = min(TY, L - y0), ez = (DIM == 3) ? min(TZ, L - z0) : 1;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const bool full = (mode == 0);
    const bool meas = (mode == 1) || d.measure;
    const bool bits_dec = (MODEL != POTTS) || d.q == 2;  // one decision bit per cluster
    GLOBAL uint8_t *g_bond = (GLOBAL uint8_t *)d.bond;
    GLOBAL uint32_t *g_label = (GLOBAL uint32_t *)d.label;

    auto gsite = [&](int lx, int ly, int lz) -> uint32_t {
        return (uint32_t)(x0 + lx) + (uint32_t)L * ((uint32_t)(y0 + ly) + (uint32_t)L * (uint32_t)(z0 + lz));
    };

    if (IS_XY && tid == 0) s_phi = xy_phi(d, n);
    if (MODEL == POTTS && meas)
        for (int c = tid; c < d.q; c += 256) s_hist[c] = 0;
    if (IS_XY) __syncthreads();
    const double phi = IS_XY ? s_phi : 0.0;

    // ---- stage states (+1 halo in every + direction) ------------------------
    // Interior: one 4-site load per quad, all issued before any LDS store.
    {
        uint32_t raw[QPT];
        float4 rawf[QPT];
#pragma unroll
        for (int j = 0; j < QPT; ++j) {
            const int qid = tid + 256 * j;
            const int qx = qid % QX, row = qid / QX;
            const int ly = row % TY, lz = row / TY;
            const int lx0 = qx * 4;
            raw[j] = 0;
            rawf[j] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (ly >= ey || lz >= ez || lx0 >= ex) continue;
            const int nv = min(4, ex - lx0);
            const uint32_t gi0 = gsite(lx0, ly, lz);
            if ((gi0 & 3u) == 0 && nv == 4) {
                if (IS_XY) {
                    const f32x4 v = *(const GLOBAL f32x4 *)((const GLOBAL float *)d.state + gi0);
                    rawf[j] = make_float4(v.x, v.y, v.z, v.w);
                }
                else raw[j] = *(const GLOBAL uint32_t *)((const GLOBAL uint8_t *)d.state + gi0);
            } else if (IS_XY) {
                const GLOBAL float *st = (const GLOBAL float *)d.state + gi0;
                rawf[j].x = st[0];
                if (nv > 1) rawf[j].y = st[1];
                if (nv > 2) rawf[j].z = st[2];
                if (nv > 3) rawf[j].w = st[3];
            } else {
                const GLOBAL uint8_t *st = (const GLOBAL uint8_t *)d.state + gi0;
                for (int m = 0; m < nv; ++m) raw[j] |= (uint32_t)st[m] << (8 * m);
            }
        }
#pragma unroll
        for (int j = 0; j < QPT; ++j) {
            const int qid = tid + 256 * j;
            const int qx = qid % QX, row = qid / QX;
            const int ly = row % TY, lz = row / TY;
            const int lx0 = qx * 4;
            if (ly >= ey || lz >= ez || lx0 >= ex) continue;
            const int nv = min(4, ex - lx0);
            const int h = lx0 + SX * (ly + SY * lz);
            // a partial quad stores only its own sites: the cell after it may be
            // the +x halo, written by another thread
            if (IS_XY) {
                const float a[4] = {rawf[j].x, rawf[j].y, rawf[j].z, rawf[j].w};
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    if (m >= nv) continue;
                    double sv, cv;
                    sincos((double)a[m] - phi, &sv, &cv);
                    s_sig[h + m] = make_double2(cv, sv);
                }
            } else if (nv == 4) {
                *(uint32_t *)&s_st[h] = raw[j];
            } else {
                for (int m = 0; m < nv; ++m) s_st[h + m] = (S)(raw[j] >> (8 * m));
            }
        }
    }
    // Halo: the +x column, the +y row and (3D) the +z layer of the tile.
    {
        constexpr int HX = TY * TZ, HY = TX * TZ, HZ = (DIM == 3) ? TX * TY : 0;
        constexpr int NHALO = HX + HY + HZ;
        constexpr int HPT = (NHALO + 255) / 256;
        S hv[HPT];
        int hh[HPT];
#pragma unroll
        for (int u = 0; u < HPT; ++u) {
            const int c = tid + 256 * u;
            hh[u] = -1;
            int hx = 0, hy = 0, hz = 0;
            if (c < HX) {
                hx = ex;
                hy = c % TY;
                hz = c / TY;
                if (hy >= ey || hz >= ez) continue;
            } else if (c < HX + HY) {
                hx = (c - HX) % TX;
                hy = ey;
                hz = (c - HX) / TX;
                if (hx >= ex || hz >= ez) continue;
            } else if (c < NHALO) {
                hx = (c - HX - HY) % TX;
                hy = (c - HX - HY) / TX;
                hz = ez;
                if (hx >= ex || hy >= ey) continue;
            } else {
                continue;
            }
            int gx = x0 + hx, gy = y0 + hy, gz = z0 + hz;
            if (gx >= L) gx -= L;
            if (gy >= L) gy -= L;
            if (DIM == 3 && gz >= L) gz -= L;
            const uint32_t gi = (uint32_t)gx + (uint32_t)L * ((uint32_t)gy + (uint32_t)L * (uint32_t)gz);
            hv[u] = ((const GLOBAL S *)d.state)[gi];
            hh[u] = hx + SX * (hy + SY * hz);
        }
#pragma unroll
        for (int u = 0; u < HPT; ++u) {
            if (hh[u] < 0) continue;
            if (IS_XY) {
                double sv, cv;
                sincos((double)hv[u] - phi, &sv, &cv);
                s_sig[hh[u]] = make_double2(cv, sv);
            } else {
                s_st[hh[u]] = hv[u];
            }
        }
    }
    // Cluster decision words of every tile row (one bit per possible root):
    // row r needs words g/32 for its sites g, which lie in Philox blocks
    // g_r/128 and g_r/128 + 1 of the cluster stream.
    if (full && bits_dec && tid < 2 * ROWS) {
        const int r = tid >> 1, half = tid & 1;
        const int ly = r % TY, lz = r / TY;
        if (ly < ey && lz < ez) {
            const uint32_t gr = gsite(0, ly, lz);
            const uint4 w = philox(make_uint4((gr >> 7) + (uint32_t)half, n, (uint32_t)TAG_CLUSTER, d.rep),
                                   d.key0, d.key1);
            *(uint4 *)&s_cw[8 * r + 4 * half] = w;
        }
    }
    __syncthreads();

    // ---- (1) bonds and measurement -------------------------------------------
    int cnt_al = 0, cnt_m = 0;
    double e_acc = 0.0, sx_acc = 0.0, sy_acc = 0.0;
    uint32_t qb[QPT];
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
        qb[j] = 0;
        const int qid = tid + 256 * j;
        const int qx = qid % QX, row = qid / QX;
        const int ly = row % TY, lz = row / TY;
        const int lx0 = qx * 4;
        if (ly >= ey || lz >= ez || lx0 >= ex) continue;
        const int nv = min(4, ex - lx0);
        const uint32_t vmask = (nv == 4) ? 0xffffffffu : ((1u << (8 * nv)) - 1u);
        const uint32_t gi0 = gsite(lx0, ly, lz);
        const int h = lx0 + SX * (ly + SY * lz);
        uint32_t px[4], py[4], pz[4];
        if (full) quad_primaries<DIM>(d, n, gi0, nv, px, py, pz);
        uint32_t bq = 0;
        if constexpr (!IS_XY) {
            const uint32_t s = *(const uint32_t *)&s_st[h];
            const uint32_t sn = (uint8_t)s_st[h + 4];
            const uint32_t sxn = (s >> 8) | (sn << 24);
            const uint32_t syn = *(const uint32_t *)&s_st[h + SX];
            const uint32_t eqx = zero_bytes(s ^ sxn) & vmask;
            const uint32_t eqy = zero_bytes(s ^ syn) & vmask;
            uint32_t eqz = 0;
            if (DIM == 3) eqz = zero_bytes(s ^ *(const uint32_t *)&s_st[h + SX * SY]) & vmask;
            if (meas) {
                cnt_al += __popc(eqx) + __popc(eqy) + __popc(eqz);
                if (MODEL == ISING) cnt_m += nv - 2 * __popc(s & 0x80808080u & vmask);
                else {
#pragma unroll
                    for (int m = 0; m < 4; ++m)
                        if (m < nv) atomicAdd(&s_hist[(s >> (8 * m)) & 0xffu], 1);
                }
            }
            if (full) {
                const uint32_t th = d.thr_hi;
                uint32_t tie = 0;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const uint32_t ax = (eqx >> (8 * m + 7)) & 1u, ay = (eqy >> (8 * m + 7)) & 1u;
                    const uint32_t az = (eqz >> (8 * m + 7)) & 1u;
                    uint32_t bm = (ax & (px[m] < th)) | ((ay & (py[m] < th)) << 1);
                    if (DIM == 3) bm |= (az & (pz[m] < th)) << 2;
                    bq |= bm << (8 * m);
                    tie |= (ax & (px[m] == th)) | (ay & (py[m] == th)) | (az & (pz[m] == th));
                }
                if (tie) {  // rare: the primary equals the threshold's high half
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const uint32_t g = gi0 + (uint32_t)m;
                        const uint32_t p[3] = {px[m], py[m], pz[m]};
                        const uint32_t eq[3] = {eqx, eqy, eqz};
#pragma unroll
                        for (int mu = 0; mu < DIM; ++mu)
                            if (((eq[mu] >> (8 * m + 7)) & 1u) && p[mu] == th &&
                                bond_secondary(d.key0, d.key1, d.rep, n, DIM, g, mu) < d.thr_lo)
                                bq |= 1u << (8 * m + mu);
                    }
                }
            }
        } else {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                if (m >= nv) continue;
                const int hm = h + m;
                const double2 a = s_sig[hm];
                if (meas) {
                    sx_acc += a.x;
                    sy_acc += a.y;
                }
                const uint32_t p[3] = {px[m], py[m], pz[m]};
#pragma unroll
                for (int mu = 0; mu < DIM; ++mu) {
                    const int hn = hm + (mu == 0 ? 1 : (mu == 1 ? SX : SX * SY));
                    const double2 c = s_sig[hn];
                    if (meas) e_acc -= a.x * c.x + a.y * c.y;
                    if (full) {
                        // u = (P 2^16 + S) 2^-32 against p = -expm1(-(2 beta s_i) s_j)
                        const double x = (d.two_beta * a.x) * c.x;
                        const double pr = -expm1(-x);
                        const double lo = (double)p[mu] * 0x1p-16, hi = (double)(p[mu] + 1u) * 0x1p-16;
                        bool on;
                        if (hi <= pr) on = true;
                        else if (lo >= pr) on = false;
                        else {
                            const uint32_t sec = bond_secondary(d.key0, d.key1, d.rep, n, DIM, gi0 + (uint32_t)m, mu);
                            on = (double)((p[mu] << 16) | sec) * 0x1p-32 < pr;
                        }
                        if (on) bq |= 1u << (8 * m + mu);
                    }
                }
            }
        }
        qb[j] = bq;
        if (full) {
            *(uint32_t *)&s_bond[lx0 + TX * (ly + TY * lz)] = bq;
            if (d.store_bonds) {
                if ((gi0 & 3u) == 0 && nv == 4) {
                    *(GLOBAL uint32_t *)(g_bond + gi0) = bq;
                } else {
                    for (int m = 0; m < nv; ++m) g_bond[gi0 + m] = (uint8_t)(bq >> (8 * m));
                }
            }
        }
    }

    // ---- measurement partials of this tile -----------------------------------
    if (meas) {
        GLOBAL int64_t *part = (GLOBAL int64_t *)d.part + (int64_t)t * d.nslots;
        if (IS_XY) {
            const double a = wave_sum_d(e_acc), b = wave_sum_d(sx_acc), c = wave_sum_d(sy_acc);
            if (lane == 0) {
                s_red[wv][0] = a;
                s_red[wv][1] = b;
                s_red[wv][2] = c;
            }
        } else {
            const int a = wave_sum_i(cnt_al), b = wave_sum_i(cnt_m);
            if (lane == 0) {
                s_red[wv][0] = (double)a;
                s_red[wv][1] = (double)b;
            }
        }
        __syncthreads();
        if (tid == 0) {
            if (IS_XY) {
                for (int c = 0; c < 3; ++c) {
                    const double v = ((s_red[0][c] + s_red[1][c]) + s_red[2][c]) + s_red[3][c];
                    part[c] = __double_as_longlong(v);
                }
            } else {
                part[0] = (int64_t)(s_red[0][0] + s_red[1][0] + s_red[2][0] + s_red[3][0]);
                if (MODEL == ISING)
                    part[1] = (int64_t)(s_red[0][1] + s_red[1][1] + s_red[2][1] + s_red[3][1]);
            }
        }
        if (MODEL == POTTS)
            for (int c = tid; c < d.q; c += 256) part[1 + c] = s_hist[c];
    }
    if (!full) return;
    __syncthreads();  // s_bond complete; staged states no longer needed
    for (int l = tid; l < T; l += 256) s_par[l] = l;
    __syncthreads();

    // ---- (2) local labelling: a row-by-row scan per wavefront ------------------
    // Lane c of a wavefront owns column c of the tile; each of the four waves
    // scans its own block of R rows (row r = y + TY z) in order.  In a row the
    // x bonds form runs (ballot + bit tricks); a run takes the label of its
    // leftmost site bonded to the row above (or, in 3D, the plane behind) and
    // otherwise its own start index.  A bonded neighbour whose label differs
    // from its run's label is an equivalence, queued and resolved afterwards
    // in the union-find table s_par (larger root under smaller), together
    // with the bonds across wave blocks and the periodic bonds inside a tile
    // that spans the lattice.  The root of site l is then s_par[s_plab[l]].
    constexpr int NONE = 0x7fffffff;
    int qn = 0;  // entries in this wave's queue (uniform)
    auto flush = [&]() {
        for (int e = lane; e < qn; e += 64) {
            const uint32_t pr = s_q[wv][e];
            lds_union(s_par, (int)(pr >> 16), (int)(pr & 0xffffu));
        }
        qn = 0;
    };
    auto push = [&](bool want, int a, int b) {
        if (qn > QCAP - 64) flush();
        const unsigned long long m = __ballot(want);
        if (want) {
            const int pos = qn + __popcll(m & ((1ull << lane) - 1ull));
            s_q[wv][pos] = ((uint32_t)a << 16) | (uint32_t)b;
        }
        qn += __popcll(m);
    };
    {
        const int c = lane;
        const int r0 = wv * R;
        const unsigned long long upto = (c == 63) ? ~0ull : ((2ull << c) - 1ull);
        const unsigned long long from = ~((1ull << c) - 1ull);
        int prevlab = NONE;
        uint32_t prevb = 0;
        for (int r = r0; r < r0 + R; ++r) {
            const int y = r % TY, z = r / TY;
            if (y >= ey || z >= ez) {  // ragged tile: rows past the lattice edge
                prevlab = NONE;
                prevb = 0;
                continue;
            }
            const int l = c + TX * r;
            const bool vc = c < ex;
            const uint32_t b = vc ? s_bond[l] : 0u;
            const unsigned long long xb = __ballot(vc && (b & 1u) && c + 1 < ex);
            const unsigned long long brk = ~(xb << 1);  // bit c: a run starts at c
            const int rs = 63 - __clzll((long long)(brk & upto));
            const int re = __ffsll((long long)(~xb & from)) - 1;
            int ca = NONE, cb = NONE;
            if (y > 0 && r - 1 >= r0 && (prevb & 2u)) ca = prevlab;
            if (DIM == 3 && z > 0 && r - TY >= r0 && (s_bond[l - TX * TY] & 4u)) cb = s_plab[l - TX * TY];
            const int cand = vc ? min(ca, cb) : NONE;
            const unsigned long long conn = __ballot(cand != NONE);
            const unsigned long long mr = conn >> rs;
            const int f = mr ? rs + __ffsll((long long)mr) - 1 : 64;
            const int fl = __shfl(cand, f & 63, 64);
            const int lab = (f <= re) ? fl : rs + TX * r;
            if (vc) s_plab[l] = (int16_t)lab;
            push(vc && ca != NONE && ca != lab, ca, lab);
            if (DIM == 3) push(vc && cb != NONE && cb != lab, cb, lab);
            prevlab = lab;
            prevb = b;
        }
    }
    __syncthreads();  // all provisional labels written
    // bonds between wave blocks and periodic bonds inside a tile spanning L
    {
        const int c = lane;
        const int r0 = wv * R;
        const bool vc = c < ex;
        for (int r = r0; r < r0 + R; ++r) {
            const int y = r % TY, z = r / TY;
            if (y >= ey || z >= ez) continue;
            const int l = c + TX * r;
            const uint32_t b = vc ? s_bond[l] : 0u;
            const int own = vc ? s_plab[l] : 0;
            // the row above lies in the previous wave's block
            const bool wy = vc && y > 0 && r - 1 < r0 && (s_bond[l - TX] & 2u);
            push(wy, wy ? s_plab[l - TX] : 0, own);
            // the plane behind lies in an earlier wave's block
            if (DIM == 3) {
                const bool wz = vc && z > 0 && r - TY < r0 && (s_bond[l - TX * TY] & 4u);
                push(wz, wz ? s_plab[l - TX * TY] : 0, own);
            }
            const bool px_ = vc && (b & 1u) && c + 1 == ex && d.tiles[0] == 1;
            push(px_, px_ ? s_plab[l - c] : 0, own);
            const bool py_ = vc && (b & 2u) && y + 1 == ey && d.tiles[1] == 1;
            push(py_, py_ ? s_plab[l - TX * y] : 0, own);
            if (DIM == 3) {
                const bool pz_ = vc && (b & 4u) && z + 1 == ez && d.tiles[2] == 1;
                push(pz_, pz_ ? s_plab[l - TX * TY * z] : 0, own);
            }
        }
        flush();
    }
    __syncthreads();
    for (int l = tid; l < T; l += 256) s_par[l] = lds_find(s_par, l);
    __syncthreads();
    // root (tile-local index) of site l
    auto root_of = [&](int l) -> int { return s_par[s_plab[l]]; };
    auto gidx = [&](int r) -> uint32_t {
        const int rx = r % TX, ry = (r / TX) % TY, rz = r / (TX * TY);
        return gsite(rx, ry, rz);
    };

    // ---- local roots draw the cluster decision; labels to HBM -----------------
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
        const int qid = tid + 256 * j;
        const int qx = qid % QX, row = qid / QX;
        const int ly = row % TY, lz = row / TY;
        const int lx0 = qx * 4;
        if (ly >= ey || lz >= ez || lx0 >= ex) continue;
        const int nv = min(4, ex - lx0);
        const uint32_t gi0 = gsite(lx0, ly, lz);
        const int l0 = lx0 + TX * (ly + TY * lz);
        const uint2 pl = *(const uint2 *)&s_plab[l0];
        const int p4[4] = {(int)(int16_t)(pl.x & 0xffffu), (int)(int16_t)(pl.x >> 16),
                           (int)(int16_t)(pl.y & 0xffffu), (int)(int16_t)(pl.y >> 16)};
        int rq[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) rq[m] = (m < nv) ? s_par[p4[m]] : -1;
        bool anyroot = false;
#pragma unroll
        for (int m = 0; m < 4; ++m) anyroot |= (rq[m] == l0 + m);
        uint32_t dec[4] = {0u, 0u, 0u, 0u};
        if (anyroot) {
            if (bits_dec) {
                const uint32_t gr = gsite(0, ly, lz);
                const uint32_t base = (gr >> 7) << 2;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const uint32_t g = gi0 + (uint32_t)m;
                    dec[m] = (s_cw[8 * row + (int)((g >> 5) - base)] >> (g & 31u)) & 1u;
                }
            } else {
                const uint4 c1 = philox(make_uint4(gi0 >> 2, n, (uint32_t)TAG_CLUSTER, d.rep), d.key0, d.key1);
                uint4 c2 = c1;
                if ((gi0 & 3u) + (uint32_t)nv > 4u)
                    c2 = philox(make_uint4((gi0 >> 2) + 1u, n, (uint32_t)TAG_CLUSTER, d.rep), d.key0, d.key1);
                uint32_t cw[4];
                quad_words(gi0, c1, c2, cw);
#pragma unroll
                for (int m = 0; m < 4; ++m) dec[m] = (uint32_t)(((uint64_t)cw[m] * (uint64_t)d.q) >> 32);
            }
        }
        uint32_t lab[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            if (m >= nv) continue;
            lab[m] = (rq[m] == l0 + m) ? (ROOT_FLAG | dec[m]) : gidx(rq[m]);
        }
        if ((gi0 & 3u) == 0 && nv == 4) {
            *(GLOBAL u32x4 *)(g_label + gi0) = (u32x4){lab[0], lab[1], lab[2], lab[3]};
        } else {
#pragma unroll
            for (int m = 0; m < 4; ++m)
                if (m < nv) g_label[gi0 + m] = lab[m];
        }
    }

    // ---- faces for the global merge --------------------------------------------
#pragma unroll
    for (int mu = 0; mu < DIM; ++mu) {
        if (d.tiles[mu] == 1) continue;
        const int F = d.face_len[mu];
        GLOBAL int32_t *fo = (GLOBAL int32_t *)d.face + d.face_off[mu] + (int64_t)t * 2 * F;
        GLOBAL int32_t *fi = fo + F;
        const int emu = (mu == 0) ? ex : (mu == 1 ? ey : ez);
        for (int kk = tid; kk < F; kk += 256) {
            int a, b;  // transverse coordinates
            bool valid;
            int lo, li;
            if (mu == 0) {
                a = kk % TY;
                b = kk / TY;
                valid = a < ey && b < ez;
                lo = (emu - 1) + TX * (a + TY * b);
                li = 0 + TX * (a + TY * b);
            } else if (mu == 1) {
                a = kk % TX;
                b = kk / TX;
                valid = a < ex && b < ez;
                lo = a + TX * ((emu - 1) + TY * b);
                li = a + TX * (0 + TY * b);
            } else {
                a = kk % TX;
                b = kk / TX;
                valid = a < ex && b < ey;
                lo = a + TX * (b + TY * (emu - 1));
                li = a + TX * b;
            }
            if (!valid) {
                fo[kk] = -1;
                fi[kk] = -1;
                continue;
            }
            fo[kk] = ((s_bond[lo] >> mu) & 1u) ? (int32_t)gidx(root_of(lo)) : -1;
            fi[kk] = (int32_t)gidx(root_of(li));
        }
    }
}

// ---------------------------------------------------------------------------
// Global label equivalence across tile faces.  grid = (ceil(tiles * FMAX /
// 256), DIM): thread e of slice mu handles element e % FMAX of the +mu face of
// tile slot e / FMAX; for every active bond crossing the face it links the
// larger of the two tile roots under the smaller with device-scope atomicMin.
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void __launch_bounds__(256) k_merge(const InstDesc *__restrict__ descs,
                                               const int2 *__restrict__ tmap, int ntiles, int fmax,
                                               uint32_t k)
{
    const int mu = blockIdx.y;
    const int e = tile_slot() * 256 + (int)threadIdx.x;
    const int ts = e / fmax, kk = e - ts * fmax;
    if (ts >= ntiles) return;
    const int2 tm = tmap[ts];
    if (tm.x < 0) return;
    const InstDesc &d = descs[tm.x];
    if (k >= d.count || d.tiles[mu] == 1) return;
    const int F = d.face_len[mu];
    if (kk >= F) return;
    const int t = tm.y;
    const int32_t a = ((const GLOBAL int32_t *)d.face)[d.face_off[mu] + (int64_t)t * 2 * F + kk];
    if (a < 0) return;
    int c[3] = {t % d.tiles[0], (t / d.tiles[0]) % d.tiles[1], (DIM == 3) ? t / (d.tiles[0] * d.tiles[1]) : 0};
    c[mu] = (c[mu] + 1 == d.tiles[mu]) ? 0 : c[mu] + 1;
    const int nb = c[0] + d.tiles[0] * (c[1] + d.tiles[1] * c[2]);
    const int32_t b = ((const GLOBAL int32_t *)d.face)[d.face_off[mu] + (int64_t)nb * 2 * F + F + kk];
    gunion(d.label, (uint32_t)a, (uint32_t)b);
}

// ---------------------------------------------------------------------------
// Reduction of the per-tile measurement partials into one record row, in a
// fixed order (deterministic, also for the XY sums).  Workgroup t of a
// lattice reduces slots t, t + ntiles, ... (XY: workgroup 0 all three and
// rotates the projected sums back by phi).
// ---------------------------------------------------------------------------
template <int MODEL>
__device__ void reduce_partials(const InstDesc &d, int t, uint32_t n, int64_t row)
{
    __shared__ double s_red[4][3];
    __shared__ double s_phi;
    const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
    GLOBAL int64_t *rec = (GLOBAL int64_t *)d.rec + row * d.nslots;
    const GLOBAL int64_t *part = (const GLOBAL int64_t *)d.part;
    if (MODEL == XY) {
        if (t != 0) return;
        if (tid == 0) s_phi = xy_phi(d, n);
        double acc[3] = {0.0, 0.0, 0.0};
        for (int tt = tid; tt < d.ntiles; tt += 256)
            for (int c = 0; c < 3; ++c) acc[c] += __longlong_as_double(part[(int64_t)tt * 3 + c]);
        for (int c = 0; c < 3; ++c) {
            const double v = wave_sum_d(acc[c]);
            if (ln == 0) s_red[wv][c] = v;
        }
        __syncthreads();
        if (tid == 0) {
            double v[3];
            for (int c = 0; c < 3; ++c) v[c] = ((s_red[0][c] + s_red[1][c]) + s_red[2][c]) + s_red[3][c];
            double sp, cp;
            sincos(s_phi, &sp, &cp);
            // sum of (cos, sin)(theta - phi) rotated back by phi
            rec[0] = __double_as_longlong(v[0]);
            rec[1] = __double_as_longlong(cp * v[1] - sp * v[2]);
            rec[2] = __double_as_longlong(sp * v[1] + cp * v[2]);
        }
        __syncthreads();
        return;
    }
    for (int slot = t; slot < d.nslots; slot += d.ntiles) {
        long long acc = 0;
        for (int tt = tid; tt < d.ntiles; tt += 256) acc += part[(int64_t)tt * d.nslots + slot];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (ln == 0) s_red[wv][0] = __longlong_as_double(acc);
        __syncthreads();
        if (tid == 0) {
            rec[slot] = __double_as_longlong(s_red[0][0]) + __double_as_longlong(s_red[1][0]) +
                        __double_as_longlong(s_red[2][0]) + __double_as_longlong(s_red[3][0]);
        }
        __syncthreads();
    }
}

// Measurement of the current configuration alone: reduce into the scratch row.
template <int MODEL>
__global__ void __launch_bounds__(256) k_reduce(const InstDesc *__restrict__ descs, const int2 *__restrict__ tmap)
{
    const int2 tm = tmap[blockIdx.x];
    if (tm.x < 0) return;
    const InstDesc &d = descs[tm.x];
    if (tm.y >= d.nslots && !(MODEL == XY && tm.y == 0)) return;
    reduce_partials<MODEL>(d, tm.y, d.sweep0, d.rec_cap);
}

// ---------------------------------------------------------------------------
// (3) every site takes its cluster root's decision.
// ---------------------------------------------------------------------------
template <int MODEL, int DIM, int TX, int TY, int TZ>
__global__ void __launch_bounds__(256) k_flip(const InstDesc *__restrict__ descs,
                                              const int2 *__restrict__ tmap, uint32_t k)
{
    constexpr int T = TX * TY * TZ;
    constexpr int QX = TX / 4;
    constexpr int NQ = T / 4;
    constexpr int QPT = (NQ + 255) / 256;
    __shared__ double s_phi;
    const int2 tm = tmap[tile_slot()];
    if (tm.x < 0) return;
    const InstDesc &d = descs[tm.x];
    if (k >= d.count) return;
    const uint32_t n = d.sweep0 + k;
    const int L = d.L;
    const int t = tm.y;
    const int tx = t % d.tiles[0];
    const int ty = (t / d.tiles[0]) % d.tiles[1];
    const int tz = (DIM == 3) ? t / (d.tiles[0] * d.tiles[1]) : 0;
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
    const int ex = min(TX, L - x0), ey = min(TY, L - y0), ez = (DIM == 3) ? min(TZ, L - z0) : 1;
    const int tid = threadIdx.x;
    // the first workgroups of a lattice also reduce the sweep's measurement
    if (d.measure && d.rec_row0 >= 0 && d.rec_row0 + (int64_t)k < d.rec_cap &&
        (t < d.nslots || (MODEL == XY && t == 0)))
        reduce_partials<MODEL>(d, t, n, d.rec_row0 + (int64_t)k);
    if (MODEL == XY) {
        if (tid == 0) s_phi = xy_phi(d, n);
        __syncthreads();
    }
    const double phi = (MODEL == XY) ? s_phi : 0.0;
    uint32_t *lab = d.label;
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
        const int qid = tid + 256 * j;
        if (qid >= NQ) continue;
        const int qx = qid % QX, row = qid / QX;
        const int ly = row % TY, lz = row / TY;
        const int lx0 = qx * 4;
        if (ly >= ey || lz >= ez || lx0 >= ex) continue;
        const int nv = min(4, ex - lx0);
        const uint32_t gi0 = (uint32_t)(x0 + lx0) +
                             (uint32_t)L * ((uint32_t)(y0 + ly) + (uint32_t)L * (uint32_t)(z0 + lz));
        const bool vec = ((gi0 & 3u) == 0) && nv == 4;
        uint32_t v[4];
        if (vec) {
            const uint4 q4 = *(const uint4 *)(lab + gi0);
            v[0] = q4.x;
            v[1] = q4.y;
            v[2] = q4.z;
            v[3] = q4.w;
        } else {
            for (int m = 0; m < 4; ++m) v[m] = (m < nv) ? lab[gi0 + m] : ROOT_FLAG;
        }
        uint32_t dec[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            uint32_t x = v[m];
            if (!(x & ROOT_FLAG)) {
                // x is the tile-local root; follow the links the merge made and
                // point x straight at the final root for the sites after us
                const uint32_t r = x;
                uint32_t g = r;
                x = lab[r];
                if (!(x & ROOT_FLAG)) {
                    while (!(x & ROOT_FLAG)) {
                        g = x;
                        x = lab[g];
                    }
                    if (lab[r] != g) lab[r] = g;
                }
            }
            dec[m] = x & 0xffu;
        }
        if (MODEL == ISING || MODEL == POTTS) {
            uint32_t packed = 0;
            for (int m = 0; m < 4; ++m) {
                const uint32_t s = (MODEL == ISING) ? (dec[m] ? 0xffu : 0x01u) : dec[m];
                packed |= s << (8 * m);
            }
            if (vec) {
                *(uint32_t *)((uint8_t *)d.state + gi0) = packed;
            } else {
                for (int m = 0; m < nv; ++m) ((uint8_t *)d.state)[gi0 + m] = (uint8_t)(packed >> (8 * m));
            }
        } else {
            float *th = (float *)d.state;
            if (vec) {
                float4 a = *(const float4 *)(th + gi0);
                if (dec[0]) a.x = xy_reflect(a.x, phi);
                if (dec[1]) a.y = xy_reflect(a.y, phi);
                if (dec[2]) a.z = xy_reflect(a.z, phi);
                if (dec[3]) a.w = xy_reflect(a.w, phi);
                *(float4 *)(th + gi0) = a;
            } else {
                for (int m = 0; m < nv; ++m)
                    if (dec[m]) th[gi0 + m] = xy_reflect(th[gi0 + m], phi);
            }
        }
    }
}

// Minimum-index labels: follow every chain to its root.
__global__ void __launch_bounds__(256) k_canon(const InstDesc *__restrict__ descs, int inst,
                                               int32_t *__restrict__ out)
{
    const InstDesc &d = descs[inst];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= d.N) return;
    uint32_t r = (uint32_t)i;
    uint32_t x = d.label[r];
    while (!(x & ROOT_FLAG)) {
        r = x;
        x = d.label[r];
    }
    out[i] = (int32_t)r;
}

// Advance every lattice's schedule by one graph chunk.
__global__ void k_advance(InstDesc *descs, int ninst)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst) return;
    InstDesc &d = descs[i];
    const uint32_t used = min(d.chunk, d.remaining);
    d.sweep0 += used;
    if (d.rec_row0 >= 0 && d.measure) d.rec_row0 += used;
    d.remaining -= used;
    d.count = min(d.chunk, d.remaining);
}

// ---------------------------------------------------------------------------
// Variant table and launchers.
// ---------------------------------------------------------------------------
#define SW_VARIANTS_ISING2 X(0, 64, 64, 1) X(1, 64, 32, 1) X(2, 64, 128, 1)
#define SW_VARIANTS_ISING3 X(0, 64, 8, 8) X(1, 64, 4, 8) X(2, 64, 8, 16)
#define SW_VARIANTS_XY2 X(0, 64, 32, 1) X(1, 64, 16, 1) X(2, 64, 64, 1)
#define SW_VARIANTS_XY3 X(0, 64, 4, 8) X(1, 64, 8, 4) X(2, 64, 4, 4)

int num_tile_variants(int, int) { return 3; }

TileShape tile_shape(int model, int dim, int v)
{
#define X(i, a, b, c) \
    if (v == i) return TileShape{a, b, c};
    if (model != XY && dim == 2) { SW_VARIANTS_ISING2 }
    if (model != XY && dim == 3) { SW_VARIANTS_ISING3 }
    if (model == XY && dim == 2) { SW_VARIANTS_XY2 }
    if (model == XY && dim == 3) { SW_VARIANTS_XY3 }
#undef X
    return TileShape{0, 0, 0};
}

int slots_for(int model, int q) { return model == ISING ? 2 : (model == POTTS ? 1 + q : 3); }

hipError_t launch_init(const InstDesc *d_desc, int inst, const InstDesc &h, hipStream_t s)
{
    const int64_t blocks4 = (h.N + 3) / 4;
    const unsigned grid = (unsigned)((blocks4 + 255) / 256);
    if (h.model == ISING) hipLaunchKernelGGL(k_init<ISING>, dim3(grid), dim3(256), 0, s, d_desc, inst);
    else if (h.model == POTTS) hipLaunchKernelGGL(k_init<POTTS>, dim3(grid), dim3(256), 0, s, d_desc, inst);
    else hipLaunchKernelGGL(k_init<XY>, dim3(grid), dim3(256), 0, s, d_desc, inst);
    return hipGetLastError();
}

template <int MODEL, int DIM>
static hipError_t bond_dispatch(int v, const InstDesc *dd, const int2 *tm, int nt, uint32_t k, int mode,
                                hipStream_t s)
{
#define X(i, a, b, c)                                                                                 \
    if (v == i) {                                                                                     \
        hipLaunchKernelGGL((k_bond<MODEL, DIM, a, b, c>), dim3(nt), dim3(256), 0, s, dd, tm, k, mode); \
        return hipGetLastError();                                                                     \
    }
    if constexpr (MODEL != XY && DIM == 2) { SW_VARIANTS_ISING2 }
    if constexpr (MODEL != XY && DIM == 3) { SW_VARIANTS_ISING3 }
    if constexpr (MODEL == XY && DIM == 2) { SW_VARIANTS_XY2 }
    if constexpr (MODEL == XY && DIM == 3) { SW_VARIANTS_XY3 }
#undef X
    return hipErrorInvalidValue;
}

template <int MODEL, int DIM>
static hipError_t flip_dispatch(int v, const InstDesc *dd, const int2 *tm, int nt, uint32_t k, hipStream_t s)
{
#define X(i, a, b, c)                                                                         \
    if (v == i) {                                                                             \
        hipLaunchKernelGGL((k_flip<MODEL, DIM, a, b, c>), dim3(nt), dim3(256), 0, s, dd, tm, k); \
        return hipGetLastError();                                                             \
    }
    if constexpr (MODEL != XY && DIM == 2) { SW_VARIANTS_ISING2 }
    if constexpr (MODEL != XY && DIM == 3) { SW_VARIANTS_ISING3 }
    if constexpr (MODEL == XY && DIM == 2) { SW_VARIANTS_XY2 }
    if constexpr (MODEL == XY && DIM == 3) { SW_VARIANTS_XY3 }
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_bond(int model, int dim, int v, const InstDesc *dd, const int2 *tm, int nt, uint32_t k,
                       int mode, hipStream_t s)
{
    if (nt <= 0) return hipSuccess;
    if (model == ISING) return dim == 2 ? bond_dispatch<ISING, 2>(v, dd, tm, nt, k, mode, s)
                                        : bond_dispatch<ISING, 3>(v, dd, tm, nt, k, mode, s);
    if (model == POTTS) return dim == 2 ? bond_dispatch<POTTS, 2>(v, dd, tm, nt, k, mode, s)
                                        : bond_dispatch<POTTS, 3>(v, dd, tm, nt, k, mode, s);
    return dim == 2 ? bond_dispatch<XY, 2>(v, dd, tm, nt, k, mode, s) : bond_dispatch<XY, 3>(v, dd, tm, nt, k, mode, s);
}

hipError_t launch_merge(int dim, int model, int v, const InstDesc *dd, const int2 *tm, int nt, uint32_t k,
                        hipStream_t s)
{
    if (nt <= 0) return hipSuccess;
    const TileShape ts = tile_shape(model, dim, v);
    const int ext[3] = {ts.tx, ts.ty, dim == 3 ? ts.tz : 1};
    const int T = ext[0] * ext[1] * ext[2];
    int fmax = 0;
    for (int mu = 0; mu < dim; ++mu) fmax = T / ext[mu] > fmax ? T / ext[mu] : fmax;
    const long long blocks = ((long long)nt * fmax + 255) / 256;
    const dim3 grid((unsigned)blocks, dim);
    if (dim == 2) hipLaunchKernelGGL((k_merge<2>), grid, dim3(256), 0, s, dd, tm, nt, fmax, k);
    else hipLaunchKernelGGL((k_merge<3>), grid, dim3(256), 0, s, dd, tm, nt, fmax, k);
    return hipGetLastError();
}

hipError_t launch_reduce(int model, const InstDesc *dd, const int2 *tm, int nt, hipStream_t s)
{
    if (nt <= 0) return hipSuccess;
    if (model == ISING) hipLaunchKernelGGL((k_reduce<ISING>), dim3(nt), dim3(256), 0, s, dd, tm);
    else if (model == POTTS) hipLaunchKernelGGL((k_reduce<POTTS>), dim3(nt), dim3(256), 0, s, dd, tm);
    else hipLaunchKernelGGL((k_reduce<XY>), dim3(nt), dim3(256), 0, s, dd, tm);
    return hipGetLastError();
}

hipError_t launch_flip(int model, int dim, int v, const InstDesc *dd, const int2 *tm, int nt, uint32_t k,
                       hipStream_t s)
{
    if (nt <= 0) return hipSuccess;
    if (model == ISING) return dim == 2 ? flip_dispatch<ISING, 2>(v, dd, tm, nt, k, s)
                                        : flip_dispatch<ISING, 3>(v, dd, tm, nt, k, s);
    if (model == POTTS) return dim == 2 ? flip_dispatch<POTTS, 2>(v, dd, tm, nt, k, s)
                                        : flip_dispatch<POTTS, 3>(v, dd, tm, nt, k, s);
    return dim == 2 ? flip_dispatch<XY, 2>(v, dd, tm, nt, k, s) : flip_dispatch<XY, 3>(v, dd, tm, nt, k, s);
}

hipError_t launch_canon(const InstDesc *dd, int inst, int64_t N, int32_t *out, hipStream_t s)
{
    const unsigned grid = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL(k_canon, dim3(grid), dim3(256), 0, s, dd, inst, out);
    return hipGetLastError();
}

hipError_t launch_advance(InstDesc *dd, int ninst, hipStream_t s)
{
    hipLaunchKernelGGL(k_advance, dim3((ninst + 255) / 256), dim3(256), 0, s, dd, ninst);
    return hipGetLastError();
}

}  // namespace swmc

namespace swmc {

// ---------------------------------------------------------------------------
// Cluster statistics of the last labelling (diagnostic path of sw_measure).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_fill_i32(int32_t *p, int64_t n, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void __launch_bounds__(256) k_csize(const InstDesc *__restrict__ descs, int inst,
                                               int32_t *__restrict__ size)
{
    const InstDesc &d = descs[inst];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= d.N) return;
    uint32_t r = (uint32_t)i;
    uint32_t x = d.label[r];
    while (!(x & ROOT_FLAG)) {
        r = x;
        x = d.label[r];
    }
    atomicAdd(size + r, 1);
}

__global__ void __launch_bounds__(256) k_cstats(const int32_t *__restrict__ size, int64_t n,
                                                unsigned long long *out)
{
    __shared__ long long s_c[4], s_m[4], s_q[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    long long c = 0, m = 0, q = 0;
    if (i < n) {
        const long long v = size[i];
        c = v > 0;
        m = v;
        q = v * v;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        c += __shfl_xor(c, off, 64);
        q += __shfl_xor(q, off, 64);
        const long long o = __shfl_xor(m, off, 64);
        m = o > m ? o : m;
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_c[wv] = c;
        s_m[wv] = m;
        s_q[wv] = q;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long cc = 0, mm = 0, qq = 0;
        for (int w = 0; w < 4; ++w) {
            cc += s_c[w];
            qq += s_q[w];
            mm = s_m[w] > mm ? s_m[w] : mm;
        }
        atomicAdd(out + 0, (unsigned long long)cc);
        atomicMax(out + 1, (unsigned long long)mm);
        atomicAdd(out + 2, (unsigned long long)qq);
    }
}

hipError_t launch_cluster_stats(const InstDesc *dd, int inst, int64_t N, int32_t *scratch,
                                unsigned long long *out3, hipStream_t s)
{
    const unsigned grid = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid), dim3(256), 0, s, scratch, N, 0);
    hipLaunchKernelGGL(k_csize, dim3(grid), dim3(256), 0, s, dd, inst, scratch);
    hipLaunchKernelGGL(k_cstats, dim3(grid), dim3(256), 0, s, (const int32_t *)scratch, N, out3);
    return hipGetLastError();
}

}  // namespace swmc
