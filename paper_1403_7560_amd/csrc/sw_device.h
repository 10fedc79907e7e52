// sw_device.h -- device helpers shared by the kernel translation units of
// libswmc (product code; the oracle does not use it).
#pragma once
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
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
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
template <> struct StateOf<CLOCK> { typedef uint16_t type; };

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

// ---- union-find on the global label words -----------------------------------
// The finds read label words without device-wide coherence (an XCD's L2 may
// hold an older value).  That is safe: a word only ever moves to a smaller
// index of the same cluster, so an old value is still an ancestor, and the
// atomicMin that links roots is device-scope and returns the current word,
// from which the union continues.
__device__ __forceinline__ uint32_t glabel_load(uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void glabel_store(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of a on the global label words, with path halving (see lds_find).
// Every step spends one unit of `budget`; when it runs out the walk returns
// NO_ROOT (a valid forest never gets there: its chains strictly decrease).
constexpr uint32_t NO_ROOT = 0xFFFFFFFFu;
__device__ __forceinline__ uint32_t gfind(uint32_t *lab, uint32_t a, uint32_t &budget)
{
    while (budget != 0u) {
        --budget;
        const uint32_t p = glabel_load(lab + a);
        if (p & ROOT_FLAG) return a;
        const uint32_t g = glabel_load(lab + p);
        if (g & ROOT_FLAG) return p;
        glabel_store(lab + a, g);
        a = g;
    }
    return NO_ROOT;
}

// Link the clusters of a and b (larger root under smaller).  Returns false
// when the walk budget ran out before the two were joined.
__device__ __forceinline__ bool gunion(uint32_t *lab, uint32_t a, uint32_t b, uint32_t budget)
{
    while (true) {
        a = gfind(lab, a, budget);
        if (a == NO_ROOT) return false;
        b = gfind(lab, b, budget);
        if (b == NO_ROOT) return false;
        if (a == b) return true;
        if (a < b) {
            const uint32_t t = a;
            a = b;
            b = t;
        }
        // roots hold ROOT_FLAG|decision > any index, so atomicMin links a root
        const uint32_t old = atomicMin(lab + a, b);
        if (old & ROOT_FLAG) return true;
        a = old;
        if (budget == 0u) return false;
        --budget;
    }
}

// Insert the pair (a, b) into an LDS hash set of mask + 1 slots (empty slots
// hold all ones).  True when this call inserted it (or found no free slot
// within eight probes): the caller links the pair; false when it was there.
__device__ __forceinline__ bool insert_pair(unsigned long long *set, uint32_t mask, uint32_t a, uint32_t b)
{
    const unsigned long long key = ((unsigned long long)a << 32) | b;
    uint32_t h = (a * 0x9E3779B1u) ^ (b * 0x85EBCA77u);
    for (int probe = 0; probe < 8; ++probe) {
        h = (h + (uint32_t)probe) & mask;
        const unsigned long long old = atomicCAS(&set[h], ~0ull, key);
        if (old == ~0ull) return true;
        if (old == key) return false;
    }
    return true;
}

// The unions of up to E pairs of one thread, advanced together: each round
// takes one path-halving find step (as gfind) on both sides of every pending
// pair, the loads of all pairs in flight at once, then links every pair
// whose two sides have reached their roots with atomicMin (larger root under
// smaller), again all at once.  A link that finds its target linked
// meanwhile continues from the word it read, as gunion does.  So a thread's
// chains overlap instead of running one after the other.  Returns false
// when the rounds exceed `budget` (a valid forest never gets there).
template <int E>
__device__ __forceinline__ bool gunion_batch(uint32_t *lab, uint32_t (&x)[E], uint32_t (&y)[E], bool (&act)[E],
                                             uint32_t budget)
{
    bool any = false;
#pragma unroll
    for (int i = 0; i < E; ++i) any |= act[i];
    while (any) {
        if (budget == 0u) return false;
        --budget;
        uint32_t px[E], py[E], gx[E], gy[E];
#pragma unroll
        for (int i = 0; i < E; ++i) {
            px[i] = py[i] = ROOT_FLAG;
            if (act[i]) {
                px[i] = glabel_load(lab + x[i]);
                py[i] = glabel_load(lab + y[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < E; ++i) {
            gx[i] = (px[i] & ROOT_FLAG) ? px[i] : glabel_load(lab + px[i]);
            gy[i] = (py[i] & ROOT_FLAG) ? py[i] : glabel_load(lab + py[i]);
        }
        bool link[E];
#pragma unroll
        for (int i = 0; i < E; ++i) {
            link[i] = false;
            if (!act[i]) continue;
            if (!(px[i] & ROOT_FLAG)) {
                if (gx[i] & ROOT_FLAG) {
                    x[i] = px[i];
                } else {
                    glabel_store(lab + x[i], gx[i]);
                    x[i] = gx[i];
                }
            }
            if (!(py[i] & ROOT_FLAG)) {
                if (gy[i] & ROOT_FLAG) {
                    y[i] = py[i];
                } else {
                    glabel_store(lab + y[i], gy[i]);
                    y[i] = gy[i];
                }
            }
            const bool rx = (px[i] & ROOT_FLAG) || (gx[i] & ROOT_FLAG);
            const bool ry = (py[i] & ROOT_FLAG) || (gy[i] & ROOT_FLAG);
            if (rx && ry) {
                if (x[i] == y[i]) act[i] = false;
                else link[i] = true;
            }
        }
        uint32_t old[E];
#pragma unroll
        for (int i = 0; i < E; ++i) {
            old[i] = ROOT_FLAG;
            if (link[i]) {
                const uint32_t hi = max(x[i], y[i]), lo = min(x[i], y[i]);
                // roots hold ROOT_FLAG|decision > any index: atomicMin links a root
                old[i] = atomicMin(lab + hi, lo);
                y[i] = lo;
            }
        }
        any = false;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            if (link[i]) {
                if (old[i] & ROOT_FLAG) act[i] = false;
                else x[i] = old[i];  // linked meanwhile: join what it points at with lo
            }
            any |= act[i];
        }
    }
    return true;
}

// Record a capped walk in the lattice's error word.
__device__ __forceinline__ void flag_error(const InstDesc &d, uint32_t bit)
{
    atomicOr(d.err, bit);
}

// Word of the root reached from label word w (a root word is returned as it
// is), following at most `cap` links; past the cap the walk is flagged and
// reads as decision 0.
template <typename P>
__device__ __forceinline__ uint32_t root_word(P lab, uint32_t w, const InstDesc &d)
{
    uint32_t steps = 0;
    while (!(w & ROOT_FLAG)) {
        if (++steps > d.walk_cap) {
            flag_error(d, ERR_WALK);
            return ROOT_FLAG;
        }
        w = lab[w];
    }
    return w;
}

#define GLOBAL __attribute__((address_space(1)))

// Tile handled by this workgroup.  Workgroups are dealt to the 8 XCDs in
// turn, so slot b's neighbour b+1 runs on another XCD; this ordering keeps
// consecutive tiles (whose halos overlap) on one XCD and its L2.
__device__ __forceinline__ int tile_slot()
{
    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    if (nb & 7) return b;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

// Bytes of t that are zero -> bit 7 of that byte set (exact per byte: the
// masked sums cannot carry into the next byte).
__device__ __forceinline__ uint32_t zero_bytes(uint32_t t)
{
    return ~(((t & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | t) & 0x80808080u;
}

// Label words of sweep n: even sweeps in `label`, odd sweeps in `label2`, so
// that a sweep reads the previous sweep's clusters while it writes its own.
__device__ __forceinline__ uint32_t *labels_of(const InstDesc &d, uint32_t n)
{
    return (n & 1u) ? d.label2 : d.label;
}

// State byte of a site whose cluster's decision is dec (Ising: bit -> +-1).
template <int MODEL>
__device__ __forceinline__ uint32_t state_of_decision(uint32_t dec)
{
    return (MODEL == ISING) ? (dec ? 0xFFu : 0x01u) : dec;
}

// Value held by lane + 1 of the wavefront (DPP wavefront shift; lane 63 gets 0).
__device__ __forceinline__ uint32_t from_right(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xf, 0xf, false);
}

// Value held by lane - 1 of the wavefront (lane 0 gets 0).
__device__ __forceinline__ uint32_t from_left(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xf, 0xf, false);
}

// ---------------------------------------------------------------------------
// Reduction of the per-tile measurement partials into one record row, in a
// fixed order (deterministic, also for the XY sums).  Workgroup t of a
// lattice (NT threads) reduces slots t, t + ntiles, ... (XY: workgroup 0 all
// three).
// ---------------------------------------------------------------------------
template <int MODEL, int NT>
__device__ void reduce_partials(const InstDesc &d, int t, int64_t row)
{
    constexpr int NW = NT / 64;
    __shared__ double s_red[NW][3];
    const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
    GLOBAL int64_t *rec = (GLOBAL int64_t *)d.rec + row * d.nslots;
    const GLOBAL int64_t *part = (const GLOBAL int64_t *)d.part;
    if (MODEL == XY) {
        if (t != 0) return;
        double acc[3] = {0.0, 0.0, 0.0};
        for (int tt = tid; tt < d.ntiles; tt += NT)
            for (int c = 0; c < 3; ++c) acc[c] += __longlong_as_double(part[(int64_t)tt * 3 + c]);
        for (int c = 0; c < 3; ++c) {
            const double v = wave_sum_d(acc[c]);
            if (ln == 0) s_red[wv][c] = v;
        }
        __syncthreads();
        if (tid == 0) {
            double v[3] = {0.0, 0.0, 0.0};
            for (int w = 0; w < NW; ++w)
                for (int c = 0; c < 3; ++c) v[c] += s_red[w][c];
            rec[0] = __double_as_longlong(v[0]);
            rec[1] = __double_as_longlong(v[1]);
            rec[2] = __double_as_longlong(v[2]);
        }
        __syncthreads();
        return;
    }
    for (int slot = t; slot < d.nslots; slot += d.ntiles) {
        long long acc = 0;
        for (int tt = tid; tt < d.ntiles; tt += NT) acc += part[(int64_t)tt * d.nslots + slot];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (ln == 0) s_red[wv][0] = __longlong_as_double(acc);
        __syncthreads();
        if (tid == 0) {
            long long v = 0;
            for (int w = 0; w < NW; ++w) v += __double_as_longlong(s_red[w][0]);
            rec[slot] = v;
        }
        __syncthreads();
    }
}

// Tile shapes: X(variant, TX, TY, TZ, wavefronts per workgroup).  The first
// shape of each table is the fastest on large lattices (it is the default
// unless it pads a small lattice much more than another shape).
#define SW_VARIANTS_ISING2 X(0, 64, 64, 1, 4) X(1, 64, 32, 1, 4) X(2, 64, 128, 1, 8) X(3, 64, 256, 1, 16) X(4, 64, 64, 1, 16)
#define SW_VARIANTS_ISING3 X(0, 64, 8, 16, 8) X(1, 64, 8, 8, 4) X(2, 64, 4, 8, 4) X(3, 64, 16, 16, 16)
#define SW_VARIANTS_XY2 X(0, 64, 32, 1, 4) X(1, 64, 16, 1, 4) X(2, 64, 64, 1, 8)
#define SW_VARIANTS_XY3 X(0, 64, 4, 8, 4) X(1, 64, 8, 4, 4) X(2, 64, 8, 8, 8) X(3, 64, 8, 16, 16)

}  // namespace swmc
