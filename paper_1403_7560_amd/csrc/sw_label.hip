// sw_label.hip -- the paper's two iterative label-equivalence labellers for
// the global phase of step (2), selectable like its program's `algorithm`
// parameter (Sec. 2, program notes):
//
//   algorithm 0, after Hawick et al.: two label variables, the labels and a
//     temporary R; three functions iterated until a scan changes nothing:
//     scanning (a bonded pair with different labels lowers R[larger label]
//     to the smaller one with atomicMin), analysis (every label root follows
//     its R chain to the end) and labeling (label <- R[label]).
//   algorithm 1, after Kalentev et al.: the labels alone, two functions,
//     no atomic operation: scanning (the larger label's word takes the
//     smaller label with a plain store) and analysis (every node follows its
//     label chain to the root and keeps it).
//
// Both work where the one-pass atomic merge (k_merge) works: on the graph
// whose nodes are tile roots and whose edges are the active bonds across tile
// faces.  The bond kernel has already labelled every tile; the fixed point
// here is the same minimum-index labelling.
//
// One persistent launch per sweep runs every iteration: a cooperative grid
// (all workgroups resident) walks the group's tiles with the same
// workgroup-to-tile mapping in every phase, and the phases are separated by
// a grid barrier.  The convergence flag of iteration `it` is a device word
// that every workgroup reads after the barrier, so no iteration returns to
// the host.  Label words and R are read and written at device (agent) scope:
// the eight XCDs' L2 caches are not coherent with each other inside a launch,
// and the convergence test must see the last value of every word.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sw_device.h"

namespace swmc {

// ctl words of one launch (zeroed before it), one 128-byte line apart where
// many workgroups poll:
//   [0] barrier arrivals; [32 (1 + x)], x < 8: the barrier generation,
//   one copy per XCD so that the polling spreads over eight lines;
//   [288] abort (a barrier waited too long); [320 + it] changed flag of
//   iteration it (it < cap).
constexpr int CTL_BAR = 0, CTL_GEN = 32, CTL_ABORT = 288, CTL_CHG = 320;
// bound of one barrier wait, in ticks of the 100 MHz real-time counter
constexpr uint64_t BARRIER_WAIT_TICKS = 50000000ull;  // 0.5 s

__device__ __forceinline__ uint32_t aload(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void astore(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide barrier of a cooperative launch.  Every word another workgroup
// reads is accessed with device-scope atomics (they go to the coherence
// point, past the XCD's L2), so the barrier needs no cache maintenance, only
// that this workgroup's accesses have completed before it arrives: a
// waitcnt, the workgroup barrier, then one relaxed device-scope increment.
// The last workgroup to arrive publishes the new generation in eight copies
// (one per XCD); the others poll their copy with relaxed loads and a sleep.
// (Acquire loads would invalidate the XCD's L2 on every poll.)  The wait is
// bounded in time: past BARRIER_WAIT_TICKS, or once another workgroup gave
// up, it sets the abort word and returns false, and every workgroup exits.
__device__ bool grid_barrier(uint32_t *ctl, uint32_t &epoch)
{
    __shared__ int s_ok;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        ++epoch;
        const uint32_t arrived =
            __hip_atomic_fetch_add(ctl + CTL_BAR, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
        int ok = 1;
        if (arrived == epoch * gridDim.x) {
            for (int x = 0; x < 8; ++x) astore(ctl + CTL_GEN + 32 * x, epoch);
        } else {
            uint32_t *gen = ctl + CTL_GEN + 32 * (blockIdx.x & 7u);
            const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
            uint32_t spins = 0;
            while (aload(gen) != epoch) {
                __builtin_amdgcn_s_sleep(8);
                if ((++spins & 63u) == 0u &&
                    (aload(ctl + CTL_ABORT) != 0u || __builtin_amdgcn_s_memrealtime() - t0 > BARRIER_WAIT_TICKS)) {
                    astore(ctl + CTL_ABORT, 1u);
                    ok = 0;
                    break;
                }
            }
        }
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// Label of a node in the label-equivalence sense: the node itself while its
// word is a root word, else the index its word holds.
__device__ __forceinline__ uint32_t label_of(const uint32_t *lab, uint32_t x)
{
    const uint32_t w = aload(lab + x);
    return (w & ROOT_FLAG) ? x : w;
}

template <int DIM, int ALG, int EMAX>
__global__ void __launch_bounds__(256) k_label_iter(const InstDesc *__restrict__ descs,
                                                    const int2 *__restrict__ tmap, int ntiles, uint32_t k,
                                                    uint32_t *ctl, int cap)
{
    // EMAX: face elements per thread (the tile shape's faces over 256 threads)
    constexpr int HB = (DIM == 2) ? 512 : 2048;  // hash slots for the unique pairs of one tile
    constexpr unsigned long long EMPTY = ~0ull;
    __shared__ unsigned long long s_set[HB];
    __shared__ int s_n;
    const int tid = threadIdx.x;
    uint32_t epoch = 0;

    // ---- phase A: the unique (out root, in root) pairs of every tile -------
    for (int slot = blockIdx.x; slot < ntiles; slot += gridDim.x) {
        const int2 tm = tmap[slot];
        if (tm.x < 0) continue;  // uniform per workgroup
        const InstDesc &d = descs[tm.x];
        if (k >= d.count) continue;
        const int t = tm.y;
        // the first workgroups of a lattice also reduce the sweep's measurement
        if (d.measure && d.rec_row0 >= 0 && d.rec_row0 + (int64_t)k < d.rec_cap &&
            (t < d.nslots || (d.model >= XY && t == 0))) {
            if (d.model == ISING) reduce_partials<ISING, 256>(d, t, d.rec_row0 + (int64_t)k);
            else if (d.model == POTTS) reduce_partials<POTTS, 256>(d, t, d.rec_row0 + (int64_t)k);
            else reduce_partials<XY, 256>(d, t, d.rec_row0 + (int64_t)k);
        }
        for (int h = tid; h < HB; h += 256) s_set[h] = EMPTY;
        if (tid == 0) s_n = 0;
        const int tc[3] = {t % d.tiles[0], (t / d.tiles[0]) % d.tiles[1],
                           (DIM == 3) ? t / (d.tiles[0] * d.tiles[1]) : 0};
        const GLOBAL int32_t *fo[DIM], *fi[DIM];
        int fend[DIM];
        int total = 0;
#pragma unroll
        for (int mu = 0; mu < DIM; ++mu) {
            const int F = d.tiles[mu] > 1 ? d.face_len[mu] : 0;
            int cn[3] = {tc[0], tc[1], tc[2]};
            cn[mu] = (cn[mu] + 1 == d.tiles[mu]) ? 0 : cn[mu] + 1;
            const int nb = cn[0] + d.tiles[0] * (cn[1] + d.tiles[1] * cn[2]);
            fo[mu] = (const GLOBAL int32_t *)d.face + d.face_off[mu] + (int64_t)t * 2 * d.face_len[mu];
            fi[mu] = (const GLOBAL int32_t *)d.face + d.face_off[mu] + (int64_t)nb * 2 * d.face_len[mu] +
                     d.face_len[mu];
            total += F;
            fend[mu] = total;
        }
        int32_t a[EMAX], b[EMAX];
#pragma unroll
        for (int i = 0; i < EMAX; ++i) {
            const int e = tid + 256 * i;
            a[i] = b[i] = -1;
            if (e < total) {
                int mu = 0, start = 0;
#pragma unroll
                for (int m = 0; m + 1 < DIM; ++m)
                    if (e >= fend[m]) {
                        mu = m + 1;
                        start = fend[m];
                    }
                const GLOBAL int32_t *po = fo[0], *pi = fi[0];
#pragma unroll
                for (int m = 1; m < DIM; ++m)
                    if (mu == m) {
                        po = fo[m];
                        pi = fi[m];
                    }
                a[i] = po[e - start];
                b[i] = pi[e - start];
            }
        }
        __syncthreads();  // hash set cleared
        GLOBAL uint64_t *edges = (GLOBAL uint64_t *)d.edges + (int64_t)t * d.edge_cap;
        uint32_t *R = d.rbuf;
#pragma unroll
        for (int i = 0; i < EMAX; ++i) {
            // a face crossed at many sites repeats the pair: the element before
            // (lane - 1, read while every lane is active) is compared first, the
            // hash set catches the rest
            const int32_t la = (int32_t)from_left((uint32_t)a[i]), lb = (int32_t)from_left((uint32_t)b[i]);
            if (a[i] < 0 || a[i] == b[i]) continue;
            if ((tid & 63) != 0 && la == a[i] && lb == b[i]) continue;
            const unsigned long long key = ((unsigned long long)(uint32_t)a[i] << 32) | (uint32_t)b[i];
            uint32_t hsh = ((uint32_t)a[i] * 0x9E3779B1u) ^ ((uint32_t)b[i] * 0x85EBCA77u);
            bool fresh = true;
            for (int probe = 0; probe < 8; ++probe) {
                hsh = (hsh + (uint32_t)probe) & (HB - 1);
                const unsigned long long old = atomicCAS(&s_set[hsh], EMPTY, key);
                if (old == EMPTY) break;
                if (old == key) {
                    fresh = false;
                    break;
                }
            }
            if (!fresh) continue;
            const int pos = atomicAdd(&s_n, 1);  // < faces of the tile = edge_cap
            edges[pos] = ((uint64_t)(uint32_t)b[i] << 32) | (uint32_t)a[i];
            if (ALG == 0) {  // Hawick: R starts as the identity on the nodes
                astore(R + a[i], (uint32_t)a[i]);
                astore(R + b[i], (uint32_t)b[i]);
            }
        }
        __syncthreads();
        if (tid == 0) d.ecount[t] = s_n;
    }
    if (!grid_barrier(ctl, epoch)) return;

    // every phase below visits the tiles this workgroup compacted above, so
    // the edge lists and counts are its own writes
    auto for_edges = [&](auto &&f) {
        for (int slot = blockIdx.x; slot < ntiles; slot += gridDim.x) {
            const int2 tm = tmap[slot];
            if (tm.x < 0) continue;
            const InstDesc &d = descs[tm.x];
            if (k >= d.count) continue;
            const int ne = __hip_atomic_load(d.ecount + tm.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            uint64_t *edges = d.edges + (int64_t)tm.y * d.edge_cap;
            uint32_t *lab = labels_of(d, d.sweep0 + k);
            for (int e = tid; e < ne; e += 256) {
                const uint64_t v = __hip_atomic_load(edges + e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                f(d, lab, make_uint2((uint32_t)v, (uint32_t)(v >> 32)));
            }
        }
    };

    int it = 0;
    bool converged = false;
    for (; it < cap; ++it) {
        // ---- scanning ----------------------------------------------------
        int changed = 0;
        for_edges([&](const InstDesc &d, uint32_t *lab, uint2 e) {
            const uint32_t la = label_of(lab, e.x), lb = label_of(lab, e.y);
            if (la == lb) return;
            const uint32_t hi = la > lb ? la : lb, lo = la > lb ? lb : la;
            changed = 1;
            if (ALG == 0) {
                atomicMin(d.rbuf + hi, lo);  // Hawick: R[larger label] lowered atomically
            } else {
                // Kalentev: the larger label's word takes the smaller one with a
                // plain store; a lost race leaves the pair for the next scan
                const uint32_t w = aload(lab + hi);
                if ((w & ROOT_FLAG) || w > lo) astore(lab + hi, lo);
            }
        });
        if (__syncthreads_or(changed) && tid == 0) astore(ctl + CTL_CHG + it, 1u);
        if (!grid_barrier(ctl, epoch)) return;
        if (aload(ctl + CTL_CHG + it) == 0u) {  // the same value in every workgroup
            converged = true;
            break;
        }
        // ---- analysis ----------------------------------------------------
        for_edges([&](const InstDesc &d, uint32_t *lab, uint2 e) {
            const uint32_t ends[2] = {e.x, e.y};
            for (int s = 0; s < 2; ++s) {
                const uint32_t x = ends[s];
                uint32_t steps = 0;
                if (ALG == 0) {
                    // a label root follows R to its end and keeps it in R[x]
                    if (label_of(lab, x) != x) continue;
                    uint32_t ref = aload(d.rbuf + x), nxt = aload(d.rbuf + ref);
                    while (nxt != ref) {
                        if (++steps > d.walk_cap) {
                            flag_error(d, ERR_WALK);
                            break;
                        }
                        ref = nxt;
                        nxt = aload(d.rbuf + ref);
                    }
                    if (ref != aload(d.rbuf + x)) astore(d.rbuf + x, ref);
                } else {
                    // every node follows its label chain to the root and keeps it
                    uint32_t r = x, w = aload(lab + x);
                    if (w & ROOT_FLAG) continue;
                    const uint32_t first = w;
                    while (!(w & ROOT_FLAG)) {
                        if (++steps > d.walk_cap) {
                            flag_error(d, ERR_WALK);
                            break;
                        }
                        r = w;
                        w = aload(lab + r);
                    }
                    if ((w & ROOT_FLAG) && r != first) astore(lab + x, r);
                }
            }
        });
        if (!grid_barrier(ctl, epoch)) return;
        if (ALG == 0) {
            // ---- labeling: label <- R[label] -------------------------------
            for_edges([&](const InstDesc &d, uint32_t *lab, uint2 e) {
                const uint32_t ends[2] = {e.x, e.y};
                for (int s = 0; s < 2; ++s) {
                    const uint32_t x = ends[s];
                    const uint32_t l = label_of(lab, x), nl = aload(d.rbuf + l);
                    if (nl != l) astore(lab + x, nl);
                }
            });
            if (!grid_barrier(ctl, epoch)) return;
        }
    }
    // ---- bookkeeping: scans run, and the cap -------------------------------
    const uint32_t scans = converged ? (uint32_t)it + 1u : (uint32_t)cap;
    if (tid == 0)
        for (int slot = blockIdx.x; slot < ntiles; slot += gridDim.x) {
            const int2 tm = tmap[slot];
            if (tm.x < 0 || tm.y != 0) continue;  // once per lattice: its tile 0
            const InstDesc &d = descs[tm.x];
            if (k >= d.count) continue;
            if (!converged) flag_error(d, ERR_ITER);
            atomicAdd((unsigned long long *)d.lstats, 1ull);
            atomicAdd((unsigned long long *)d.lstats + 1, (unsigned long long)scans);
            atomicMax((unsigned long long *)d.lstats + 2, (unsigned long long)scans);
        }
}

// Fill n words with v (a kernel, not a memset: safe inside captured graphs).
__global__ void __launch_bounds__(256) k_fill_u32(uint32_t *p, int n, uint32_t v)
{
    for (int i = threadIdx.x; i < n; i += 256) p[i] = v;
}

// Device words a launch of the iterative labeller needs in `ctl`.
int label_ctl_words(int cap) { return CTL_CHG + cap; }

template <int DIM, int ALG, int EMAX>
static hipError_t launch_iter(const InstDesc *dd, const int2 *tm, int nt, uint32_t k, uint32_t *ctl, int cap,
                              hipStream_t s)
{
    // the whole grid must be resident: at most what the occupancy allows
    static int per_cu = -1, cus = 0;
    if (per_cu < 0) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_label_iter<DIM, ALG, EMAX>, 256, 0);
        if (e != hipSuccess) return e;
        if (per_cu < 1) return hipErrorLaunchOutOfResources;
    }
    // two workgroups per CU keep enough accesses in flight for the few
    // edges a phase has, and an eighth of the workgroups the barrier would
    // have at full occupancy
    const int cap_grid = (per_cu < 2 ? per_cu : 2) * cus;
    const int grid = nt < cap_grid ? nt : cap_grid;
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, s, ctl, label_ctl_words(cap), 0u);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    void *args[] = {(void *)&dd, (void *)&tm, (void *)&nt, (void *)&k, (void *)&ctl, (void *)&cap};
    return hipLaunchCooperativeKernel((const void *)k_label_iter<DIM, ALG, EMAX>, dim3(grid), dim3(256), args, 0, s);
}

template <int MODEL, int DIM>
static hipError_t label_dispatch(int v, int alg, const InstDesc *dd, const int2 *tm, int nt, uint32_t k,
                                 uint32_t *ctl, int cap, hipStream_t s)
{
#define X(i, a, b, c, w)                                                                          \
    if (v == i) {                                                                                 \
        constexpr int E = ((b) * (c) + (a) * (c) + (DIM == 3 ? (a) * (b) : 0) + 255) / 256;       \
        return alg == 0 ? launch_iter<DIM, 0, E>(dd, tm, nt, k, ctl, cap, s)                       \
                        : launch_iter<DIM, 1, E>(dd, tm, nt, k, ctl, cap, s);                      \
    }
    if constexpr (MODEL < XY && DIM == 2) { SW_VARIANTS_ISING2 }
    if constexpr (MODEL < XY && DIM == 3) { SW_VARIANTS_ISING3 }
    if constexpr (MODEL >= XY && DIM == 2) { SW_VARIANTS_XY2 }
    if constexpr (MODEL >= XY && DIM == 3) { SW_VARIANTS_XY3 }
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_label_iter(int dim, int model, int variant, int alg, const InstDesc *dd, const int2 *tm, int nt,
                             uint32_t k, uint32_t *ctl, int cap, hipStream_t s)
{
    if (nt <= 0) return hipSuccess;
    if ((alg != 0 && alg != 1) || cap < 1) return hipErrorInvalidValue;
    if (model >= XY)
        return dim == 2 ? label_dispatch<XY, 2>(variant, alg, dd, tm, nt, k, ctl, cap, s)
                        : label_dispatch<XY, 3>(variant, alg, dd, tm, nt, k, ctl, cap, s);
    return dim == 2 ? label_dispatch<ISING, 2>(variant, alg, dd, tm, nt, k, ctl, cap, s)
                    : label_dispatch<ISING, 3>(variant, alg, dd, tm, nt, k, ctl, cap, s);
}

}  // namespace swmc
