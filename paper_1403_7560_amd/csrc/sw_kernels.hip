// sw_kernels.hip -- gfx950 kernels of the Swendsen-Wang sweep.
//
// One sweep (Sec. 2 of the paper: (1) active bonds, (2) cluster labelling,
// (3) random state per cluster) is three launches per (model, dim) group:
//
//   k_bond   one workgroup per lattice tile, lane = tile column, each
//            wavefront a block of rows in registers.  Draws the bond words
//            (Philox4x32-10, one block per four rows of a column), forms the
//            bonds, measures the incoming configuration, then labels the
//            tile's clusters: a row-by-row scan of x-bond runs inheriting
//            labels from the row above (label equivalence, fixed point =
//            minimum index), with a union-find in LDS over run starts for the
//            remaining equivalences.  Local roots receive their cluster
//            decision; labels and the tile's two faces per direction go to HBM.
//   k_merge  global label equivalence across tiles: for every active bond
//            that crosses a tile face, link the larger root under the smaller
//            with device-scope atomicMin (Hawick's atomicMin on R[label],
//            retried until linked, so one pass reaches the fixed point).
//   k_flip   at the end of a launch chain, every site takes its root's
//            decision of the chain's last sweep (Ising +-1, Potts state, XY
//            mirror); within the chain k_bond applies each sweep's decisions
//            as it reads the next sweep's incoming states.
//
// Kernels read a per-lattice descriptor and a tile map, so one launch covers
// any number of lattices of one (model, dim) group (the batched form).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "sw_device.h"

namespace swmc {

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
        } else if (MODEL == CLOCK) {
            ((uint16_t *)d.state)[i] = (uint16_t)(((uint64_t)ws[m] * (uint64_t)d.q) >> 32);
        } else {
            const double t = ((double)ws[m] * 0x1p-32) * TWO_PI_D;
            float f = (float)t;
            if (f >= (float)TWO_PI_D) f = 0.0f;
            ((float *)d.state)[i] = f;
        }
    }
}

// ---------------------------------------------------------------------------
// Global label equivalence across tile faces.  One workgroup per tile: for
// every active bond across one of the tile's +mu faces, the two tile roots
// are linked on the global label words, the larger under the smaller, with
// device-scope atomicMin (Hawick's atomicMin on R[label], retried until it
// links, so one pass reaches the fixed point).  A cluster crosses a face at
// many sites with the same pair of tile roots, so the pairs are first made
// unique in an LDS hash set (the face element before each one is compared
// first, which removes most repeats without touching the set); the thread
// that inserts a pair links it.  All face elements of the tile are loaded at
// once, before any link, and a thread's links advance together
// (gunion_batch).  NT = 256 threads per workgroup (128-thread workgroups for
// the 2D tiles, twice the tiles per CU, were slower: the first workgroups'
// reduction of the records lengthens).  The first workgroups of a lattice
// also reduce the sweep's measurement partials.
// ---------------------------------------------------------------------------
template <int DIM, int EMAX, int NT>
__global__ void __launch_bounds__(NT) k_merge(const InstDesc *__restrict__ descs,
                                              const int2 *__restrict__ tmap, uint32_t k)
{
    // EMAX: face elements per thread (the tile shape's faces over NT threads)
    constexpr int HB = (DIM == 2) ? 512 : 2048;  // hash slots (about the face elements with a bond)
    constexpr unsigned long long EMPTY = ~0ull;
    __shared__ unsigned long long s_set[HB];
    const int2 tm = tmap[tile_slot()];
    if (tm.x < 0) return;
    const InstDesc &d = descs[tm.x];
    if (k >= d.count) return;
    const int t = tm.y;
    const int tid = threadIdx.x;
    // the first workgroups of a lattice also reduce the sweep's measurement
    if (d.measure && d.rec_row0 >= 0 && d.rec_row0 + (int64_t)k < d.rec_cap &&
        (t < d.nslots || (d.model >= XY && t == 0))) {
        if (d.model == ISING) reduce_partials<ISING, NT>(d, t, d.rec_row0 + (int64_t)k);
        else if (d.model == POTTS) reduce_partials<POTTS, NT>(d, t, d.rec_row0 + (int64_t)k);
        else reduce_partials<XY, NT>(d, t, d.rec_row0 + (int64_t)k);
    }
    uint32_t *lab = labels_of(d, d.sweep0 + k);
    for (int h = tid; h < HB; h += NT) s_set[h] = EMPTY;
    // the faces with a neighbour tile, one after the other in element order
    const int tc[3] = {t % d.tiles[0], (t / d.tiles[0]) % d.tiles[1],
                       (DIM == 3) ? t / (d.tiles[0] * d.tiles[1]) : 0};
    const GLOBAL int32_t *fo[DIM], *fi[DIM];
    int fend[DIM];  // end of face mu in element order
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
    // element e: face mu, position kk; out side a (-1: no bond), in side b
    int32_t a[EMAX], b[EMAX], pa[EMAX], pb[EMAX];
    bool first[EMAX];
#pragma unroll
    for (int i = 0; i < EMAX; ++i) {
        const int e = tid + NT * i;
        a[i] = b[i] = pa[i] = pb[i] = -1;
        first[i] = true;
        if (e < total) {
            int mu = 0, start = 0;
#pragma unroll
            for (int m = 0; m + 1 < DIM; ++m)
                if (e >= fend[m]) {
                    mu = m + 1;
                    start = fend[m];
                }
            const int kk = e - start;
            const GLOBAL int32_t *po = fo[0], *pi = fi[0];
#pragma unroll
            for (int m = 1; m < DIM; ++m)
                if (mu == m) {
                    po = fo[m];
                    pi = fi[m];
                }
            a[i] = po[kk];
            b[i] = pi[kk];
            first[i] = kk == 0;
            // lane 0 loads the element before it; the other lanes take their
            // left neighbour's below
            if ((tid & 63) == 0 && kk > 0) {
                pa[i] = po[kk - 1];
                pb[i] = pi[kk - 1];
            }
        }
    }
    __syncthreads();  // hash set cleared
    // the unique pairs this thread inserted are the ones it links
    uint32_t x[EMAX], y[EMAX];
    bool act[EMAX];
#pragma unroll
    for (int i = 0; i < EMAX; ++i) {
        act[i] = false;
        x[i] = (uint32_t)a[i];
        y[i] = (uint32_t)b[i];
        if (NT * i >= total) continue;  // uniform
        const int32_t la = (int32_t)from_left((uint32_t)a[i]), lb = (int32_t)from_left((uint32_t)b[i]);
        if ((tid & 63) != 0) {
            pa[i] = la;
            pb[i] = lb;
        }
        if (a[i] < 0) continue;
        if (!first[i] && pa[i] == a[i] && pb[i] == b[i]) continue;  // same pair as the element before
        act[i] = insert_pair(s_set, HB - 1, (uint32_t)a[i], (uint32_t)b[i]);
    }
    if (!gunion_batch<EMAX>(lab, x, y, act, d.walk_cap)) flag_error(d, ERR_WALK);
}

// Measurement of the current configuration alone: reduce into the scratch row.
template <int MODEL>
__global__ void __launch_bounds__(256) k_reduce(const InstDesc *__restrict__ descs, const int2 *__restrict__ tmap)
{
    const int2 tm = tmap[blockIdx.x];
    if (tm.x < 0) return;
    const InstDesc &d = descs[tm.x];
    if (tm.y >= d.nslots && !(MODEL == XY && tm.y == 0)) return;
    reduce_partials<MODEL, 256>(d, tm.y, d.rec_cap);
}

// Minimum-index labels: follow every chain to its root.
__global__ void __launch_bounds__(256) k_canon(const InstDesc *__restrict__ descs, int inst,
                                               int32_t *__restrict__ out)
{
    const InstDesc &d = descs[inst];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= d.N) return;
    const uint32_t *lab = labels_of(d, d.sweep0 - 1u);  // the last labelled sweep
    uint32_t r = (uint32_t)i;
    uint32_t x = lab[r], steps = 0;
    while (!(x & ROOT_FLAG)) {
        if (++steps > d.walk_cap) {
            flag_error(d, ERR_WALK);
            break;
        }
        r = x;
        x = lab[r];
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
// Variant table and launchers: X(variant, TX, TY, TZ, wavefronts per workgroup).
// The first shape of each table is the fastest on large lattices (it is the
// default unless it pads a small lattice much more than another shape).
// ---------------------------------------------------------------------------

int num_tile_variants(int model, int dim)
{
    int n = 0;
#define X(i, a, b, c, w) ++n;
    if (model < XY && dim == 2) { SW_VARIANTS_ISING2 }
    if (model < XY && dim == 3) { SW_VARIANTS_ISING3 }
    if (model >= XY && dim == 2) { SW_VARIANTS_XY2 }
    if (model >= XY && dim == 3) { SW_VARIANTS_XY3 }
#undef X
    return n;
}

TileShape tile_shape(int model, int dim, int v)
{
#define X(i, a, b, c, w) \
    if (v == i) return TileShape{a, b, c};
    if (model < XY && dim == 2) { SW_VARIANTS_ISING2 }
    if (model < XY && dim == 3) { SW_VARIANTS_ISING3 }
    if (model >= XY && dim == 2) { SW_VARIANTS_XY2 }
    if (model >= XY && dim == 3) { SW_VARIANTS_XY3 }
#undef X
    return TileShape{0, 0, 0};
}

bool tile_interior(int dim, int L, const TileShape &ts, int t)
{
    const int nx = (L + ts.tx - 1) / ts.tx, ny = (L + ts.ty - 1) / ts.ty;
    const int tx = t % nx, ty = (t / nx) % ny, tz = t / (nx * ny);
    return (tx + 1) * ts.tx <= L && (ty + 1) * ts.ty <= L && (dim == 2 || (tz + 1) * ts.tz <= L);
}

int slots_for(int model, int q) { return model == ISING ? 2 : (model == POTTS ? 1 + q : 3); }  // XY, clock: E, Mx, My

hipError_t launch_init(const InstDesc *d_desc, int inst, const InstDesc &h, hipStream_t s)
{
    const int64_t blocks4 = (h.N + 3) / 4;
    const unsigned grid = (unsigned)((blocks4 + 255) / 256);
    if (h.model == ISING) hipLaunchKernelGGL(k_init<ISING>, dim3(grid), dim3(256), 0, s, d_desc, inst);
    else if (h.model == POTTS) hipLaunchKernelGGL(k_init<POTTS>, dim3(grid), dim3(256), 0, s, d_desc, inst);
    else if (h.model == XY) hipLaunchKernelGGL(k_init<XY>, dim3(grid), dim3(256), 0, s, d_desc, inst);
    else hipLaunchKernelGGL(k_init<CLOCK>, dim3(grid), dim3(256), 0, s, d_desc, inst);
    return hipGetLastError();
}

template <int MODEL, int DIM>
static hipError_t merge_dispatch(int v, const InstDesc *dd, const int2 *tm, int nt, uint32_t k, hipStream_t s)
{
    // face elements of a tile: +x face TY TZ, +y face TX TZ, +z face TX TY
#define X(i, a, b, c, w)                                                                                   \
    if (v == i) {                                                                                          \
        constexpr int FT = (b) * (c) + (a) * (c) + (DIM == 3 ? (a) * (b) : 0);                            \
        constexpr int NTM = 256;                                                                           \
        hipLaunchKernelGGL((k_merge<DIM, (FT + NTM - 1) / NTM, NTM>), dim3(nt), dim3(NTM), 0, s, dd, tm, k); \
        return hipGetLastError();                                                                          \
    }
    if constexpr (MODEL < XY && DIM == 2) { SW_VARIANTS_ISING2 }
    if constexpr (MODEL < XY && DIM == 3) { SW_VARIANTS_ISING3 }
    if constexpr (MODEL >= XY && DIM == 2) { SW_VARIANTS_XY2 }
    if constexpr (MODEL >= XY && DIM == 3) { SW_VARIANTS_XY3 }
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_merge(int dim, int model, int v, const InstDesc *dd, const int2 *tm, int nt, uint32_t k,
                        hipStream_t s)
{
    if (nt <= 0) return hipSuccess;
    if (model >= XY) return dim == 2 ? merge_dispatch<XY, 2>(v, dd, tm, nt, k, s) : merge_dispatch<XY, 3>(v, dd, tm, nt, k, s);
    return dim == 2 ? merge_dispatch<ISING, 2>(v, dd, tm, nt, k, s) : merge_dispatch<ISING, 3>(v, dd, tm, nt, k, s);
}

hipError_t launch_reduce(int model, const InstDesc *dd, const int2 *tm, int nt, hipStream_t s)
{
    if (nt <= 0) return hipSuccess;
    if (model == ISING) hipLaunchKernelGGL((k_reduce<ISING>), dim3(nt), dim3(256), 0, s, dd, tm);
    else if (model == POTTS) hipLaunchKernelGGL((k_reduce<POTTS>), dim3(nt), dim3(256), 0, s, dd, tm);
    else hipLaunchKernelGGL((k_reduce<XY>), dim3(nt), dim3(256), 0, s, dd, tm);
    return hipGetLastError();
}

// Compute units of the current device (256 on the MI355X; also when no
// device answers).
static int device_cus()
{
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) {
            (void)hipGetLastError();
            n = 256;
        }
        cus = n;
    }
    return cus;
}

// 2D Ising/Potts shape 0 (64x64 tiles, 4 wavefronts) runs the 16-wavefront
// kernels of the same tile (shape 4) when the launch covers at most one tile
// per CU: such a launch cannot fill the GPU, and the shorter work per
// wavefront lowers its latency (2D Ising, us per sweep: L = 64 17.0 -> 10.7;
// L = 1024, one tile per CU, 34.8 -> 27.0; at L = 1536, 2.25 tiles per CU,
// the 4-wavefront kernel is the faster, 39.9 against 42.4).
// The tiles, and so the trajectory, are the same.
static int launch_variant(int model, int dim, int v, int nt)
{
    if (model < XY && dim == 2 && v == 0 && nt <= device_cus() && num_tile_variants(model, dim) > 4) return 4;
    return v;
}

hipError_t launch_bond(int model, int dim, int v, const InstDesc *dd, const int2 *tm, int nt, int nf, uint32_t k,
                       int mode, hipStream_t s, hipEvent_t t0, hipEvent_t t1)
{
    if (nt <= 0) return hipSuccess;
    if (nf < 0 || nf > nt) return hipErrorInvalidValue;
    v = launch_variant(model, dim, v, nt);
    if (model == ISING) return launch_bond_ising(dim, v, dd, tm, nt, nf, k, mode, s, t0, t1);
    if (model == POTTS) return launch_bond_potts(dim, v, dd, tm, nt, nf, k, mode, s, t0, t1);
    if (model == XY) return launch_bond_xy(dim, v, dd, tm, nt, nf, k, mode, s, t0, t1);
    return launch_bond_clock(dim, v, dd, tm, nt, nf, k, mode, s, t0, t1);
}

hipError_t launch_flip(int model, int dim, int v, const InstDesc *dd, const int2 *tm, int nt, uint32_t k,
                       hipStream_t s)
{
    v = launch_variant(model, dim, v, nt);
    if (nt <= 0) return hipSuccess;
    if (model == ISING) return launch_flip_ising(dim, v, dd, tm, nt, k, s);
    if (model == POTTS) return launch_flip_potts(dim, v, dd, tm, nt, k, s);
    if (model == XY) return launch_flip_xy(dim, v, dd, tm, nt, k, s);
    return launch_flip_clock(dim, v, dd, tm, nt, k, s);
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
    const uint32_t *lab = labels_of(d, d.sweep0 - 1u);  // the last labelled sweep
    uint32_t r = (uint32_t)i;
    uint32_t x = lab[r], steps = 0;
    while (!(x & ROOT_FLAG)) {
        if (++steps > d.walk_cap) {
            flag_error(d, ERR_WALK);
            break;
        }
        r = x;
        x = lab[r];
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

// ---------------------------------------------------------------------------
// Cluster statistics without any allocation, for callers that cannot call
// hipMalloc: the per-root sizes and the three sums live in one file-scope
// device array of STATIC_STATS_SITES + 8 words (16 MiB), which each GPU holds
// until the process ends.  Its name is a host-side stand-in in host code:
// the device address comes from hipGetSymbolAddress, once per device with
// that device current, and only that address is handed to kernels.  Every
// call on a GPU shares the array (overlapping calls race); each call clears
// what it uses.
// ---------------------------------------------------------------------------
static __device__ __align__(256) int32_t scratch[STATIC_STATS_SITES + 8];

static std::mutex g_scratch_mu;
static void *g_scratch_dev[MAX_DEVICES];

static hipError_t scratch_address(int32_t **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = p;
    }
    *out = (int32_t *)g_scratch_dev[dev];
    return hipSuccess;
}

hipError_t cluster_stats_static(const InstDesc *dd, int inst, int64_t N, unsigned long long host_out[3],
                                hipStream_t s)
{
    if (N < 1 || N > STATIC_STATS_SITES) return hipErrorInvalidValue;
    int32_t *base = nullptr;
    hipError_t e = scratch_address(&base);
    if (e != hipSuccess) return e;
    // sizes in words [0, N); the sums (three u64) after the last site slot,
    // 8-byte aligned because STATIC_STATS_SITES is even
    unsigned long long *out3 = (unsigned long long *)(base + STATIC_STATS_SITES);
    const unsigned grid = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid), dim3(256), 0, s, base, N, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, s, base + STATIC_STATS_SITES, (int64_t)6, 0);
    hipLaunchKernelGGL(k_csize, dim3(grid), dim3(256), 0, s, dd, inst, base);
    hipLaunchKernelGGL(k_cstats, dim3(grid), dim3(256), 0, s, (const int32_t *)base, N, out3);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(host_out, out3, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

}  // namespace swmc
