// sw_engine.cpp -- host runtime behind the C ABI in include/sw.h.
//
// Owns device memory, builds the per-lattice descriptors and tile maps the
// kernels read, drives the plain form (one lattice, one launch per kernel),
// the batched form (all lattices of a (model, dim) group in one launch, chunks
// of sweeps replayed from a captured HIP graph) and the served form
// (continuous batching of submitted jobs under an HBM budget).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/sw.h"
#include "sw_internal.h"

using namespace swmc;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(x)                                                                        \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess)                                                            \
            return fail(SW_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

const double PI_D_HOST = 3.141592653589793238462643383279;
const double TWO_PI_D_HOST = 6.283185307179586476925286766559;

size_t state_bytes(int model) { return model == XY ? 4 : (model == CLOCK ? 2 : 1); }

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Bond threshold floor(p 2^32) for Ising / Potts (Sec. 2, step (1)).
uint64_t bond_threshold(int model, double beta)
{
    const double p = (model == ISING) ? -std::expm1(-2.0 * beta) : -std::expm1(-beta);
    if (!(p > 0.0)) return 0;
    return (uint64_t)std::floor(std::ldexp(p, 32));
}

int validate(int model, int dim, int L, int q, double beta)
{
    if (model < 0 || model > 3) return fail(SW_E_INVALID, "model must be 0 (Ising), 1 (Potts), 2 (XY) or 3 (clock)");
    if (dim != 2 && dim != 3) return fail(SW_E_INVALID, "dim must be 2 or 3");
    if (L < 3) return fail(SW_E_INVALID, "L must be >= 3");
    double n = 1.0;
    for (int k = 0; k < dim; ++k) n *= (double)L;
    if (n > 2147483647.0) return fail(SW_E_INVALID, "L^dim must be < 2^31");
    if (model == POTTS && (q < 2 || q > 256)) return fail(SW_E_INVALID, "Potts needs 2 <= q <= 256");
    if (model == ISING && !(q == 0 || q == 2)) return fail(SW_E_INVALID, "Ising takes q = 2 (or 0)");
    if (model == CLOCK && (q < 2 || q > CLOCK_QMAX || (q & 1)))
        return fail(SW_E_INVALID, "the clock model needs an even q in [2, 512]");
    if (!(beta >= 0.0) || !std::isfinite(beta)) return fail(SW_E_INVALID, "beta must be finite and >= 0");
    return SW_OK;
}

// Reads and clears a device error word (ERR_* bits) once the work that may
// set it has completed; SW_E_NOCONV when a bit was set.
int check_error_word(uint32_t *err)
{
    uint32_t e = 0;
    HIPCHK(hipMemcpy(&e, err, 4, hipMemcpyDeviceToHost));
    if (e == 0) return SW_OK;
    const uint32_t zero = 0;
    HIPCHK(hipMemcpy(err, &zero, 4, hipMemcpyHostToDevice));
    std::string what;
    if (e & ERR_WALK) what += "a label walk or union exceeded its step cap";
    if (e & ERR_ITER) what += std::string(what.empty() ? "" : "; ") + "iterative labelling hit its iteration cap";
    return fail(SW_E_NOCONV, "labelling did not reach its fixed point: " + what);
}

}  // namespace

// ---------------------------------------------------------------------------
// Device memory a server recycles: the buffers of a retired job's lattice go
// back to a free list and the next admissions take them, so that jobs come
// and go without hipFree (which waits for the device) or hipMalloc.  A block
// is reused for a request of up to 1/8 less than its size; the free list
// holds at most `cap` bytes (the largest blocks are released beyond it).
// Blocks return only once the work that used them has completed (a server
// retires jobs between ticks).
// ---------------------------------------------------------------------------
struct DevicePool {
    std::multimap<size_t, void *> free_blocks;  // size -> block
    std::unordered_map<void *, size_t> sizes;   // every block the pool allocated
    size_t cached = 0;
    size_t cap = 0;

    hipError_t get(void **p, size_t n)
    {
        n = std::max<size_t>(n, 256);
        auto it = free_blocks.lower_bound(n);
        if (it != free_blocks.end() && it->first <= n + n / 8) {
            *p = it->second;
            cached -= it->first;
            free_blocks.erase(it);
            return hipSuccess;
        }
        hipError_t e = hipMalloc(p, n);
        if (e == hipSuccess) sizes[*p] = n;
        return e;
    }

    void put(void *p)
    {
        if (!p) return;
        auto s = sizes.find(p);
        if (s == sizes.end()) {
            (void)hipFree(p);
            return;
        }
        free_blocks.emplace(s->second, p);
        cached += s->second;
        while (cached > cap && !free_blocks.empty()) {
            auto big = std::prev(free_blocks.end());
            cached -= big->first;
            sizes.erase(big->second);
            (void)hipFree(big->second);
            free_blocks.erase(big);
        }
    }

    ~DevicePool()
    {
        for (auto &kv : free_blocks) (void)hipFree(kv.second);
    }
};

// ---------------------------------------------------------------------------
// One lattice and its device buffers.
// ---------------------------------------------------------------------------
struct Lattice;
// Appends the tiles of lattice j of a tile map: those wholly inside the lattice
// to `full`, those cut by its edge to `cut`.
static void append_tiles(const Lattice &l, int j, std::vector<int2> &full, std::vector<int2> &cut);

struct Lattice {
    int model = 0, dim = 2, L = 0, q = 2;
    double beta = 0.0;
    uint64_t seed = 0;
    uint32_t rep = 0;
    int64_t N = 0;
    int variant = 0;
    TileShape ts{0, 0, 0};
    int tiles[3] = {1, 1, 1};
    int ntiles = 0;
    int nfull = 0;  // tiles wholly inside the lattice, listed first in d_tmap
    int nslots = 0;
    int64_t sweep = 0;      // index of the next sweep
    int64_t rec_count = 0;  // records since the last reset
    int64_t rec_cap = 0;
    bool measure = true;
    bool store_bonds = true;
    // index of the last sweep whose labels are in the label buffers (-1: none);
    // the buffer is picked by its parity, whatever the sweep index is now
    int64_t labelled = -1;
    uint32_t walk_cap = 0;  // bound of every label walk (set to N + 1 at creation)
    uint32_t *err = nullptr;  // device error word (ERR_* bits); labelling statistics at byte 64
    // global phase of the labelling: SW_LABEL_UNION (one atomic pass), or the
    // paper's iterative SW_LABEL_HAWICK / SW_LABEL_KALENTEV (plain form)
    int labeller = SW_LABEL_UNION;
    int max_iters = 0;
    int edge_cap = 0;              // unique face pairs a tile can hold
    uint64_t *edges = nullptr;     // [ntiles][edge_cap]
    int32_t *ecount = nullptr;     // [ntiles]
    uint32_t *rbuf = nullptr;      // Hawick's R, N words
    uint32_t *ctl = nullptr;       // barrier and convergence words of one launch
    int ctl_words = 0;
    uint32_t *clock_thr = nullptr;  // clock model: bond thresholds of projection-index pairs
    double *clock_trig = nullptr;   // clock model: cos, sin of 2 pi k / q
    void *state = nullptr;
    uint32_t *label = nullptr;   // label words of even sweeps
    uint32_t *label2 = nullptr;  // label words of odd sweeps
    float *theta_w[2] = {nullptr, nullptr};  // XY: angles entering even / odd sweeps
    uint8_t *bond = nullptr;
    int32_t *face = nullptr;
    int64_t *part = nullptr;
    int64_t *rec = nullptr;
    int64_t face_off[3] = {0, 0, 0};
    int32_t face_len[3] = {0, 0, 0};
    InstDesc *d_solo = nullptr;  // descriptor for solo sweeps
    int2 *d_tmap = nullptr;      // tile map for solo sweeps
    hipStream_t stream = nullptr;
    // per-kernel event timing
    int profiling = 0;  // 1: events around k_bond; 2: also around the global phase and the flip
    // events bracket the launches of every PROFILE_EVERY-th sweep only: an
    // event pair around every launch would slow the sweep it measures
    static constexpr int64_t PROFILE_EVERY = 16;
    std::vector<hipEvent_t> events;
    double prof_ms[3] = {0, 0, 0};
    int64_t prof_n[3] = {0, 0, 0};
    // served lattices take their device buffers from the server's pool
    DevicePool *pool = nullptr;

    template <typename T>
    hipError_t dmalloc(T **p, size_t n)
    {
        void *v = nullptr;
        const hipError_t e = pool ? pool->get(&v, n) : hipMalloc(&v, n);
        *p = (T *)v;
        return e;
    }
    void dfree(void *p)
    {
        if (!p) return;
        if (pool) pool->put(p);
        else (void)hipFree(p);
    }

    ~Lattice()
    {
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        release();
    }

    int ensure_events(size_t n)
    {
        while (events.size() < n) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            events.push_back(e);
        }
        return SW_OK;
    }

    void release()
    {
        void *ptrs[] = {state, label, label2, theta_w[0], theta_w[1], bond, face, part, rec, d_solo, d_tmap, err,
                        edges, ecount, rbuf, ctl, clock_thr, clock_trig};
        for (void *p : ptrs) dfree(p);
        state = nullptr;
        label = nullptr;
        label2 = nullptr;
        theta_w[0] = theta_w[1] = nullptr;
        bond = nullptr;
        face = nullptr;
        part = nullptr;
        rec = nullptr;
        d_solo = nullptr;
        d_tmap = nullptr;
        err = nullptr;
        edges = nullptr;
        ecount = nullptr;
        rbuf = nullptr;
        ctl = nullptr;
        clock_thr = nullptr;
        clock_trig = nullptr;
    }

    static int64_t footprint(int model, int dim, int L, int q, int variant)
    {
        TileShape s = tile_shape(model, dim, variant);
        int t[3] = {(L + s.tx - 1) / s.tx, (L + s.ty - 1) / s.ty, dim == 3 ? (L + s.tz - 1) / s.tz : 1};
        int64_t N = 1;
        for (int k = 0; k < dim; ++k) N *= L;
        const int64_t nt = (int64_t)t[0] * t[1] * t[2];
        const int64_t T = (int64_t)s.tx * s.ty * (dim == 3 ? s.tz : 1);
        int64_t face = 0;
        const int ext[3] = {s.tx, s.ty, dim == 3 ? s.tz : 1};
        for (int mu = 0; mu < dim; ++mu)
            if (t[mu] > 1) face += nt * 2 * (T / ext[mu]) * 4;
        const int ns = slots_for(model, q);
        const int64_t tables = model == CLOCK ? (int64_t)(q / 2 + 1) * (q / 2 + 1) * 4 + 2 * q * 8 : 0;
        return N * (int64_t)state_bytes(model) * (model >= XY ? 3 : 1) + 2 * N * 4 + N + face + nt * ns * 8 +
               1025 * ns * 8 + tables + 256 +
               (int64_t)sizeof(InstDesc) + nt * 8;
    }

    InstDesc desc() const
    {
        InstDesc d;
        std::memset(&d, 0, sizeof(d));
        d.model = model;
        d.dim = dim;
        d.L = L;
        d.q = q;
        for (int k = 0; k < 3; ++k) d.tiles[k] = tiles[k];
        d.ntiles = ntiles;
        d.nslots = nslots;
        d.N = N;
        d.thr = (model >= XY) ? 0 : bond_threshold(model, beta);
        d.thr_hi = (uint32_t)(d.thr >> 16);
        d.thr_lo = (uint32_t)(d.thr & 0xffffu);
        d.two_beta = 2.0 * beta;
        d.key0 = (uint32_t)(seed & 0xffffffffu);
        d.key1 = (uint32_t)(seed >> 32);
        d.rep = rep;
        d.sweep0 = (uint32_t)sweep;
        d.count = 0;
        d.remaining = 0;
        d.chunk = 1;
        d.measure = measure ? 1 : 0;
        d.store_bonds = store_bonds ? 1 : 0;
        d.rec_row0 = measure ? rec_count : -1;
        d.rec_cap = rec_cap;
        d.state = state;
        d.label = label;
        d.label2 = label2;
        d.theta_w[0] = theta_w[0];
        d.theta_w[1] = theta_w[1];
        d.bond = bond;
        d.face = face;
        for (int k = 0; k < 3; ++k) {
            d.face_off[k] = face_off[k];
            d.face_len[k] = face_len[k];
        }
        d.part = part;
        d.rec = rec;
        d.err = err;
        d.walk_cap = walk_cap;
        d.edges = edges;
        d.ecount = ecount;
        d.edge_cap = edge_cap;
        d.rbuf = rbuf;
        d.lstats = (uint64_t *)((char *)err + 64);
        d.clock_thr = clock_thr;
        d.clock_trig = clock_trig;
        return d;
    }

    // Clock model tables (per q and beta): the integer bond threshold of two
    // projection indices m1, m2 in [0, q/2] -- floor(p 2^32), capped at
    // 2^32 - 1, with p = -expm1(-(2 beta)(cos(pi m1/q) cos(pi m2/q))); the
    // index q/2 (a spin perpendicular to the axis) never bonds -- and the
    // paper's pair-energy table rule[k] = cos(2 pi k/q) with sin(2 pi k/q)
    // for the magnetisation.
    int build_clock_tables()
    {
        const int H = q / 2 + 1;
        std::vector<double> c(H);
        for (int m = 0; m < H; ++m) c[m] = std::cos((PI_D_HOST * (double)m) / (double)q);
        std::vector<uint32_t> thr((size_t)H * H, 0u);
        for (int a = 0; a < H - 1; ++a)
            for (int b = 0; b < H - 1; ++b) {
                const double x = (2.0 * beta) * (c[a] * c[b]);
                const double p = -std::expm1(-x);
                if (!(p > 0.0)) continue;
                const double t = std::floor(std::ldexp(p, 32));
                thr[(size_t)a * H + b] = t >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)t;
            }
        std::vector<double> trig(2 * (size_t)q);
        for (int k = 0; k < q; ++k) {
            trig[k] = std::cos((TWO_PI_D_HOST * (double)k) / (double)q);
            trig[q + k] = std::sin((TWO_PI_D_HOST * (double)k) / (double)q);
        }
        if (dmalloc(&clock_thr, thr.size() * 4) != hipSuccess || dmalloc(&clock_trig, trig.size() * 8) != hipSuccess)
            return fail(SW_E_NOMEM, "clock table allocation failed");
        HIPCHK(hipMemcpy(clock_thr, thr.data(), thr.size() * 4, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(clock_trig, trig.data(), trig.size() * 8, hipMemcpyHostToDevice));
        return SW_OK;
    }

    // Select the global labelling phase; the iterative ones get their edge
    // lists, Hawick's R and the launch control words here.
    int set_labeller(int alg, int cap)
    {
        if (alg != SW_LABEL_HAWICK && alg != SW_LABEL_KALENTEV && alg != SW_LABEL_UNION)
            return fail(SW_E_INVALID, "algorithm must be 0 (Hawick), 1 (Kalentev) or 2 (union)");
        if (cap < 1 || cap > 4096) return fail(SW_E_INVALID, "iteration cap must be in [1, 4096]");
        if (alg != SW_LABEL_UNION) {
            int ec = 0;
            const int ext[3] = {ts.tx, ts.ty, dim == 3 ? ts.tz : 1};
            const int64_t T = (int64_t)ext[0] * ext[1] * ext[2];
            for (int mu = 0; mu < dim; ++mu)
                if (tiles[mu] > 1) ec += (int)(T / ext[mu]);
            if (!edges && dmalloc(&edges, (size_t)ntiles * std::max(ec, 1) * 8) != hipSuccess)
                return fail(SW_E_NOMEM, "edge list allocation failed");
            if (!ecount && dmalloc(&ecount, (size_t)ntiles * 4) != hipSuccess)
                return fail(SW_E_NOMEM, "edge count allocation failed");
            if (alg == SW_LABEL_HAWICK && !rbuf && dmalloc(&rbuf, (size_t)N * 4) != hipSuccess)
                return fail(SW_E_NOMEM, "R allocation failed");
            const int words = label_ctl_words(cap);
            if (words > ctl_words) {
                dfree(ctl);
                ctl = nullptr;
                if (dmalloc(&ctl, (size_t)words * 4) != hipSuccess) return fail(SW_E_NOMEM, "control words allocation failed");
                ctl_words = words;
            }
            edge_cap = ec;
        }
        labeller = alg;
        max_iters = cap;
        const uint64_t zero[3] = {0, 0, 0};
        HIPCHK(hipMemcpy((char *)err + 64, zero, sizeof(zero), hipMemcpyHostToDevice));
        return SW_OK;
    }

    // Global phase of sweep k of the current chain.
    hipError_t launch_global(uint32_t k)
    {
        if (ntiles <= 1) return hipSuccess;  // one tile: no faces, the bond kernel wrote the record
        if (labeller == SW_LABEL_UNION) return launch_merge(dim, model, variant, d_solo, d_tmap, ntiles, k, stream);
        return launch_label_iter(dim, model, variant, labeller, d_solo, d_tmap, ntiles, k, ctl, max_iters, stream);
    }

    // Descriptor whose previous sweep is the last labelled one (the label
    // readers take the buffer of sweep0 - 1).
    InstDesc labelled_desc() const
    {
        InstDesc d = desc();
        d.sweep0 = (uint32_t)(labelled + 1);
        return d;
    }

    // Reads and clears the device error word after a synchronised chain.
    int check_errors() { return check_error_word(err); }

    int grow_records(int64_t need)
    {
        if (need <= rec_cap) return SW_OK;
        int64_t cap = std::max<int64_t>(need, 2 * rec_cap);
        int64_t *p = nullptr;
        if (dmalloc(&p, (size_t)(cap + 1) * nslots * 8) != hipSuccess)
            return fail(SW_E_NOMEM, "record buffer allocation failed");
        if (rec && rec_count > 0)
            HIPCHK(hipMemcpy(p, rec, (size_t)rec_count * nslots * 8, hipMemcpyDeviceToDevice));
        dfree(rec);
        rec = p;
        rec_cap = cap;
        return SW_OK;
    }

    int create(int model_, int dim_, int L_, int q_, double beta_, uint64_t seed_, uint32_t rep_,
               int variant_, hipStream_t s)
    {
        int rc = validate(model_, dim_, L_, q_, beta_);
        if (rc) return rc;
        model = model_;
        dim = dim_;
        L = L_;
        q = (model == ISING) ? 2 : (model == XY ? 0 : q_);  // Potts and clock keep their q
        beta = beta_;
        seed = seed_;
        rep = rep_;
        variant = variant_;
        stream = s;
        ts = tile_shape(model, dim, variant);
        if (ts.tx == 0) return fail(SW_E_INVALID, "unknown tile variant");
        N = 1;
        for (int k = 0; k < dim; ++k) N *= L;
        tiles[0] = (L + ts.tx - 1) / ts.tx;
        tiles[1] = (L + ts.ty - 1) / ts.ty;
        tiles[2] = dim == 3 ? (L + ts.tz - 1) / ts.tz : 1;
        ntiles = tiles[0] * tiles[1] * tiles[2];
        nslots = slots_for(model, q);
        const int ext[3] = {ts.tx, ts.ty, dim == 3 ? ts.tz : 1};
        const int64_t T = (int64_t)ext[0] * ext[1] * ext[2];
        int64_t face_total = 0;
        for (int mu = 0; mu < 3; ++mu) {
            face_len[mu] = (mu < dim) ? (int32_t)(T / ext[mu]) : 0;
            face_off[mu] = face_total;
            if (mu < dim && tiles[mu] > 1) face_total += (int64_t)ntiles * 2 * face_len[mu];
        }
        if (dmalloc(&state, (size_t)N * state_bytes(model)) != hipSuccess ||
            dmalloc(&label, (size_t)N * 4) != hipSuccess || dmalloc(&label2, (size_t)N * 4) != hipSuccess ||
            dmalloc(&bond, (size_t)N) != hipSuccess ||
            (model >= XY && (dmalloc(&theta_w[0], (size_t)N * state_bytes(model)) != hipSuccess ||
                             dmalloc(&theta_w[1], (size_t)N * state_bytes(model)) != hipSuccess)) ||
            dmalloc(&face, (size_t)std::max<int64_t>(face_total, 1) * 4) != hipSuccess ||
            dmalloc(&part, (size_t)ntiles * nslots * 8) != hipSuccess ||
            dmalloc(&d_solo, sizeof(InstDesc)) != hipSuccess ||
            dmalloc(&d_tmap, (size_t)ntiles * sizeof(int2)) != hipSuccess ||
            dmalloc(&err, 256) != hipSuccess) {
            (void)hipGetLastError();
            return fail(SW_E_NOMEM, "device allocation failed");
        }
        walk_cap = (uint32_t)(N + 1);
        max_iters = 64;
        if (model == CLOCK) {
            rc = build_clock_tables();
            if (rc) return rc;
        }
        rc = grow_records(1024);
        if (rc) return rc;
        HIPCHK(hipMemsetAsync(err, 0, 256, stream));
        std::vector<int2> tm, cut;
        append_tiles(*this, 0, tm, cut);
        nfull = (int)tm.size();
        tm.insert(tm.end(), cut.begin(), cut.end());
        HIPCHK(hipMemcpy(d_tmap, tm.data(), tm.size() * sizeof(int2), hipMemcpyHostToDevice));
        HIPCHK(hipMemsetAsync(bond, 0, (size_t)N, stream));
        // face slots outside the lattice (ragged tiles) are never written and
        // must read as "no bond" (-1)
        HIPCHK(hipMemsetAsync(face, 0xFF, (size_t)std::max<int64_t>(face_total, 1) * 4, stream));
        // hot start
        InstDesc d = desc();
        HIPCHK(hipMemcpyAsync(d_solo, &d, sizeof(d), hipMemcpyHostToDevice, stream));
        HIPCHK(hipStreamSynchronize(stream));
        HIPCHK(launch_init(d_solo, 0, d, stream));
        HIPCHK(hipStreamSynchronize(stream));
        return SW_OK;
    }

    // Solo sweeps: one lattice, one launch per kernel per sweep.
    int sweep_solo(int64_t n)
    {
        while (n > 0) {
            const int64_t m = std::min<int64_t>(n, 1 << 30);
            if (sweep + m > 0xFFFFFFFFll) return fail(SW_E_INVALID, "sweep index would pass 2^32");
            if (measure) {
                int rc = grow_records(rec_count + m);
                if (rc) return rc;
            }
            InstDesc d = desc();
            d.count = (uint32_t)m;
            HIPCHK(hipMemcpyAsync(d_solo, &d, sizeof(d), hipMemcpyHostToDevice, stream));
            HIPCHK(hipStreamSynchronize(stream));
            // timed sweeps: those whose index is a multiple of PROFILE_EVERY
            const int64_t first_timed = (PROFILE_EVERY - sweep % PROFILE_EVERY) % PROFILE_EVERY;
            const int64_t ntimed = first_timed < m ? (m - 1 - first_timed) / PROFILE_EVERY + 1 : 0;
            if (profiling) {
                // 4 per timed sweep, then the pair around the chain's flip
                int rc = ensure_events((size_t)(4 * std::max<int64_t>(ntimed, 1) + 2));
                if (rc) return rc;
            }
            hipEvent_t *fev = profiling > 1 ? &events[events.size() - 2] : nullptr;
            // each sweep's bond kernel applies the previous sweep's cluster
            // decisions; the chain's last decisions are applied once at the end
            for (int64_t k = 0; k < m; ++k) {
                const bool timed = profiling && k >= first_timed && (k - first_timed) % PROFILE_EVERY == 0;
                hipEvent_t *ev = timed ? &events[(size_t)(4 * ((k - first_timed) / PROFILE_EVERY))] : nullptr;
                // the bond launch records ev[0] / ev[1] itself (its own start and end)
                HIPCHK(launch_bond(model, dim, variant, d_solo, d_tmap, ntiles, nfull, (uint32_t)k, 0, stream,
                                   ev ? ev[0] : nullptr, ev ? ev[1] : nullptr));
                HIPCHK(launch_global((uint32_t)k));
                if (ev && profiling > 1) HIPCHK(hipEventRecord(ev[2], stream));
            }
            if (fev) HIPCHK(hipEventRecord(fev[0], stream));
            HIPCHK(launch_flip(model, dim, variant, d_solo, d_tmap, ntiles, FLIP_LAST, stream));
            if (fev) HIPCHK(hipEventRecord(fev[1], stream));
            HIPCHK(hipStreamSynchronize(stream));
            if (fev) {
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, fev[0], fev[1]));
                prof_ms[2] += ms;
                prof_n[2] += 1;
            }
            if (profiling) {
                const int nk = profiling > 1 ? 2 : 1;
                for (int64_t k = 0; k < ntimed; ++k) {
                    for (int c = 0; c < nk; ++c) {
                        float ms = 0.f;
                        HIPCHK(hipEventElapsedTime(&ms, events[(size_t)(4 * k + c)], events[(size_t)(4 * k + c + 1)]));
                        prof_ms[c] += ms;
                        prof_n[c] += 1;
                    }
                }
            }
            sweep += m;
            if (measure) rec_count += m;
            if (m > 0) labelled = sweep - 1;
            n -= m;
            int rc = check_errors();
            if (rc) return rc;
        }
        return SW_OK;
    }

    // Measure the current configuration alone into the scratch record row.
    int measure_now(std::vector<int64_t> &row)
    {
        InstDesc d = desc();
        d.count = 1;
        HIPCHK(hipMemcpyAsync(d_solo, &d, sizeof(d), hipMemcpyHostToDevice, stream));
        HIPCHK(hipStreamSynchronize(stream));
        HIPCHK(launch_bond(model, dim, variant, d_solo, d_tmap, ntiles, nfull, 0, 1, stream));
        HIPCHK(launch_reduce(model, d_solo, d_tmap, ntiles, stream));
        row.assign(nslots, 0);
        HIPCHK(hipMemcpyAsync(row.data(), rec + rec_cap * nslots, (size_t)nslots * 8, hipMemcpyDeviceToHost,
                              stream));
        HIPCHK(hipStreamSynchronize(stream));
        return SW_OK;
    }

    sw_record to_record(const int64_t *r, int64_t sweep_index) const
    {
        sw_record o;
        std::memset(&o, 0, sizeof(o));
        o.sweep = sweep_index;
        const double dN = (double)dim * (double)N;
        if (model == ISING) {
            const int64_t al = r[0], M = r[1];
            o.energy = dN - 2.0 * (double)al;
            o.mx = (double)M;
            o.mag = (double)M;
            o.mag2 = (double)M * (double)M;
        } else if (model == POTTS) {
            o.energy = dN - (double)r[0];
            __int128 s2 = 0;
            for (int k = 0; k < q; ++k) s2 += (__int128)r[1 + k] * r[1 + k];
            const __int128 num = (__int128)q * s2 - (__int128)N * N;
            o.mag2 = (double)num / (double)(q - 1);
            o.mag = std::sqrt(std::max(0.0, o.mag2));
        } else {  // XY and clock: E, Mx, My as doubles
            double v[3];
            std::memcpy(v, r, sizeof(v));
            o.energy = v[0];
            o.mx = v[1];
            o.my = v[2];
            o.mag2 = v[1] * v[1] + v[2] * v[2];
            o.mag = std::sqrt(o.mag2);
        }
        return o;
    }

    int series(std::vector<sw_record> &out, int64_t max)
    {
        const int64_t n = std::min<int64_t>(rec_count, max);
        out.clear();
        if (n <= 0) return SW_OK;
        std::vector<int64_t> raw((size_t)n * nslots);
        HIPCHK(hipMemcpy(raw.data(), rec, raw.size() * 8, hipMemcpyDeviceToHost));
        const int64_t first = sweep - rec_count;
        for (int64_t i = 0; i < n; ++i) out.push_back(to_record(&raw[(size_t)i * nslots], first + i));
        return SW_OK;
    }

    int cluster_stats(sw_cluster_stats *cs)
    {
        std::memset(cs, 0, sizeof(*cs));
        if (labelled < 0) return SW_OK;
        int32_t *scratch = nullptr;
        unsigned long long *out = nullptr;
        if (hipMalloc(&scratch, (size_t)N * 4) != hipSuccess || hipMalloc(&out, 24) != hipSuccess) {
            if (scratch) (void)hipFree(scratch);
            return fail(SW_E_NOMEM, "cluster statistics scratch allocation failed");
        }
        unsigned long long h[3] = {0, 0, 0};
        // its sweep index names the last labelled sweep's buffer
        InstDesc d = labelled_desc();
        hipError_t e = hipMemcpyAsync(d_solo, &d, sizeof(d), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(out, h, 24, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = launch_cluster_stats(d_solo, 0, N, scratch, out, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(h, out, 24, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        (void)hipFree(scratch);
        (void)hipFree(out);
        if (e != hipSuccess) return fail(SW_E_DEVICE, std::string("cluster statistics: ") + hipGetErrorString(e));
        cs->n_clusters = (int64_t)h[0];
        cs->max_cluster = (int64_t)h[1];
        cs->sum_c2 = (int64_t)h[2];
        return check_errors();
    }

    // Moments of the recorded series since the last reset (the current
    // configuration alone when nothing is recorded): Sec. 2's printed
    // outputs (<m^2>, <m^4>, energy and specific heat per spin) plus <|m|>
    // and the moment ratio of Sec. 3, Eq. (6).
    int moments(sw_moments *o)
    {
        std::vector<sw_record> recs;
        if (rec_count > 0) {
            int rc = series(recs, rec_count);
            if (rc) return rc;
        } else {
            std::vector<int64_t> row;
            int rc = measure_now(row);
            if (rc) return rc;
            recs.push_back(to_record(row.data(), sweep));
        }
        const double n = (double)recs.size(), dN = (double)N, n2 = dN * dN;
        double a1 = 0, a2 = 0, a4 = 0, ae = 0;
        for (const sw_record &r : recs) {
            const double x = r.mag2 / n2;
            a1 += std::fabs(r.mag) / dN;
            a2 += x;
            a4 += x * x;
            ae += r.energy / dN;
        }
        const double em = ae / n;
        double ve = 0, ae2 = 0;  // two passes: the variance without cancellation
        for (const sw_record &r : recs) {
            const double e = r.energy / dN;
            ve += (e - em) * (e - em);
            ae2 += e * e;
        }
        std::memset(o, 0, sizeof(*o));
        o->n = (int64_t)recs.size();
        o->abs_m = a1 / n;
        o->m2 = a2 / n;
        o->m4 = a4 / n;
        o->energy = em;
        o->energy2 = ae2 / n;
        // C/N = beta^2 (<E^2> - <E>^2) / N = beta^2 N (<e^2> - <e>^2), e = E/N
        o->specific_heat = beta * beta * dN * (ve / n);
        o->binder = o->m2 > 0.0 ? o->m4 / (o->m2 * o->m2) : 0.0;
        return SW_OK;
    }

    int averages(double *m2, double *m4, double *energy)
    {
        sw_moments o;
        int rc = moments(&o);
        if (rc) return rc;
        if (m2) *m2 = o.m2;
        if (m4) *m4 = o.m4;
        if (energy) *energy = o.energy;
        return SW_OK;
    }
};

static void append_tiles(const Lattice &l, int j, std::vector<int2> &full, std::vector<int2> &cut)
{
    for (int t = 0; t < l.ntiles; ++t) (tile_interior(l.dim, l.L, l.ts, t) ? full : cut).push_back(make_int2(j, t));
}

struct sw_ctx {
    Lattice *lat = nullptr;
    bool owned = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
};

// Streams live until the process ends and are handed out again in the order
// they were given back.  The runtime binds a stream to one of its few hardware
// queues at the stream's first launch; streams created after others were
// destroyed can land two to a queue while other queues sit idle, which
// serialises launches meant to overlap (measured: a second server in one
// process ran 10% slower than the first until its streams were reused).
static std::mutex g_stream_mu;
static std::deque<std::pair<int, hipStream_t>> g_free_streams;  // (device, stream)
static std::unordered_map<hipStream_t, int> g_stream_dev;

static hipStream_t make_stream()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_stream_mu);
    for (auto it = g_free_streams.begin(); it != g_free_streams.end(); ++it)
        if (it->first == dev) {
            hipStream_t s = it->second;
            g_free_streams.erase(it);
            return s;
        }
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    g_stream_dev[s] = dev;
    return s;
}

// Give a stream from make_stream back once its work has finished.
static void release_stream(hipStream_t s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s);
    std::lock_guard<std::mutex> lk(g_stream_mu);
    auto it = g_stream_dev.find(s);
    if (it == g_stream_dev.end()) return;
    g_free_streams.emplace_back(it->second, s);
}

// ---------------------------------------------------------------------------
// Tile shapes chosen by the tuner, per (model, dim, L); lattices created
// without an explicit shape take the tuned one, else shape 0.  The shape
// never changes a trajectory (labels are canonical, random words are drawn
// per site), only the speed.
// ---------------------------------------------------------------------------
static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int>, int> g_tuned;

// Shape of a lattice nobody has tuned: the first of the table (the fastest on
// large lattices) unless padding the lattice to whole tiles of it costs more
// than sn/sd (a quarter) over the shape that pads least.
static int default_tile(int model, int dim, int L, int64_t sn = 5, int64_t sd = 4)
{
    auto padded = [&](int v) {
        const TileShape s = tile_shape(model, dim, v);
        const int e[3] = {s.tx, s.ty, dim == 3 ? s.tz : 1};
        int64_t p = 1;
        for (int mu = 0; mu < dim; ++mu) {
            if (e[mu] <= 0) return INT64_MAX;  // no such shape
            p *= (int64_t)((L + e[mu] - 1) / e[mu]) * e[mu];
        }
        return p;
    };
    if (num_tile_variants(model, dim) <= 0 || L <= 0) return 0;
    int best = 0;
    int64_t pmin = padded(0);
    for (int v = 1; v < num_tile_variants(model, dim); ++v)
        if (padded(v) < pmin) {
            best = v;
            pmin = padded(v);
        }
    return padded(0) * sd <= pmin * sn ? 0 : best;
}

static int tuned_tile(int model, int dim, int L)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(std::make_tuple(model, dim, L));
    return it == g_tuned.end() ? default_tile(model, dim, L) : it->second;
}

// The same for a served job.  The server's launches cover many lattices and
// fill the chip, and there the first shape is the fastest per padded site
// (the 300-job served mix ran at 55.8 updates/ns against 54.9 under the rule
// above): it gives way only to a shape that pads the lattice to under two
// thirds as many sites.
static int served_tile(int model, int dim, int L)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(std::make_tuple(model, dim, L));
    return it == g_tuned.end() ? default_tile(model, dim, L, 3, 2) : it->second;
}

// ---------------------------------------------------------------------------
// Batched form.
// ---------------------------------------------------------------------------
struct Group {
    int model, dim, variant;
    std::vector<int> members;
    int ntiles = 0;
    int nfull = 0;  // leading tile-map entries wholly inside their lattice
    int2 *d_tmap = nullptr;
};

// The lattices of a batch are dealt to a few parts, each with its own
// stream, descriptors, tile maps and captured graph: the parts' launches are
// independent, so one part's latency-bound label merge can run beside
// another part's bond kernel on the CUs the first leaves free.
struct BatchPart {
    std::vector<int> members;  // batch indices; the part's descriptor j is members[j]
    std::vector<Group> groups;
    InstDesc *d_desc = nullptr;
    InstDesc *h_desc = nullptr;  // pinned
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipGraphExec_t graph = nullptr;
    int graph_chunk = 0;

    ~BatchPart()
    {
        if (graph) (void)hipGraphExecDestroy(graph);
        for (Group &g : groups)
            if (g.d_tmap) (void)hipFree(g.d_tmap);
        if (d_desc) (void)hipFree(d_desc);
        if (h_desc) (void)hipHostFree(h_desc);
        if (own_stream && stream) release_stream(stream);
    }
};

struct sw_batch_s {
    std::vector<std::unique_ptr<Lattice>> lats;
    std::vector<std::unique_ptr<sw_ctx>> views;
    std::vector<std::unique_ptr<BatchPart>> parts;
    uint32_t *d_err = nullptr;   // error word shared by the members' batched launches
    hipStream_t stream = nullptr;  // the batch's first stream (part 0's)
    int chunk = 16;

    ~sw_batch_s()
    {
        parts.clear();
        if (d_err) (void)hipFree(d_err);
        lats.clear();
        if (stream) release_stream(stream);
    }

    // Deal the lattices to n parts (largest first, each to the part with the
    // fewest sites so far) and build every part's groups and tile maps.
    int build_parts(int n)
    {
        if (stream) HIPCHK(hipStreamSynchronize(stream));
        for (auto &pt : parts)
            if (pt->stream) HIPCHK(hipStreamSynchronize(pt->stream));
        parts.clear();
        n = std::max(1, std::min<int>(n, (int)lats.size()));
        std::vector<int> order((size_t)lats.size());
        for (size_t j = 0; j < lats.size(); ++j) order[j] = (int)j;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return lats[a]->N > lats[b]->N; });
        std::vector<int64_t> load((size_t)n, 0);
        for (int i = 0; i < n; ++i) parts.emplace_back(new BatchPart());
        for (int j : order) {
            const int p = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            parts[p]->members.push_back(j);
            load[p] += lats[j]->N;
        }
        for (int p = 0; p < n; ++p) {
            BatchPart &pt = *parts[p];
            std::sort(pt.members.begin(), pt.members.end());
            if (p == 0) {
                pt.stream = stream;
            } else {
                pt.stream = make_stream();
                if (!pt.stream) return fail(SW_E_DEVICE, "hipStreamCreate failed");
                pt.own_stream = true;
            }
            std::map<std::tuple<int, int, int>, int> index;
            for (int jl = 0; jl < (int)pt.members.size(); ++jl) {
                Lattice &l = *lats[pt.members[jl]];
                l.stream = pt.stream;  // the member's own calls run on its part's stream
                views[pt.members[jl]]->stream = pt.stream;
                auto key = std::make_tuple(l.model, l.dim, l.variant);
                auto it = index.find(key);
                if (it == index.end()) {
                    index[key] = (int)pt.groups.size();
                    pt.groups.push_back(Group{l.model, l.dim, l.variant, {}, 0, 0, nullptr});
                    it = index.find(key);
                }
                pt.groups[it->second].members.push_back(jl);
            }
            for (Group &g : pt.groups) {
                std::vector<int2> tm, cut;
                for (int jl : g.members) append_tiles(*lats[pt.members[jl]], jl, tm, cut);
                g.nfull = (int)tm.size();
                tm.insert(tm.end(), cut.begin(), cut.end());
                g.ntiles = (int)tm.size();
                if (hipMalloc(&g.d_tmap, tm.size() * sizeof(int2)) != hipSuccess)
                    return fail(SW_E_NOMEM, "tile map allocation failed");
                HIPCHK(hipMemcpy(g.d_tmap, tm.data(), tm.size() * sizeof(int2), hipMemcpyHostToDevice));
            }
            const size_t m = pt.members.size();
            if (hipMalloc(&pt.d_desc, m * sizeof(InstDesc)) != hipSuccess ||
                hipHostMalloc(&pt.h_desc, m * sizeof(InstDesc), hipHostMallocDefault) != hipSuccess)
                return fail(SW_E_NOMEM, "descriptor allocation failed");
        }
        if (!d_err) {
            if (hipMalloc(&d_err, 256) != hipSuccess) return fail(SW_E_NOMEM, "error word allocation failed");
            HIPCHK(hipMemset(d_err, 0, 256));
        }
        return SW_OK;
    }

    int enqueue_chunk(BatchPart &pt, int S)
    {
        for (int k = 0; k < S; ++k) {
            for (const Group &g : pt.groups)
                HIPCHK(launch_bond(g.model, g.dim, g.variant, pt.d_desc, g.d_tmap, g.ntiles, g.nfull, (uint32_t)k, 0,
                                   pt.stream));
            for (const Group &g : pt.groups)
                HIPCHK(launch_merge(g.dim, g.model, g.variant, pt.d_desc, g.d_tmap, g.ntiles, (uint32_t)k, pt.stream));
        }
        for (const Group &g : pt.groups)
            HIPCHK(launch_flip(g.model, g.dim, g.variant, pt.d_desc, g.d_tmap, g.ntiles, FLIP_LAST, pt.stream));
        HIPCHK(launch_advance(pt.d_desc, (int)pt.members.size(), pt.stream));
        return SW_OK;
    }

    int capture(BatchPart &pt, int S)
    {
        if (pt.graph && pt.graph_chunk == S) return SW_OK;
        if (pt.graph) {
            (void)hipGraphExecDestroy(pt.graph);
            pt.graph = nullptr;
        }
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(pt.stream, hipStreamCaptureModeThreadLocal));
        int rc = enqueue_chunk(pt, S);
        hipError_t e = hipStreamEndCapture(pt.stream, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        HIPCHK(e);
        e = hipGraphInstantiate(&pt.graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPCHK(e);
        pt.graph_chunk = S;
        return SW_OK;
    }

    int sweep_counts(const int64_t *counts)
    {
        int64_t maxc = 0;
        for (size_t j = 0; j < lats.size(); ++j) {
            if (counts[j] < 0) return fail(SW_E_INVALID, "negative sweep count");
            if (lats[j]->sweep + counts[j] > 0xFFFFFFFFll) return fail(SW_E_INVALID, "sweep index would pass 2^32");
            if (counts[j] >= (1ll << 31)) return fail(SW_E_INVALID, "sweep count too large");
            maxc = std::max(maxc, counts[j]);
        }
        if (maxc == 0) return SW_OK;
        const int S = chunk;
        for (size_t j = 0; j < lats.size(); ++j) {
            Lattice &l = *lats[j];
            if (l.measure) {
                int rc = l.grow_records(l.rec_count + counts[j]);
                if (rc) return rc;
            }
        }
        // every part's chunks are queued before any wait: the parts run at once
        for (auto &ptp : parts) {
            BatchPart &pt = *ptp;
            int64_t pmax = 0;
            for (size_t jl = 0; jl < pt.members.size(); ++jl) {
                const int j = pt.members[jl];
                InstDesc d = lats[j]->desc();
                d.remaining = (uint32_t)counts[j];
                d.chunk = (uint32_t)S;
                d.count = (uint32_t)std::min<int64_t>(S, counts[j]);
                d.err = d_err;
                pt.h_desc[jl] = d;
                pmax = std::max(pmax, counts[j]);
            }
            if (pmax == 0) continue;
            HIPCHK(hipMemcpyAsync(pt.d_desc, pt.h_desc, pt.members.size() * sizeof(InstDesc), hipMemcpyHostToDevice,
                                  pt.stream));
            int rc = capture(pt, S);
            if (rc) return rc;
            const int64_t nchunks = (pmax + S - 1) / S;
            for (int64_t c = 0; c < nchunks; ++c) HIPCHK(hipGraphLaunch(pt.graph, pt.stream));
        }
        for (auto &ptp : parts) HIPCHK(hipStreamSynchronize(ptp->stream));
        for (size_t j = 0; j < lats.size(); ++j) {
            Lattice &l = *lats[j];
            if (counts[j] == 0) continue;
            l.sweep += counts[j];
            if (l.measure) l.rec_count += counts[j];
            l.labelled = l.sweep - 1;
        }
        return check_error_word(d_err);
    }
};

// ---------------------------------------------------------------------------
// Served form.
// ---------------------------------------------------------------------------
// Streams a server can deal each tick's groups to (it uses 4 unless told).
constexpr int SERVER_STREAMS = 8;

struct ServerJob {
    int64_t id;
    sw_job job;
    int64_t footprint;
    double submit_s = 0, start_s = 0, finish_s = 0;
    std::unique_ptr<Lattice> lat;
    int64_t done = 0;
    int status = 0;  // SW_E_NOCONV once a tick it took part in was flagged
};

struct sw_server_s {
    // first member: destroyed last, after every lattice has returned its blocks
    DevicePool pool;
    int64_t budget = 0, used = 0;
    int max_active = 1;
    int chunk = 32;
    int64_t next_id = 0;
    std::deque<std::unique_ptr<ServerJob>> queue;
    std::vector<std::unique_ptr<ServerJob>> active;
    std::vector<std::unique_ptr<ServerJob>> incoming;  // admitted while a tick ran; active from the next
    std::map<int64_t, sw_job_result> results;
    std::map<int64_t, std::vector<uint8_t>> final_state;
    // Each tick's groups are dealt to `nstreams` parts with a stream each, so
    // that the small launches of different groups run side by side; new jobs
    // are created on the admission stream while a tick runs.
    std::vector<hipStream_t> streams;
    hipStream_t admit_stream = nullptr;
    hipEvent_t desc_ready = nullptr;
    std::vector<int> group_part;  // part of each group
    int nparts = 4;               // streams in use (<= streams.size())
    // batched launch state for the current active set
    std::vector<Group> groups;
    InstDesc *d_desc = nullptr;
    InstDesc *h_desc = nullptr;
    uint32_t *d_err = nullptr;  // error word shared by every tick's launches
    int desc_cap = 0;
    bool dirty = true;

    ~sw_server_s()
    {
        for (hipStream_t st : streams) (void)hipStreamSynchronize(st);
        for (Group &g : groups) pool.put(g.d_tmap);
        if (d_desc) (void)hipFree(d_desc);
        if (h_desc) (void)hipHostFree(h_desc);
        if (d_err) (void)hipFree(d_err);
        active.clear();
        incoming.clear();
        queue.clear();
        if (desc_ready) (void)hipEventDestroy(desc_ready);
        for (hipStream_t st : streams) release_stream(st);
        if (admit_stream) release_stream(admit_stream);
    }

    int rebuild()
    {
        for (Group &g : groups) pool.put(g.d_tmap);
        groups.clear();
        if ((int)active.size() > desc_cap) {
            if (d_desc) (void)hipFree(d_desc);
            if (h_desc) (void)hipHostFree(h_desc);
            desc_cap = std::max<int>((int)active.size(), 2 * desc_cap);
            if (hipMalloc(&d_desc, (size_t)desc_cap * sizeof(InstDesc)) != hipSuccess ||
                hipHostMalloc(&h_desc, (size_t)desc_cap * sizeof(InstDesc), hipHostMallocDefault) != hipSuccess)
                return fail(SW_E_NOMEM, "descriptor allocation failed");
        }
        std::map<std::tuple<int, int, int>, int> index;
        for (int j = 0; j < (int)active.size(); ++j) {
            const Lattice &l = *active[j]->lat;
            auto key = std::make_tuple(l.model, l.dim, l.variant);
            if (!index.count(key)) {
                index[key] = (int)groups.size();
                groups.push_back(Group{l.model, l.dim, l.variant, {}, 0, 0, nullptr});
            }
            groups[index[key]].members.push_back(j);
        }
        std::vector<int64_t> gsites(groups.size(), 0);
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            Group &g = groups[gi];
            std::vector<int2> tm, cut;
            for (int j : g.members) {
                append_tiles(*active[j]->lat, j, tm, cut);
                gsites[gi] += active[j]->lat->N;
            }
            g.nfull = (int)tm.size();
            tm.insert(tm.end(), cut.begin(), cut.end());
            g.ntiles = (int)tm.size();
            void *tmv = nullptr;
            if (pool.get(&tmv, tm.size() * sizeof(int2)) != hipSuccess)
                return fail(SW_E_NOMEM, "tile map allocation failed");
            g.d_tmap = (int2 *)tmv;
            HIPCHK(hipMemcpy(g.d_tmap, tm.data(), tm.size() * sizeof(int2), hipMemcpyHostToDevice));
        }
        // groups to parts: largest first, each to the part with the fewest sites
        std::vector<int> order(groups.size());
        for (size_t gi = 0; gi < groups.size(); ++gi) order[gi] = (int)gi;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return gsites[x] > gsites[y]; });
        std::vector<int64_t> load((size_t)nparts, 0);
        group_part.assign(groups.size(), 0);
        for (int gi : order) {
            const int p = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            group_part[gi] = p;
            load[p] += gsites[gi];
        }
        dirty = false;
        return SW_OK;
    }

    // Results of jobs whose last sweep has run (their tick has completed).
    int retire(bool all_done_only)
    {
        (void)all_done_only;
        for (size_t j = 0; j < active.size();) {
            ServerJob &sj = *active[j];
            if (sj.done < sj.job.sweeps) {
                ++j;
                continue;
            }
            sw_job_result r;
            std::memset(&r, 0, sizeof(r));
            r.id = sj.id;
            r.sweeps = sj.done;
            r.submit_s = sj.submit_s;
            r.start_s = sj.start_s;
            r.finish_s = sj.finish_s;
            int rc = sj.lat->averages(&r.m2, &r.m4, &r.energy);
            r.status = sj.status ? sj.status : rc;
            std::vector<uint8_t> st((size_t)sj.lat->N * state_bytes(sj.lat->model));
            if (hipMemcpy(st.data(), sj.lat->state, st.size(), hipMemcpyDeviceToHost) != hipSuccess)
                r.status = SW_E_DEVICE;
            final_state[sj.id] = std::move(st);
            results[sj.id] = r;
            used -= sj.footprint;
            active.erase(active.begin() + j);
            dirty = true;
        }
        return SW_OK;
    }

    // Cancel job `id`. Between ticks no work of any job is in flight (a tick
    // ends with its streams synchronised and admission synchronises the new
    // lattice), so a queued job simply leaves the queue and a running one
    // leaves the active set at once, its budget freed. The result of a
    // running job keeps the sweeps it ran, their averages and its state.
    int cancel(int64_t id)
    {
        if (results.count(id)) return 1;
        sw_job_result r;
        std::memset(&r, 0, sizeof(r));
        r.id = id;
        r.status = SW_E_CANCELLED;
        for (auto it = queue.begin(); it != queue.end(); ++it) {
            if ((*it)->id != id) continue;
            r.submit_s = (*it)->submit_s;
            r.start_s = r.finish_s = now_s();
            results[id] = r;
            queue.erase(it);
            return SW_OK;
        }
        for (size_t j = 0; j < active.size(); ++j) {
            ServerJob &sj = *active[j];
            if (sj.id != id) continue;
            r.sweeps = sj.done;
            r.submit_s = sj.submit_s;
            r.start_s = sj.start_s;
            r.finish_s = now_s();
            if (sj.done > 0) {
                int rc = sj.lat->averages(&r.m2, &r.m4, &r.energy);
                if (rc) return rc;
            }
            std::vector<uint8_t> st((size_t)sj.lat->N * state_bytes(sj.lat->model));
            HIPCHK(hipMemcpy(st.data(), sj.lat->state, st.size(), hipMemcpyDeviceToHost));
            final_state[id] = std::move(st);
            results[id] = r;
            used -= sj.footprint;
            active.erase(active.begin() + j);
            dirty = true;
            return SW_OK;
        }
        return fail(SW_E_NOTFOUND, "unknown job id");
    }

    // Create the lattices of queued jobs that fit (on the admission stream).
    int admit(double t)
    {
        while (!queue.empty() && (int)(active.size() + incoming.size()) < max_active &&
               used + queue.front()->footprint <= budget) {
            std::unique_ptr<ServerJob> sj = std::move(queue.front());
            queue.pop_front();
            sj->lat.reset(new Lattice());
            sj->lat->pool = &pool;
            const sw_job_desc &jd = sj->job.lattice;
            int rc = sj->lat->create(jd.model, jd.dim, jd.L, jd.q, jd.beta, jd.seed, jd.replica,
                                     served_tile(jd.model, jd.dim, jd.L), admit_stream);
            if (rc == SW_OK) rc = sj->lat->grow_records(sj->job.sweeps);
            if (rc) {
                sw_job_result r;
                std::memset(&r, 0, sizeof(r));
                r.id = sj->id;
                r.status = rc;
                r.submit_s = sj->submit_s;
                r.start_s = r.finish_s = t;
                results[sj->id] = r;
                continue;
            }
            sj->start_s = t;
            used += sj->footprint;
            incoming.push_back(std::move(sj));
        }
        return SW_OK;
    }

    int64_t step()
    {
        int rc;
        bool launched = false;
        int64_t maxc = 0;
        if (!active.empty()) {
            if (dirty) {
                rc = rebuild();
                if (rc) return rc;
            }
            for (size_t j = 0; j < active.size(); ++j) {
                Lattice &l = *active[j]->lat;
                const int64_t c = std::min<int64_t>(chunk, active[j]->job.sweeps - active[j]->done);
                rc = l.grow_records(l.rec_count + c);
                if (rc) return rc;
                InstDesc d = l.desc();
                d.remaining = (uint32_t)c;
                d.chunk = (uint32_t)chunk;
                d.count = (uint32_t)c;
                d.err = d_err;
                h_desc[j] = d;
                maxc = std::max(maxc, c);
            }
            HIPCHK(hipMemcpyAsync(d_desc, h_desc, active.size() * sizeof(InstDesc), hipMemcpyHostToDevice,
                                  streams[0]));
            HIPCHK(hipEventRecord(desc_ready, streams[0]));
            for (int p = 1; p < nparts; ++p) HIPCHK(hipStreamWaitEvent(streams[p], desc_ready, 0));
            for (int p = 0; p < nparts; ++p) {
                hipStream_t st = streams[p];
                for (int64_t k = 0; k < maxc; ++k) {
                    for (size_t gi = 0; gi < groups.size(); ++gi) {
                        if (group_part[gi] != p) continue;
                        const Group &g = groups[gi];
                        HIPCHK(launch_bond(g.model, g.dim, g.variant, d_desc, g.d_tmap, g.ntiles, g.nfull, (uint32_t)k, 0, st));
                        HIPCHK(launch_merge(g.dim, g.model, g.variant, d_desc, g.d_tmap, g.ntiles, (uint32_t)k, st));
                    }
                }
                for (size_t gi = 0; gi < groups.size(); ++gi)
                    if (group_part[gi] == p) {
                        const Group &g = groups[gi];
                        HIPCHK(launch_flip(g.model, g.dim, g.variant, d_desc, g.d_tmap, g.ntiles, FLIP_LAST, st));
                    }
            }
            launched = true;
        }
        // while the tick runs: new jobs are created
        rc = admit(now_s());
        if (rc) return rc;
        if (launched) {
            for (int p = 0; p < nparts; ++p) HIPCHK(hipStreamSynchronize(streams[p]));
            const double t = now_s();
            // a flagged tick marks every job that took part in it
            const bool flagged = check_error_word(d_err) != SW_OK;
            for (size_t j = 0; j < active.size(); ++j) {
                ServerJob &sj = *active[j];
                const int64_t c = std::min<int64_t>(chunk, sj.job.sweeps - sj.done);
                sj.done += c;
                sj.lat->sweep += c;
                sj.lat->rec_count += c;
                if (c > 0) sj.lat->labelled = sj.lat->sweep - 1;
                if (c > 0 && flagged) sj.status = SW_E_NOCONV;
                if (c > 0 && sj.done == sj.job.sweeps) sj.finish_s = t;
            }
        }
        rc = retire(true);
        if (rc) return rc;
        if (!incoming.empty()) {
            for (auto &sj : incoming) {
                if (sj->job.sweeps == 0) sj->finish_s = now_s();
                active.push_back(std::move(sj));
            }
            incoming.clear();
            dirty = true;
            rc = retire(true);  // jobs of zero sweeps
            if (rc) return rc;
        }
        return (int64_t)(queue.size() + active.size());
    }
};

// ---------------------------------------------------------------------------
// C ABI.
// ---------------------------------------------------------------------------
extern "C" {

const char *sw_last_error(void) { return g_err.c_str(); }

sw_handle sw_create_tiled(int model, int dim, int L, int q, double beta, uint64_t seed, uint32_t replica,
                          int tile)
{
    g_err.clear();
    if (validate(model, dim, L, q, beta)) return nullptr;  // before any use of the shape tables
    if (tile < -1 || (tile >= 0 && tile >= num_tile_variants(model, dim))) {
        fail(SW_E_INVALID, "unknown tile shape");
        return nullptr;
    }
    if (tile < 0) tile = tuned_tile(model, dim, L);
    std::unique_ptr<sw_ctx> h(new sw_ctx());
    h->stream = make_stream();
    if (!h->stream) {
        fail(SW_E_DEVICE, "hipStreamCreate failed (no HIP device?)");
        return nullptr;
    }
    h->own_stream = true;
    h->lat = new Lattice();
    h->owned = true;
    int rc = h->lat->create(model, dim, L, q, beta, seed, replica, tile, h->stream);
    if (rc) {
        delete h->lat;
        release_stream(h->stream);
        h->lat = nullptr;
        return nullptr;
    }
    return h.release();
}

sw_handle sw_create_replica(int model, int dim, int L, int q, double beta, uint64_t seed, uint32_t replica)
{
    return sw_create_tiled(model, dim, L, q, beta, seed, replica, -1);
}

int sw_tile_count(int model, int dim)
{
    if (model < 0 || model > 3 || (dim != 2 && dim != 3)) return fail(SW_E_INVALID, "bad model or dim");
    return num_tile_variants(model, dim);
}

int sw_tile_shape(int model, int dim, int tile, int *tx, int *ty, int *tz)
{
    if (model < 0 || model > 3 || (dim != 2 && dim != 3)) return fail(SW_E_INVALID, "bad model or dim");
    if (tile < 0 || tile >= num_tile_variants(model, dim)) return fail(SW_E_INVALID, "unknown tile shape");
    const TileShape t = tile_shape(model, dim, tile);
    if (tx) *tx = t.tx;
    if (ty) *ty = t.ty;
    if (tz) *tz = dim == 3 ? t.tz : 1;
    return SW_OK;
}

int sw_get_tile(sw_handle h)
{
    if (!h || !h->lat) return fail(SW_E_INVALID, "NULL handle");
    return h->lat->variant;
}

int sw_tune(int model, int dim, int L, int q, double beta, int sweeps, int *best, double *ms_per_sweep)
{
    g_err.clear();
    if (sweeps < 1 || sweeps > 100000) return fail(SW_E_INVALID, "sweeps must be in [1, 100000]");
    int rc = validate(model, dim, L, model == ISING ? 2 : q, beta);
    if (rc) return rc;
    hipStream_t st = make_stream();
    if (!st) return fail(SW_E_DEVICE, "hipStreamCreate failed (no HIP device?)");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        release_stream(st);
        return fail(SW_E_DEVICE, "hipEventCreate failed");
    }
    const int nv = num_tile_variants(model, dim);
    int arg = 0;
    double tbest = 0.0;
    for (int v = 0; v < nv && rc == SW_OK; ++v) {
        Lattice lat;
        rc = lat.create(model, dim, L, q, beta, 0x7e57ull + (uint64_t)v, 0, v, st);
        if (rc == SW_OK) rc = lat.sweep_solo(2);
        if (rc != SW_OK) break;
        float ms = 0.0f;
        if (hipEventRecord(e0, st) != hipSuccess) rc = fail(SW_E_DEVICE, "hipEventRecord failed");
        if (rc == SW_OK) rc = lat.sweep_solo(sweeps);
        if (rc == SW_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            rc = fail(SW_E_DEVICE, "event timing failed");
        if (rc != SW_OK) break;
        const double per = (double)ms / sweeps;
        if (ms_per_sweep) ms_per_sweep[v] = per;
        if (v == 0 || per < tbest) {
            tbest = per;
            arg = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    release_stream(st);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[std::make_tuple(model, dim, L)] = arg;
    }
    if (best) *best = arg;
    return SW_OK;
}

sw_handle sw_create(int model, int dim, int L, int q, double beta, uint64_t seed)
{
    return sw_create_replica(model, dim, L, q, beta, seed, 0);
}

void sw_destroy(sw_handle h)
{
    if (!h) return;
    if (h->owned) {
        delete h->lat;
        if (h->own_stream && h->stream) release_stream(h->stream);
        delete h;
    }
}

#define CHECK_H(h)                                                   \
    do {                                                             \
        if (!(h) || !(h)->lat) return fail(SW_E_INVALID, "NULL handle"); \
    } while (0)

int sw_sweep(sw_handle h, int64_t n)
{
    CHECK_H(h);
    if (n < 0) return fail(SW_E_INVALID, "negative sweep count");
    return h->lat->sweep_solo(n);
}

int sw_measure(sw_handle h, double *m2, double *m4, double *energy, sw_cluster_stats *cs)
{
    CHECK_H(h);
    int rc = h->lat->averages(m2, m4, energy);
    if (rc) return rc;
    if (cs) return h->lat->cluster_stats(cs);
    return SW_OK;
}

int sw_get_moments(sw_handle h, sw_moments *out)
{
    CHECK_H(h);
    if (!out) return fail(SW_E_INVALID, "NULL output");
    return h->lat->moments(out);
}

int sw_cluster_stats_noalloc(sw_handle h, sw_cluster_stats *cs)
{
    CHECK_H(h);
    if (!cs) return fail(SW_E_INVALID, "NULL output");
    Lattice &l = *h->lat;
    std::memset(cs, 0, sizeof(*cs));
    if (l.N > STATIC_STATS_SITES)
        return fail(SW_E_INVALID, "lattice has " + std::to_string(l.N) + " sites; the allocation-free cluster "
                    "statistics hold at most " + std::to_string(STATIC_STATS_SITES));
    if (l.labelled < 0) return SW_OK;
    // its sweep index names the last labelled sweep's buffer
    InstDesc d = l.labelled_desc();
    HIPCHK(hipMemcpyAsync(l.d_solo, &d, sizeof(d), hipMemcpyHostToDevice, l.stream));
    unsigned long long out[3] = {0, 0, 0};
    HIPCHK(cluster_stats_static(l.d_solo, 0, l.N, out, l.stream));
    cs->n_clusters = (int64_t)out[0];
    cs->max_cluster = (int64_t)out[1];
    cs->sum_c2 = (int64_t)out[2];
    return l.check_errors();
}

int sw_set_labeller(sw_handle h, int algorithm, int max_iterations)
{
    CHECK_H(h);
    return h->lat->set_labeller(algorithm, max_iterations);
}

int sw_get_label_stats(sw_handle h, int64_t *labellings, int64_t *scans, int64_t *max_scans)
{
    CHECK_H(h);
    uint64_t v[3];
    HIPCHK(hipMemcpy(v, (char *)h->lat->err + 64, sizeof(v), hipMemcpyDeviceToHost));
    if (labellings) *labellings = (int64_t)v[0];
    if (scans) *scans = (int64_t)v[1];
    if (max_scans) *max_scans = (int64_t)v[2];
    return SW_OK;
}

int sw_set_walk_cap(sw_handle h, int64_t cap)
{
    CHECK_H(h);
    if (cap < 1 || cap > 0xFFFFFFFFll) return fail(SW_E_INVALID, "walk cap must be in [1, 2^32 - 1]");
    h->lat->walk_cap = (uint32_t)cap;
    return SW_OK;
}

int sw_reset_measure(sw_handle h)
{
    CHECK_H(h);
    h->lat->rec_count = 0;
    return SW_OK;
}

int64_t sw_series(sw_handle h, sw_record *out, int64_t max)
{
    CHECK_H(h);
    if (max < 0 || (max > 0 && !out)) return fail(SW_E_INVALID, "bad output buffer");
    std::vector<sw_record> v;
    int rc = h->lat->series(v, max);
    if (rc) return rc;
    if (!v.empty()) std::memcpy(out, v.data(), v.size() * sizeof(sw_record));
    return (int64_t)v.size();
}

int sw_set_measure(sw_handle h, int on)
{
    CHECK_H(h);
    h->lat->measure = on != 0;
    if (!h->lat->measure) h->lat->rec_count = 0;
    return SW_OK;
}

int sw_profile(sw_handle h, int on)
{
    CHECK_H(h);
    if (on < 0 || on > 2) return fail(SW_E_INVALID, "profiling level must be 0, 1 or 2");
    h->lat->profiling = on;
    if (on)
        for (int c = 0; c < 3; ++c) {
            h->lat->prof_ms[c] = 0.0;
            h->lat->prof_n[c] = 0;
        }
    return SW_OK;
}

int sw_profile_read(sw_handle h, double *ms, int64_t *launches)
{
    CHECK_H(h);
    for (int c = 0; c < 3; ++c) {
        if (ms) ms[c] = h->lat->prof_ms[c];
        if (launches) launches[c] = h->lat->prof_n[c];
    }
    return SW_OK;
}

int64_t sw_sweep_index(sw_handle h)
{
    CHECK_H(h);
    return h->lat->sweep;
}

int sw_set_sweep_index(sw_handle h, int64_t n)
{
    CHECK_H(h);
    if (n < 0 || n > 0xFFFFFFFFll) return fail(SW_E_INVALID, "sweep index out of range");
    h->lat->sweep = n;
    h->lat->rec_count = 0;
    return SW_OK;
}

int sw_get_state(sw_handle h, void *host)
{
    CHECK_H(h);
    if (!host) return fail(SW_E_INVALID, "NULL buffer");
    Lattice &l = *h->lat;
    HIPCHK(hipMemcpy(host, l.state, (size_t)l.N * state_bytes(l.model), hipMemcpyDeviceToHost));
    return SW_OK;
}

int sw_set_state(sw_handle h, const void *host)
{
    CHECK_H(h);
    if (!host) return fail(SW_E_INVALID, "NULL buffer");
    Lattice &l = *h->lat;
    if (l.model == ISING) {
        const int8_t *s = (const int8_t *)host;
        for (int64_t i = 0; i < l.N; ++i)
            if (s[i] != 1 && s[i] != -1) return fail(SW_E_INVALID, "Ising states must be +1 or -1");
    } else if (l.model == POTTS) {
        const uint8_t *s = (const uint8_t *)host;
        for (int64_t i = 0; i < l.N; ++i)
            if (s[i] >= l.q) return fail(SW_E_INVALID, "Potts states must be < q");
    } else if (l.model == CLOCK) {
        const uint16_t *s = (const uint16_t *)host;
        for (int64_t i = 0; i < l.N; ++i)
            if (s[i] >= l.q) return fail(SW_E_INVALID, "clock states must be < q");
    } else {
        const float *s = (const float *)host;
        const float top = (float)6.283185307179586476925286766559;
        for (int64_t i = 0; i < l.N; ++i)
            if (!(s[i] >= 0.0f && s[i] < top)) return fail(SW_E_INVALID, "XY angles must be in [0, 2pi)");
    }
    HIPCHK(hipMemcpy(l.state, host, (size_t)l.N * state_bytes(l.model), hipMemcpyHostToDevice));
    return SW_OK;
}

int sw_get_labels(sw_handle h, int32_t *host)
{
    CHECK_H(h);
    if (!host) return fail(SW_E_INVALID, "NULL buffer");
    Lattice &l = *h->lat;
    if (l.labelled < 0) {
        for (int64_t i = 0; i < l.N; ++i) host[i] = (int32_t)i;
        return SW_OK;
    }
    int32_t *tmp = nullptr;
    if (hipMalloc(&tmp, (size_t)l.N * 4) != hipSuccess) return fail(SW_E_NOMEM, "label scratch allocation failed");
    InstDesc d = l.labelled_desc();
    hipError_t e = hipMemcpyAsync(l.d_solo, &d, sizeof(d), hipMemcpyHostToDevice, l.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(l.stream);
    if (e == hipSuccess) e = launch_canon(l.d_solo, 0, l.N, tmp, l.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(host, tmp, (size_t)l.N * 4, hipMemcpyDeviceToHost, l.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(l.stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return fail(SW_E_DEVICE, std::string("labels: ") + hipGetErrorString(e));
    return l.check_errors();
}

int sw_get_bonds(sw_handle h, uint8_t *host)
{
    CHECK_H(h);
    if (!host) return fail(SW_E_INVALID, "NULL buffer");
    Lattice &l = *h->lat;
    HIPCHK(hipMemcpy(host, l.bond, (size_t)l.N, hipMemcpyDeviceToHost));
    return SW_OK;
}

int sw_info(sw_handle h, int *model, int *dim, int *L, int *q, double *beta, uint64_t *seed, uint32_t *replica)
{
    CHECK_H(h);
    const Lattice &l = *h->lat;
    if (model) *model = l.model;
    if (dim) *dim = l.dim;
    if (L) *L = l.L;
    if (q) *q = l.q;
    if (beta) *beta = l.beta;
    if (seed) *seed = l.seed;
    if (replica) *replica = l.rep;
    return SW_OK;
}

sw_batch sw_batch_create(const sw_job_desc *jobs, int n)
{
    g_err.clear();
    if (!jobs || n < 1) {
        fail(SW_E_INVALID, "need at least one job");
        return nullptr;
    }
    std::unique_ptr<sw_batch_s> b(new sw_batch_s());
    b->stream = make_stream();
    if (!b->stream) {
        fail(SW_E_DEVICE, "hipStreamCreate failed (no HIP device?)");
        return nullptr;
    }
    for (int j = 0; j < n; ++j) {
        std::unique_ptr<Lattice> l(new Lattice());
        int rc = l->create(jobs[j].model, jobs[j].dim, jobs[j].L, jobs[j].q, jobs[j].beta, jobs[j].seed,
                           jobs[j].replica, tuned_tile(jobs[j].model, jobs[j].dim, jobs[j].L), b->stream);
        if (rc) return nullptr;
        std::unique_ptr<sw_ctx> v(new sw_ctx());
        v->lat = l.get();
        v->owned = false;
        v->stream = b->stream;
        b->views.push_back(std::move(v));
        b->lats.push_back(std::move(l));
    }
    if (b->build_parts(n >= 2 ? 2 : 1)) return nullptr;
    return b.release();
}

int sw_batch_sweep(sw_batch b, int64_t n)
{
    if (!b) return fail(SW_E_INVALID, "NULL batch");
    if (n < 0) return fail(SW_E_INVALID, "negative sweep count");
    std::vector<int64_t> c(b->lats.size(), n);
    return b->sweep_counts(c.data());
}

int sw_batch_sweep_counts(sw_batch b, const int64_t *counts)
{
    if (!b || !counts) return fail(SW_E_INVALID, "NULL argument");
    return b->sweep_counts(counts);
}

int sw_batch_size(sw_batch b) { return b ? (int)b->lats.size() : 0; }

sw_handle sw_batch_member(sw_batch b, int j)
{
    if (!b || j < 0 || j >= (int)b->lats.size()) {
        fail(SW_E_INVALID, "member index out of range");
        return nullptr;
    }
    return b->views[j].get();
}

int sw_batch_set_chunk(sw_batch b, int s)
{
    if (!b || s < 1 || s > 4096) return fail(SW_E_INVALID, "chunk must be in [1, 4096]");
    b->chunk = s;
    return SW_OK;
}

int sw_batch_set_streams(sw_batch b, int n)
{
    if (!b || n < 1 || n > 8) return fail(SW_E_INVALID, "streams must be in [1, 8]");
    return b->build_parts(n);
}

void sw_batch_destroy(sw_batch b) { delete b; }

int64_t sw_footprint(int model, int dim, int L, int q)
{
    if (validate(model, dim, L, (model == ISING) ? 2 : q, 0.0)) return SW_E_INVALID;
    return Lattice::footprint(model, dim, L, (model == ISING) ? 2 : (model == XY ? 0 : q), 0);  // Potts, clock: q
}

sw_server sw_server_create(int64_t budget, int max_active, int chunk)
{
    g_err.clear();
    if (budget <= 0 || max_active < 1 || chunk < 1) {
        fail(SW_E_INVALID, "budget, max_active and chunk must be positive");
        return nullptr;
    }
    std::unique_ptr<sw_server_s> s(new sw_server_s());
    s->budget = budget;
    s->max_active = max_active;
    s->chunk = chunk;
    s->pool.cap = (size_t)std::min<int64_t>(budget / 4, (int64_t)4 << 30);
    for (int p = 0; p < SERVER_STREAMS; ++p) {
        hipStream_t st = make_stream();
        if (!st) {
            fail(SW_E_DEVICE, "hipStreamCreate failed (no HIP device?)");
            return nullptr;
        }
        s->streams.push_back(st);
    }
    s->admit_stream = make_stream();
    if (!s->admit_stream || hipEventCreateWithFlags(&s->desc_ready, hipEventDisableTiming) != hipSuccess) {
        fail(SW_E_DEVICE, "hipStreamCreate / hipEventCreate failed");
        return nullptr;
    }
    if (hipMalloc(&s->d_err, 256) != hipSuccess || hipMemset(s->d_err, 0, 256) != hipSuccess) {
        fail(SW_E_NOMEM, "server error word allocation failed");
        return nullptr;
    }
    return s.release();
}

int64_t sw_server_submit(sw_server s, const sw_job *job)
{
    if (!s || !job) return fail(SW_E_INVALID, "NULL argument");
    const sw_job_desc &jd = job->lattice;
    int rc = validate(jd.model, jd.dim, jd.L, jd.model == ISING ? 2 : jd.q, jd.beta);
    if (rc) return rc;
    if (job->sweeps < 0 || job->sweeps >= (1ll << 31)) return fail(SW_E_INVALID, "bad sweep count");
    const int64_t fp = sw_footprint(jd.model, jd.dim, jd.L, jd.q);
    if (fp > s->budget) return fail(SW_E_INVALID, "job footprint exceeds the HBM budget");
    std::unique_ptr<ServerJob> sj(new ServerJob());
    sj->id = s->next_id++;
    sj->job = *job;
    sj->footprint = fp;
    sj->submit_s = now_s();
    const int64_t id = sj->id;
    s->queue.push_back(std::move(sj));
    return id;
}

int64_t sw_server_step(sw_server s)
{
    if (!s) return fail(SW_E_INVALID, "NULL server");
    return s->step();
}

int sw_server_poll(sw_server s, int64_t id, sw_job_result *out, void *state)
{
    if (!s) return fail(SW_E_INVALID, "NULL server");
    auto it = s->results.find(id);
    if (it == s->results.end()) {
        if (id >= 0 && id < s->next_id) return 1;
        return fail(SW_E_NOTFOUND, "unknown job id");
    }
    if (out) *out = it->second;
    if (state) {
        auto st = s->final_state.find(id);
        if (st != s->final_state.end()) std::memcpy(state, st->second.data(), st->second.size());
    }
    return SW_OK;
}

int sw_server_cancel(sw_server s, int64_t id)
{
    if (!s) return fail(SW_E_INVALID, "NULL server");
    return s->cancel(id);
}

int sw_server_set_streams(sw_server s, int n)
{
    if (!s || n < 1 || n > SERVER_STREAMS) return fail(SW_E_INVALID, "streams must be in [1, 8]");
    for (hipStream_t st : s->streams) HIPCHK(hipStreamSynchronize(st));
    s->nparts = n;
    s->dirty = true;
    return SW_OK;
}

void sw_server_destroy(sw_server s) { delete s; }

}  // extern "C"
