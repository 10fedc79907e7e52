"""MI355X Swendsen-Wang engine: Python binding of libswmc.so (include/sw.h).

Argument marshalling only -- every step of a sweep runs in the library's HIP
kernels.  The library must be built (`python -m paper_1403_7560_amd.build`);
importing this module without it raises, there is no fallback path.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libswmc.so")

ISING, POTTS, XY, CLOCK = 0, 1, 2, 3
LABEL_HAWICK, LABEL_KALENTEV, LABEL_UNION = 0, 1, 2
STATE_DTYPE = {ISING: np.int8, POTTS: np.uint8, XY: np.float32, CLOCK: np.uint16}
ERRORS = {-1: "SW_E_INVALID", -2: "SW_E_NOMEM", -3: "SW_E_DEVICE", -4: "SW_E_NOCONV",
          -5: "SW_E_BUSY", -6: "SW_E_NOTFOUND", -7: "SW_E_CANCELLED"}


class SWError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class ClusterStats(ctypes.Structure):
    _fields_ = [("n_clusters", ctypes.c_int64), ("max_cluster", ctypes.c_int64),
                ("sum_c2", ctypes.c_int64)]


class Moments(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("abs_m", ctypes.c_double), ("m2", ctypes.c_double),
                ("m4", ctypes.c_double), ("energy", ctypes.c_double), ("energy2", ctypes.c_double),
                ("specific_heat", ctypes.c_double), ("binder", ctypes.c_double)]


class Record(ctypes.Structure):
    _fields_ = [("sweep", ctypes.c_int64), ("energy", ctypes.c_double), ("mag", ctypes.c_double),
                ("mag2", ctypes.c_double), ("mx", ctypes.c_double), ("my", ctypes.c_double)]


RECORD_DTYPE = np.dtype([("sweep", np.int64), ("energy", np.float64), ("mag", np.float64),
                         ("mag2", np.float64), ("mx", np.float64), ("my", np.float64)])
assert RECORD_DTYPE.itemsize == ctypes.sizeof(Record)


class JobDesc(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int), ("dim", ctypes.c_int), ("L", ctypes.c_int),
                ("q", ctypes.c_int), ("beta", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("replica", ctypes.c_uint32)]


class Job(ctypes.Structure):
    _fields_ = [("lattice", JobDesc), ("sweeps", ctypes.c_int64)]


class JobResult(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int), ("sweeps", ctypes.c_int64),
                ("submit_s", ctypes.c_double), ("start_s", ctypes.c_double),
                ("finish_s", ctypes.c_double), ("m2", ctypes.c_double), ("m4", ctypes.c_double),
                ("energy", ctypes.c_double)]


# C ABI: name -> (restype, argtypes).  Every symbol include/sw.h declares.
vp, i32, i64, u32, u64, dbl = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint32,
                               ctypes.c_uint64, ctypes.c_double)
SIGNATURES = {
    "sw_create": (vp, [i32, i32, i32, i32, dbl, u64]),
    "sw_create_replica": (vp, [i32, i32, i32, i32, dbl, u64, u32]),
    "sw_create_tiled": (vp, [i32, i32, i32, i32, dbl, u64, u32, i32]),
    "sw_tile_count": (i32, [i32, i32]),
    "sw_tile_shape": (i32, [i32, i32, i32, vp, vp, vp]),
    "sw_get_tile": (i32, [vp]),
    "sw_tune": (i32, [i32, i32, i32, i32, dbl, i32, vp, vp]),
    "sw_sweep": (i32, [vp, i64]),
    "sw_measure": (i32, [vp, vp, vp, vp, vp]),
    "sw_reset_measure": (i32, [vp]),
    "sw_get_moments": (i32, [vp, vp]),
    "sw_set_walk_cap": (i32, [vp, i64]),
    "sw_set_labeller": (i32, [vp, i32, i32]),
    "sw_cluster_stats_noalloc": (i32, [vp, vp]),
    "sw_get_label_stats": (i32, [vp, vp, vp, vp]),
    "sw_series": (i64, [vp, vp, i64]),
    "sw_set_measure": (i32, [vp, i32]),
    "sw_destroy": (None, [vp]),
    "sw_last_error": (ctypes.c_char_p, []),
    "sw_profile": (i32, [vp, i32]),
    "sw_profile_read": (i32, [vp, vp, vp]),
    "sw_sweep_index": (i64, [vp]),
    "sw_set_sweep_index": (i32, [vp, i64]),
    "sw_get_state": (i32, [vp, vp]),
    "sw_set_state": (i32, [vp, vp]),
    "sw_get_labels": (i32, [vp, vp]),
    "sw_get_bonds": (i32, [vp, vp]),
    "sw_info": (i32, [vp, vp, vp, vp, vp, vp, vp, vp]),
    "sw_batch_create": (vp, [vp, i32]),
    "sw_batch_sweep": (i32, [vp, i64]),
    "sw_batch_sweep_counts": (i32, [vp, vp]),
    "sw_batch_size": (i32, [vp]),
    "sw_batch_member": (vp, [vp, i32]),
    "sw_batch_set_chunk": (i32, [vp, i32]),
    "sw_batch_set_streams": (i32, [vp, i32]),
    "sw_batch_destroy": (None, [vp]),
    "sw_server_create": (vp, [i64, i32, i32]),
    "sw_server_submit": (i64, [vp, vp]),
    "sw_server_step": (i64, [vp]),
    "sw_server_poll": (i32, [vp, i64, vp, vp]),
    "sw_server_cancel": (i32, [vp, i64]),
    "sw_footprint": (i64, [i32, i32, i32, i32]),
    "sw_server_set_streams": (i32, [vp, i32]),
    "sw_server_destroy": (None, [vp]),
}

_lib = None


def lib():
    """The loaded libswmc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1403_7560_amd.build` (no fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error():
    return lib().sw_last_error().decode()


def _check(rc):
    if rc < 0:
        raise SWError(int(rc), last_error())
    return rc


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def nsites(dim, L):
    return L ** dim


class Lattice:
    """One lattice (plain form).  Mirrors sw_create_replica / sw_* calls."""

    def __init__(self, model, dim, L, q=2, beta=0.0, seed=0, replica=0, tile=None, _handle=None):
        self.model, self.dim, self.L = model, dim, L
        self.q = 2 if model == ISING else (0 if model == XY else q)
        self.N = L ** dim
        self._owned = _handle is None
        if _handle is None:
            if tile is None:
                h = lib().sw_create_replica(model, dim, L, self.q, float(beta), seed, replica)
            else:
                h = lib().sw_create_tiled(model, dim, L, self.q, float(beta), seed, replica, int(tile))
            if not h:
                raise SWError(-1, last_error())
            self.h = h
        else:
            self.h = _handle

    def close(self):
        if self._owned and self.h:
            lib().sw_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def face_elements(self):
        """Tile-face slots the global labelling phase reads per side (host
        arithmetic on the tile shape)."""
        ext = tile_shape(self.model, self.dim, self.tile)[:self.dim]
        tiles = [-(-self.L // e) for e in ext]
        nt = 1
        for t in tiles:
            nt *= t
        T = 1
        for e in ext:
            T *= e
        return sum(nt * (T // ext[mu]) for mu in range(self.dim) if tiles[mu] > 1)

    @property
    def tile(self):
        """Index of the tile shape this lattice runs with."""
        return _check(lib().sw_get_tile(self.h))

    def sweep(self, n):
        _check(lib().sw_sweep(self.h, int(n)))

    def measure(self):
        m2, m4, e = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        cs = ClusterStats()
        _check(lib().sw_measure(self.h, ctypes.byref(m2), ctypes.byref(m4), ctypes.byref(e),
                                ctypes.byref(cs)))
        return {"m2": m2.value, "m4": m4.value, "energy": e.value,
                "n_clusters": cs.n_clusters, "max_cluster": cs.max_cluster, "sum_c2": cs.sum_c2}

    def moments(self):
        """<|m|>, <m^2>, <m^4>, <E>/N, <(E/N)^2>, specific heat per spin and
        the moment ratio over the recorded series (sw_get_moments)."""
        m = Moments()
        _check(lib().sw_get_moments(self.h, ctypes.byref(m)))
        return {f: getattr(m, f) for f, _ in Moments._fields_}

    def set_labeller(self, algorithm, max_iterations=64):
        """0 Hawick, 1 Kalentev (the paper's iterative labellers), 2 one-pass union."""
        _check(lib().sw_set_labeller(self.h, int(algorithm), int(max_iterations)))

    def label_stats(self):
        v = np.zeros(3, dtype=np.int64)
        _check(lib().sw_get_label_stats(self.h, _ptr(v[0:]), _ptr(v[1:]), _ptr(v[2:])))
        return {"labellings": int(v[0]), "scans": int(v[1]), "max_scans": int(v[2])}

    def set_walk_cap(self, cap):
        _check(lib().sw_set_walk_cap(self.h, int(cap)))

    def cluster_stats_noalloc(self):
        """Cluster statistics of the last labelling through the allocation-free
        entry point (sw_cluster_stats_noalloc)."""
        cs = ClusterStats()
        _check(lib().sw_cluster_stats_noalloc(self.h, ctypes.byref(cs)))
        return {"n_clusters": cs.n_clusters, "max_cluster": cs.max_cluster, "sum_c2": cs.sum_c2}

    def reset_measure(self):
        _check(lib().sw_reset_measure(self.h))

    def set_measure(self, on):
        _check(lib().sw_set_measure(self.h, 1 if on else 0))

    def series(self, max_records=None):
        """The recorded series, oldest first (at most max_records): a dict of
        arrays sweep, energy, mag, mag2, mx, my."""
        limit = max_records if max_records is not None else 1 << 40
        cap = min(limit, 1024)
        while True:  # a buffer that grows until the whole series fits
            buf = (Record * cap)()
            got = _check(lib().sw_series(self.h, buf, cap))
            if got < cap or cap >= limit:
                break
            cap = min(limit, cap * 8)
        a = np.frombuffer(buf, dtype=RECORD_DTYPE, count=got)
        return {k: a[k].copy() for k in RECORD_DTYPE.names}

    def profile(self, level):
        """0 off; 1 time the bond kernel of every 16th sweep; 2 also its merge."""
        _check(lib().sw_profile(self.h, int(level)))

    def profile_read(self):
        ms = np.zeros(3)
        n = np.zeros(3, dtype=np.int64)
        _check(lib().sw_profile_read(self.h, _ptr(ms), _ptr(n)))
        return {"bond": (ms[0], n[0]), "merge": (ms[1], n[1]), "flip": (ms[2], n[2])}

    def sweep_index(self):
        return _check(lib().sw_sweep_index(self.h))

    def set_sweep_index(self, n):
        _check(lib().sw_set_sweep_index(self.h, int(n)))

    def get_state(self):
        s = np.empty(self.N, dtype=STATE_DTYPE[self.model])
        _check(lib().sw_get_state(self.h, _ptr(s)))
        return s

    def set_state(self, s):
        s = np.ascontiguousarray(s, dtype=STATE_DTYPE[self.model])
        assert s.size == self.N
        _check(lib().sw_set_state(self.h, _ptr(s)))

    def get_labels(self):
        lab = np.empty(self.N, dtype=np.int32)
        _check(lib().sw_get_labels(self.h, _ptr(lab)))
        return lab

    def get_bonds(self):
        b = np.empty(self.N, dtype=np.uint8)
        _check(lib().sw_get_bonds(self.h, _ptr(b)))
        return b


class Batch:
    """Many lattices sweeping in shared launches (sw_batch_*)."""

    def __init__(self, jobs):
        arr = (JobDesc * len(jobs))()
        for i, j in enumerate(jobs):
            model = j["model"]
            q = 2 if model == ISING else (0 if model == XY else j.get("q", 2))
            arr[i] = JobDesc(model, j["dim"], j["L"], q, float(j.get("beta", 0.0)),
                             j.get("seed", 0), j.get("replica", 0))
        h = lib().sw_batch_create(arr, len(jobs))
        if not h:
            raise SWError(-1, last_error())
        self.h = h
        self.members = []
        for i, j in enumerate(jobs):
            mh = lib().sw_batch_member(h, i)
            self.members.append(Lattice(j["model"], j["dim"], j["L"], j.get("q", 2), _handle=mh))

    def sweep(self, n):
        _check(lib().sw_batch_sweep(self.h, int(n)))

    def sweep_counts(self, counts):
        c = np.ascontiguousarray(counts, dtype=np.int64)
        assert c.size == len(self.members)
        _check(lib().sw_batch_sweep_counts(self.h, _ptr(c)))

    def set_chunk(self, s):
        _check(lib().sw_batch_set_chunk(self.h, int(s)))

    def set_streams(self, n):
        _check(lib().sw_batch_set_streams(self.h, int(n)))

    def close(self):
        if self.h:
            for m in self.members:
                m.h = None
            lib().sw_batch_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def footprint(model, dim, L, q=2):
    return _check(lib().sw_footprint(model, dim, L, q))


class Server:
    """Continuous-batching job server (sw_server_*)."""

    def __init__(self, hbm_budget_bytes, max_active=64, chunk=32):
        h = lib().sw_server_create(int(hbm_budget_bytes), int(max_active), int(chunk))
        if not h:
            raise SWError(-1, last_error())
        self.h = h

    def submit(self, model, dim, L, q=2, beta=0.0, seed=0, replica=0, sweeps=0):
        qq = 2 if model == ISING else (0 if model == XY else q)
        job = Job(JobDesc(model, dim, L, qq, float(beta), seed, replica), int(sweeps))
        return _check(lib().sw_server_submit(self.h, ctypes.byref(job)))

    def step(self):
        return _check(lib().sw_server_step(self.h))

    def set_streams(self, n):
        _check(lib().sw_server_set_streams(self.h, int(n)))

    def cancel(self, job_id):
        """True when the job was cancelled, False if it had already finished."""
        return _check(lib().sw_server_cancel(self.h, int(job_id))) == 0

    def poll(self, job_id, model=None, N=None):
        r = JobResult()
        state = None
        if model is not None:
            state = np.empty(N, dtype=STATE_DTYPE[model])
        rc = _check(lib().sw_server_poll(self.h, int(job_id), ctypes.byref(r),
                                         _ptr(state) if state is not None else None))
        if rc == 1:
            return None
        out = {f: getattr(r, f) for f, _ in JobResult._fields_}
        if state is not None:
            out["state"] = state
        return out

    def close(self):
        if self.h:
            lib().sw_server_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tile_count(model, dim):
    return _check(lib().sw_tile_count(model, dim))


def tile_shape(model, dim, tile):
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().sw_tile_shape(model, dim, tile, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def tune(model, dim, L, q=2, beta=0.0, sweeps=20):
    """Time every tile shape on a scratch lattice; the fastest becomes the
    shape of lattices created afterwards for (model, dim, L).  Returns
    (best, ms per sweep of each shape)."""
    q = 2 if model == ISING else (0 if model == XY else q)
    n = tile_count(model, dim)
    best = ctypes.c_int()
    ms = (ctypes.c_double * n)()
    _check(lib().sw_tune(model, dim, L, q, float(beta), int(sweeps), ctypes.byref(best), ms))
    return best.value, list(ms)
