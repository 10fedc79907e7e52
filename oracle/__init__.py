"""CPU oracle of the Swendsen-Wang sweep (ctypes front end of sw_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark; never by the product package.  The C
source states the paper passages each step follows and the readings taken
where the paper is silent.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsworacle.so")
SRC = os.path.join(HERE, "sw_oracle.c")

ISING, POTTS, XY, CLOCK = 0, 1, 2, 3
TAG_BOND, TAG_BOND_Z, TAG_BOND_TIE, TAG_CLUSTER, TAG_GLOBAL, TAG_INIT = range(6)
STATE_DTYPE = {ISING: np.int8, POTTS: np.uint8, XY: np.float32, CLOCK: np.uint16}


def build(force=True):
    """Compile the oracle with gcc (no FMA contraction, so the XY arithmetic is
    evaluated exactly in the order written)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-o", LIB_PATH, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u32, u64, dbl = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                                       ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double)
        L.swo_philox4x32_10.argtypes = [vp, vp, vp]
        L.swo_word.argtypes = [u64, u32, u32, u32, u64]
        L.swo_word.restype = u32
        L.swo_bond_uniform.argtypes = [u64, u32, u32, i32, i32, u64, i32]
        L.swo_bond_uniform.restype = u32
        L.swo_cluster_decision.argtypes = [i32, i32, u64, u32, u32, i32, i32, u64]
        L.swo_cluster_decision.restype = u32
        L.swo_threshold.argtypes = [i32, dbl]
        L.swo_threshold.restype = u64
        L.swo_init_state.argtypes = [i32, i32, i32, i32, u64, u32, vp]
        L.swo_xy_phi.argtypes = [u64, u32, u32]
        L.swo_xy_phi.restype = dbl
        L.swo_bonds.argtypes = [i32, i32, i32, i32, dbl, u64, u32, u32, vp, vp]
        L.swo_bonds.restype = i64
        L.swo_labels_uf.argtypes = [i32, i32, vp, vp]
        L.swo_labels_bfs.argtypes = [i32, i32, vp, vp]
        L.swo_set_clusters.argtypes = [i32, i32, i32, i32, u64, u32, u32, vp, vp]
        L.swo_measure.argtypes = [i32, i32, i32, i32, vp, vp, vp, vp, vp, vp]
        L.swo_cluster_stats.argtypes = [i64, vp, vp]
        L.swo_clock_axis.argtypes = [u64, u32, u32, i32]
        L.swo_clock_axis.restype = u32
        L.swo_clock_projection.argtypes = [i32, u32, u32, vp, vp]
        L.swo_clock_threshold.argtypes = [i32, dbl, i32, i32]
        L.swo_clock_threshold.restype = u64
        L.swo_clock_mirror.argtypes = [i32, u32, u32]
        L.swo_clock_mirror.restype = ctypes.c_uint16
        L.swo_sweeps.argtypes = [i32, i32, i32, i32, dbl, u64, u32, u32, i64, vp,
                                 vp, vp, vp, vp, vp, vp, vp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().swo_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def word(seed, rep, tag, sweep, w):
    return int(lib().swo_word(seed, rep, tag, sweep, w))


def bond_uniform(seed, rep, sweep, dim, L, g, mu):
    return int(lib().swo_bond_uniform(seed, rep, sweep, dim, L, g, mu))


def cluster_decision(model, q, seed, rep, sweep, dim, L, g):
    return int(lib().swo_cluster_decision(model, q, seed, rep, sweep, dim, L, g))


def threshold(model, beta):
    return int(lib().swo_threshold(model, float(beta)))


def nsites(dim, L):
    return L ** dim


def init_state(model, dim, L, q, seed, rep=0):
    s = np.zeros(nsites(dim, L), dtype=STATE_DTYPE[model])
    lib().swo_init_state(model, dim, L, q, seed, rep, _p(s))
    return s


def xy_phi(seed, rep, sweep):
    return float(lib().swo_xy_phi(seed, rep, sweep))


def clock_axis(seed, rep, sweep, q):
    return int(lib().swo_clock_axis(seed, rep, sweep, q))


def clock_projection(q, p, r):
    m, s = ctypes.c_int(), ctypes.c_int()
    lib().swo_clock_projection(q, p, r, ctypes.byref(m), ctypes.byref(s))
    return m.value, s.value


def clock_threshold(q, beta, m1, m2):
    return int(lib().swo_clock_threshold(q, float(beta), m1, m2))


def clock_mirror(q, p, r):
    return int(lib().swo_clock_mirror(q, p, r))


def bonds(model, dim, L, q, beta, seed, rep, sweep, state):
    state = np.ascontiguousarray(state, dtype=STATE_DTYPE[model])
    b = np.zeros(nsites(dim, L), dtype=np.uint8)
    n = lib().swo_bonds(model, dim, L, q, float(beta), seed, rep, sweep, _p(state), _p(b))
    return b, int(n)


def labels_uf(dim, L, b):
    b = np.ascontiguousarray(b, dtype=np.uint8)
    lab = np.zeros(nsites(dim, L), dtype=np.int32)
    lib().swo_labels_uf(dim, L, _p(b), _p(lab))
    return lab


def labels_bfs(dim, L, b):
    b = np.ascontiguousarray(b, dtype=np.uint8)
    lab = np.zeros(nsites(dim, L), dtype=np.int32)
    lib().swo_labels_bfs(dim, L, _p(b), _p(lab))
    return lab


def set_clusters(model, dim, L, q, seed, rep, sweep, labels, state):
    s = np.array(state, dtype=STATE_DTYPE[model], copy=True)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    lib().swo_set_clusters(model, dim, L, q, seed, rep, sweep, _p(lab), _p(s))
    return s


def measure(model, dim, L, q, state):
    state = np.ascontiguousarray(state, dtype=STATE_DTYPE[model])
    e, x, y = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    al = ctypes.c_int64()
    counts = np.zeros(max(q, 1), dtype=np.int64)
    lib().swo_measure(model, dim, L, q, _p(state), ctypes.byref(e), ctypes.byref(x),
                      ctypes.byref(y), ctypes.byref(al), _p(counts) if model == POTTS else None)
    return {"energy": e.value, "mx": x.value, "my": y.value, "aligned": al.value,
            "counts": counts if model == POTTS else None}


def cluster_stats(labels):
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    out = np.zeros(3, dtype=np.int64)
    lib().swo_cluster_stats(lab.size, _p(lab), _p(out))
    return {"n_clusters": int(out[0]), "max_cluster": int(out[1]), "sum_c2": int(out[2])}


def sweeps(model, dim, L, q, beta, seed, rep, n0, nsweeps, state, record=True, last=True):
    """Run sweeps n0 .. n0+nsweeps-1 on a copy of `state`.  Returns a dict with
    the final state, per-sweep records of the configuration entering each
    sweep and the bonds/labels of the last sweep."""
    N = nsites(dim, L)
    s = np.array(state, dtype=STATE_DTYPE[model], copy=True)
    rec = None
    if record:
        rec = {"energy": np.zeros(nsweeps), "mx": np.zeros(nsweeps), "my": np.zeros(nsweeps),
               "aligned": np.zeros(nsweeps, dtype=np.int64),
               "counts": np.zeros((nsweeps, q), dtype=np.int64) if model == POTTS else None}
    b = np.zeros(N, dtype=np.uint8) if last else None
    lab = np.zeros(N, dtype=np.int32) if last else None
    lib().swo_sweeps(model, dim, L, q, float(beta), seed, rep, n0, nsweeps, _p(s),
                     _p(rec["energy"]) if rec else None, _p(rec["mx"]) if rec else None,
                     _p(rec["my"]) if rec else None, _p(rec["aligned"]) if rec else None,
                     _p(rec["counts"]) if (rec and model == POTTS) else None,
                     _p(b), _p(lab))
    return {"state": s, "records": rec, "bonds": b, "labels": lab}
