"""Pins of the oracle's cluster labelling (Sec. 2, step (2); label equivalence
whose fixed point is the minimum site index of each cluster).

Union-find and breadth-first search are two independent labelling methods in
the oracle; both are checked against scipy's connected components (a library
routine) and against a brute-force fixed-point iteration written here, on
random bond sets, and against the invariants every min-index labelling has.
"""
import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import oracle


def edges(dim, L, bonds):
    N = L ** dim
    idx = np.arange(N)
    coords = [idx % L, (idx // L) % L] + ([idx // (L * L)] if dim == 3 else [])
    src, dst = [], []
    for mu in range(dim):
        c = [a.copy() for a in coords]
        c[mu] = (c[mu] + 1) % L
        j = c[0] + L * c[1] + (L * L * c[2] if dim == 3 else 0)
        on = (bonds >> mu) & 1 == 1
        src.append(idx[on])
        dst.append(j[on])
    return np.concatenate(src), np.concatenate(dst)


def scipy_min_labels(dim, L, bonds):
    N = L ** dim
    s, d = edges(dim, L, bonds)
    g = coo_matrix((np.ones(len(s)), (s, d)), shape=(N, N))
    _, comp = connected_components(g, directed=False)
    mins = np.full(comp.max() + 1, N)
    np.minimum.at(mins, comp, np.arange(N))
    return mins[comp].astype(np.int32)


def brute_fixed_point(dim, L, bonds):
    # label equivalence by plain relaxation: label <- min over active neighbours
    N = L ** dim
    lab = np.arange(N)
    s, d = edges(dim, L, bonds)
    while True:
        new = lab.copy()
        np.minimum.at(new, s, lab[d])
        np.minimum.at(new, d, lab[s])
        if np.array_equal(new, lab):
            return lab.astype(np.int32)
        lab = new


def random_bonds(rng, dim, L, p):
    N = L ** dim
    b = np.zeros(N, dtype=np.uint8)
    for mu in range(dim):
        b |= ((rng.random(N) < p).astype(np.uint8) << mu)
    return b


@pytest.mark.parametrize("dim,L", [(2, 3), (2, 4), (2, 7), (2, 33), (3, 3), (3, 4), (3, 6)])
@pytest.mark.parametrize("p", [0.0, 0.3, 0.5, 0.7, 1.0])
def test_labels_agree(dim, L, p):
    rng = np.random.default_rng(1000 * dim + L + int(10 * p))
    for _ in range(3):
        b = random_bonds(rng, dim, L, p)
        uf = oracle.labels_uf(dim, L, b)
        bfs = oracle.labels_bfs(dim, L, b)
        ref = scipy_min_labels(dim, L, b)
        np.testing.assert_array_equal(uf, ref)
        np.testing.assert_array_equal(bfs, ref)
        if L <= 7:
            np.testing.assert_array_equal(uf, brute_fixed_point(dim, L, b))


@pytest.mark.parametrize("dim,L", [(2, 16), (3, 8)])
def test_label_invariants(dim, L):
    rng = np.random.default_rng(7)
    b = random_bonds(rng, dim, L, 0.45)
    lab = oracle.labels_uf(dim, L, b)
    i = np.arange(L ** dim)
    assert np.all(lab <= i)
    assert np.all(lab[lab] == lab)
    s, d = edges(dim, L, b)
    assert np.all(lab[s] == lab[d])
    st = oracle.cluster_stats(lab)
    sizes = np.bincount(lab, minlength=L ** dim)
    assert st["n_clusters"] == int((sizes > 0).sum())
    assert st["max_cluster"] == int(sizes.max())
    assert st["sum_c2"] == int((sizes.astype(np.int64) ** 2).sum())
    assert int(sizes.sum()) == L ** dim


def test_wraparound_cluster():
    # a single active x-row in a 5x5 lattice wraps into one cluster of 5
    L = 5
    b = np.zeros(L * L, dtype=np.uint8)
    b[2 * L:3 * L] = 1
    lab = oracle.labels_uf(2, L, b)
    assert np.all(lab[2 * L:3 * L] == 2 * L)
    rest = np.r_[0:2 * L, 3 * L:L * L]
    assert np.array_equal(lab[rest], rest)
