"""The allocation-free entry point sw_cluster_stats_noalloc against the
allocating path (sw_measure's cluster statistics) and the oracle: two calls
in a row on one GPU, the second on a smaller lattice (the shared device
array keeps the first call's contents), plus the size limit."""
import sys

import numpy as np
import pytest

import oracle

sw = pytest.importorskip("paper_1403_7560_amd")
pytestmark = pytest.mark.gpu

ISING, POTTS = oracle.ISING, oracle.POTTS


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_noalloc_cluster_stats_two_calls_second_smaller():
    for model, dim, L, q, beta, seed in [(ISING, 2, 300, 2, 0.44, 3), (POTTS, 3, 30, 3, 1.0, 4),
                                         (ISING, 2, 40, 2, 0.5, 5)]:
        say(f"[noalloc] model={model} dim={dim} L={L}")
        lat = sw.Lattice(model, dim, L, q, beta, seed)
        assert lat.cluster_stats_noalloc() == {"n_clusters": 0, "max_cluster": 0, "sum_c2": 0}
        lat.sweep(4)
        got = lat.cluster_stats_noalloc()
        m = lat.measure()
        assert got == {k: m[k] for k in ("n_clusters", "max_cluster", "sum_c2")}
        ref = oracle.sweeps(model, dim, L, q, beta, seed, 0, 0, 4, oracle.init_state(model, dim, L, q, seed))
        assert got == oracle.cluster_stats(ref["labels"])
        assert got["n_clusters"] >= 1 and sum([got["max_cluster"]]) <= L ** dim
        lat.close()


def test_noalloc_rejects_lattices_beyond_its_array():
    say("[noalloc] 2D L=2100 (4.41e6 sites > 2^22)")
    lat = sw.Lattice(ISING, 2, 2100, 2, 0.44, 1)
    lat.sweep(1)
    with pytest.raises(sw.SWError) as e:
        lat.cluster_stats_noalloc()
    assert e.value.code == -1 and "at most" in str(e.value)
    lat.close()
