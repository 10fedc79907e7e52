"""GPU parity: the HIP path (through the C ABI) against the oracle.

Ising and Potts: states, labels and bonds must match bit for bit after N
sweeps, and the per-sweep records exactly.  XY: bonds must match exactly and
angles within 1e-5 rad (circular distance); the FP64 bond test and the mirror
are evaluated in the same order on both sides, so they are expected to agree
bit for bit as well.

Sizes span several tiles with a ragged tail (the default tiles are 64x64
(Ising/Potts) and 64x32 (XY) in 2D, 64x8x16 and 64x4x8 in 3D) plus lattices
smaller than one tile, where the periodic wrap stays inside the tile; every
other tile shape runs on ragged lattices too.  2D Ising/Potts launches of at
most one 64x64 tile per CU run the 16-wavefront kernels of that tile; the
1100 and 1030 cases have more tiles and run the 4-wavefront ones.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1403_7560_amd import inputs

sw = pytest.importorskip("paper_1403_7560_amd")
pytestmark = pytest.mark.gpu

ISING, POTTS, XY = oracle.ISING, oracle.POTTS, oracle.XY
TWO_PI_F = np.float32(2 * math.pi)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def circ(a, b):
    d = np.abs(a.astype(np.float64) - b.astype(np.float64))
    return np.minimum(d, 2 * math.pi - d)


def compare_lattice(model, got_state, got_labels, got_bonds, ref):
    np.testing.assert_array_equal(got_bonds, ref["bonds"], err_msg="bonds differ")
    if model == XY:
        assert circ(got_state, ref["state"]).max(initial=0.0) < 1e-5
    else:
        np.testing.assert_array_equal(got_state, ref["state"], err_msg="states differ")
    np.testing.assert_array_equal(got_labels, ref["labels"], err_msg="labels differ")


def compare_records(model, dim, L, q, series, rec):
    N = L ** dim
    if model == ISING:
        np.testing.assert_array_equal(series["energy"], rec["energy"])
        np.testing.assert_array_equal(series["mx"], rec["mx"])
    elif model == POTTS:
        np.testing.assert_array_equal(series["energy"], rec["energy"])
        np.testing.assert_allclose(series["mag2"], rec["mx"], rtol=1e-12, atol=1e-6)
    else:
        np.testing.assert_allclose(series["energy"], rec["energy"], rtol=1e-9, atol=1e-9 * dim * N)
        np.testing.assert_allclose(series["mx"], rec["mx"], rtol=1e-9, atol=1e-9 * N)
        np.testing.assert_allclose(series["my"], rec["my"], rtol=1e-9, atol=1e-9 * N)


CASES = [
    # model, dim, L, q, T, sweeps
    (ISING, 2, 3, 2, 2.269185, 20),
    (ISING, 2, 64, 2, 2.269185, 30),
    (ISING, 2, 130, 2, 2.0, 8),
    (ISING, 2, 257, 2, 2.5, 4),
    (POTTS, 2, 5, 3, 0.994972861, 20),
    (POTTS, 2, 130, 3, 0.994972861, 6),
    (POTTS, 2, 67, 10, 0.701231568, 6),
    (POTTS, 2, 40, 256, 0.3, 4),
    (POTTS, 2, 50, 2, 1.7, 5),      # q = 2: one-bit decisions, state counts packed
    (POTTS, 2, 45, 11, 0.7, 4),     # q = 11: the smallest q counted with LDS atomics
    (POTTS, 2, 70, 65, 0.5, 4),     # q > 64: state counts read from two wavefronts' queue memory
    (POTTS, 2, 130, 129, 0.45, 3),  # q > 128: and from three
    # more 64x64 tiles than CUs: the 4-wavefront kernels (fewer run the
    # 16-wavefront ones on the same tiles), here with tiles cut by the edge
    (ISING, 2, 1100, 2, 2.269185, 3),
    (POTTS, 2, 1030, 3, 0.994972861, 2),
    (POTTS, 3, 20, 129, 0.7, 3),
    (ISING, 3, 3, 2, 4.5115, 20),
    (ISING, 3, 33, 2, 4.5115, 5),
    (ISING, 3, 40, 2, 4.0, 4),
    (ISING, 3, 72, 2, 4.5115, 3),  # interior tiles of every 3D shape
    (POTTS, 3, 66, 3, 1.6, 2),
    (POTTS, 3, 17, 3, 1.8, 5),
    (POTTS, 3, 34, 4, 1.6, 3),
    (POTTS, 3, 20, 10, 1.2, 3),     # q = 10: the largest q with packed state counts
    (XY, 2, 5, 0, 0.89, 15),
    (XY, 2, 70, 0, 0.89, 5),
    (XY, 2, 131, 0, 1.2, 3),
    (XY, 3, 3, 0, 2.2019, 15),
    (XY, 3, 18, 0, 2.2019, 4),
    (XY, 3, 33, 0, 2.0, 3),
    (XY, 3, 68, 0, 2.2019, 2),  # interior tiles
]


@pytest.mark.parametrize("model,dim,L,q,T,n", CASES)
def test_hot_start_and_sweeps(model, dim, L, q, T, n):
    say(f"[parity] model={model} dim={dim} L={L} q={q} T={T} sweeps={n}")
    seed = 1000 + 17 * L + model
    beta = 1.0 / T
    lat = sw.Lattice(model, dim, L, q, beta, seed)
    s0 = oracle.init_state(model, dim, L, q, seed)
    got0 = lat.get_state()
    if model == XY:
        np.testing.assert_array_equal(got0.view(np.uint32), s0.view(np.uint32))
    else:
        np.testing.assert_array_equal(got0, s0)
    lat.sweep(n)
    ref = oracle.sweeps(model, dim, L, q, beta, seed, 0, 0, n, s0)
    compare_lattice(model, lat.get_state(), lat.get_labels(), lat.get_bonds(), ref)
    compare_records(model, dim, L, q, lat.series(), ref["records"])
    assert lat.sweep_index() == n
    lat.close()


TILE_CASES = [(ISING, 2, 150, 2, 2.269185), (POTTS, 2, 99, 4, 0.91), (ISING, 3, 21, 2, 4.5115),
              (POTTS, 3, 17, 3, 1.8), (XY, 2, 70, 0, 0.9), (XY, 3, 19, 0, 2.2019),
              # sides with tiles wholly inside the lattice for every shape
              (ISING, 2, 300, 2, 2.269185), (ISING, 3, 80, 2, 4.5115), (XY, 3, 72, 0, 2.2019)]


@pytest.mark.parametrize("model,dim,L,q,T", TILE_CASES)
def test_every_tile_shape(model, dim, L, q, T):
    """The tile shape changes the launch, never the trajectory."""
    n, seed, beta = 4, 31 + L, 1.0 / T
    s0 = oracle.init_state(model, dim, L, q, seed)
    ref = oracle.sweeps(model, dim, L, q, beta, seed, 0, 0, n, s0)
    for tile in range(sw.tile_count(model, dim)):
        say(f"[tile] model={model} dim={dim} L={L} tile={tile} {sw.tile_shape(model, dim, tile)}")
        lat = sw.Lattice(model, dim, L, q, beta, seed, tile=tile)
        assert lat.tile == tile
        lat.sweep(n)
        compare_lattice(model, lat.get_state(), lat.get_labels(), lat.get_bonds(), ref)
        compare_records(model, dim, L, q, lat.series(), ref["records"])
        lat.close()


def test_tuner_picks_a_shape_used_by_later_lattices():
    say("[tune] Ising 2D L=200")
    best, ms = sw.tune(ISING, 2, 200, 2, 0.44, sweeps=3)
    assert 0 <= best < sw.tile_count(ISING, 2)
    assert len(ms) == sw.tile_count(ISING, 2) and all(m > 0 for m in ms)
    assert ms[best] == min(ms)
    lat = sw.Lattice(ISING, 2, 200, 2, 0.44, 5)
    assert lat.tile == best
    lat.sweep(3)
    ref = oracle.sweeps(ISING, 2, 200, 2, 0.44, 5, 0, 0, 3, oracle.init_state(ISING, 2, 200, 2, 5))
    compare_lattice(ISING, lat.get_state(), lat.get_labels(), lat.get_bonds(), ref)
    b = sw.Batch([dict(model=ISING, dim=2, L=200, q=2, beta=0.44, seed=5, replica=0)])
    assert b.members[0].tile == best
    with pytest.raises(sw.SWError):
        sw.Lattice(ISING, 2, 64, 2, 0.44, 1, tile=sw.tile_count(ISING, 2))


def test_default_tile_shape_follows_padding():
    """Untuned lattices take shape 0 unless another pads them much less."""
    def padded(model, dim, L, t):
        p = 1
        for e in sw.tile_shape(model, dim, t)[:dim]:
            p *= -(-L // e) * e
        return p
    for model, dim, L in [(ISING, 3, 256), (ISING, 3, 20), (XY, 3, 12), (ISING, 2, 4096), (POTTS, 2, 40)]:
        say(f"[default tile] model={model} dim={dim} L={L}")
        lat = sw.Lattice(model, dim, L, 2 if model != XY else 0, 0.3, 3)
        n = sw.tile_count(model, dim)
        pads = [padded(model, dim, L, t) for t in range(n)]
        best = min(range(n), key=lambda t: (pads[t], t))
        want = 0 if pads[0] * 4 <= pads[best] * 5 else best
        assert lat.tile == want, (model, dim, L, lat.tile, want, pads)
        lat.close()


@pytest.mark.parametrize("model,dim,L,q,T", [(ISING, 2, 100, 2, 2.3), (POTTS, 3, 20, 5, 1.0),
                                             (XY, 2, 66, 0, 1.1), (XY, 3, 20, 0, 2.2)])
def test_window_from_generated_state(model, dim, L, q, T):
    """Resume at a later stream position from a seeded synthetic state."""
    say(f"[window] model={model} dim={dim} L={L} q={q}")
    seed, n0, n = 77, 123456, 3
    beta = 1.0 / T
    st = inputs.random_state(model, dim, L, q, seed=5)
    lat = sw.Lattice(model, dim, L, q, beta, seed, replica=3)
    lat.set_state(st)
    lat.set_sweep_index(n0)
    lat.sweep(n)
    ref = oracle.sweeps(model, dim, L, q, beta, seed, 3, n0, n, st)
    compare_lattice(model, lat.get_state(), lat.get_labels(), lat.get_bonds(), ref)
    compare_records(model, dim, L, q, lat.series(), ref["records"])
    lat.close()


def test_sweeps_split_across_calls():
    say("[split] Ising 2D L=80 in 3 calls")
    lat = sw.Lattice(ISING, 2, 80, 2, 0.44, 9)
    for n in (3, 0, 5, 1):
        lat.sweep(n)
    ref = oracle.sweeps(ISING, 2, 80, 2, 0.44, 9, 0, 0, 9, oracle.init_state(ISING, 2, 80, 2, 9))
    compare_lattice(ISING, lat.get_state(), lat.get_labels(), lat.get_bonds(), ref)
    compare_records(ISING, 2, 80, 2, lat.series(), ref["records"])


def test_profiling_times_every_16th_sweep_and_changes_nothing():
    say("[profile] Ising 2D L=130, sweeps 5..44 timed, then compared with the oracle")
    lat = sw.Lattice(ISING, 2, 130, 2, 0.44, 21)
    lat.sweep(5)
    lat.profile(2)
    lat.sweep(40)  # sweep indices 5..44: 16 and 32 are timed
    p = lat.profile_read()
    lat.profile(0)
    assert p["bond"][1] == 2 and p["merge"][1] == 2 and p["flip"][1] == 1
    assert p["bond"][0] > 0.0 and p["merge"][0] > 0.0 and p["flip"][0] > 0.0
    ref = oracle.sweeps(ISING, 2, 130, 2, 0.44, 21, 0, 0, 45, oracle.init_state(ISING, 2, 130, 2, 21))
    compare_lattice(ISING, lat.get_state(), lat.get_labels(), lat.get_bonds(), ref)


@pytest.mark.parametrize("beta", [0.0, 50.0])
def test_degenerate_couplings(beta):
    """beta = 0: no bond is active, every site is its own cluster.
    beta -> infinity: every aligned bond is active (p = 1)."""
    say(f"[degenerate] beta={beta}")
    for model, dim, L, q in [(ISING, 2, 37, 2), (POTTS, 3, 9, 3), (XY, 2, 19, 0)]:
        lat = sw.Lattice(model, dim, L, q, beta, 4)
        s0 = oracle.init_state(model, dim, L, q, 4)
        assert np.array_equal(lat.get_state().view(np.uint8), s0.view(np.uint8))
        lat.sweep(2)
        ref = oracle.sweeps(model, dim, L, q, beta, 4, 0, 0, 2, s0)
        compare_lattice(model, lat.get_state(), lat.get_labels(), lat.get_bonds(), ref)
        if beta == 0.0:
            assert np.array_equal(lat.get_labels(), np.arange(L ** dim, dtype=np.int32))


def test_measure_and_cluster_stats():
    say("[measure] Ising 2D L=64 and Potts 3D")
    for model, dim, L, q, beta in [(ISING, 2, 64, 2, 1 / 2.269185), (POTTS, 3, 12, 3, 0.5)]:
        seed = 31
        lat = sw.Lattice(model, dim, L, q, beta, seed)
        s0 = oracle.init_state(model, dim, L, q, seed)
        assert np.array_equal(lat.get_state().view(np.uint8), s0.view(np.uint8))
        lat.sweep(10)
        lat.reset_measure()
        lat.sweep(25)
        got = lat.measure()
        ref = oracle.sweeps(model, dim, L, q, beta, seed, 0, 0, 35, s0)
        N = L ** dim
        mx = ref["records"]["mx"][10:]
        m2 = (mx / N) ** 2 if model == ISING else mx / N ** 2
        assert got["m2"] == pytest.approx(m2.mean(), rel=1e-12)
        assert got["m4"] == pytest.approx((m2 ** 2).mean(), rel=1e-12)
        assert got["energy"] == pytest.approx(ref["records"]["energy"][10:].mean() / N, rel=1e-12)
        cs = oracle.cluster_stats(ref["labels"])
        assert (got["n_clusters"], got["max_cluster"], got["sum_c2"]) == (
            cs["n_clusters"], cs["max_cluster"], cs["sum_c2"])


def test_invalid_arguments():
    say("[invalid]")
    for args in [(4, 2, 10, 2), (ISING, 4, 10, 2), (ISING, 2, 2, 2), (POTTS, 2, 10, 1),
                 (POTTS, 2, 10, 257), (ISING, 3, 1291, 2)]:
        with pytest.raises(sw.SWError):
            sw.Lattice(*args, beta=0.4, seed=1)
    with pytest.raises(sw.SWError):
        sw.Lattice(ISING, 2, 10, 2, beta=-1.0)
    lat = sw.Lattice(POTTS, 2, 10, 3, 0.5, 1)
    bad = np.full(100, 3, dtype=np.uint8)
    with pytest.raises(sw.SWError):
        lat.set_state(bad)
    with pytest.raises(sw.SWError):
        lat.sweep(-1)
