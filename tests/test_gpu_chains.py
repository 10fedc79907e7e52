"""GPU parity on long chains and on the bookkeeping around them.

  * the 2D Ising workload exactly as configured (L = 64, T = 2.269185,
    seed 1, 1000 sweeps, a record every sweep): state, bonds and labels
    compared with the oracle after every 100 sweeps, and all 1000 records;
  * a chain longer than the record buffer's first allocation (1024 rows),
    so that its growth (copy and double) is compared with the oracle too;
  * labels and cluster statistics read after the sweep index was moved
    (they belong to the last sweep run, whatever the index says now);
  * the moments of the recorded series (Sec. 2's printed outputs: <m^2>,
    <m^4>, energy and specific heat per spin; <|m|>; Sec. 3's moment ratio)
    against the same numbers computed from the oracle's records;
  * the error path of the bounded label walks: a tiny walk cap makes every
    kernel stop early and the call report SW_E_NOCONV, after which the
    device still runs a correct chain.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1403_7560_amd import inputs

sw = pytest.importorskip("paper_1403_7560_amd")
pytestmark = pytest.mark.gpu

from test_gpu_parity import compare_lattice, compare_records  # noqa: E402

ISING, POTTS, XY = oracle.ISING, oracle.POTTS, oracle.XY


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_c1_exactly_as_configured():
    (j,), n = inputs.workload("C1")
    assert (j["L"], j["seed"], n) == (64, 1, 1000)
    say(f"[C1] Ising 2D L=64 T=2.269185 seed 1, {n} sweeps in windows of 100")
    lat = sw.Lattice(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"])
    st = oracle.init_state(j["model"], j["dim"], j["L"], j["q"], j["seed"])
    np.testing.assert_array_equal(lat.get_state(), st)
    energy, mx = [], []
    for w in range(n // 100):
        lat.sweep(100)
        ref = oracle.sweeps(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], 0, 100 * w, 100, st)
        compare_lattice(j["model"], lat.get_state(), lat.get_labels(), lat.get_bonds(), ref)
        st = ref["state"]
        energy.append(ref["records"]["energy"])
        mx.append(ref["records"]["mx"])
    got = lat.series()
    assert len(got["sweep"]) == n and np.array_equal(got["sweep"], np.arange(n))
    np.testing.assert_array_equal(got["energy"], np.concatenate(energy))
    np.testing.assert_array_equal(got["mx"], np.concatenate(mx))
    lat.close()


@pytest.mark.parametrize("model,dim,L,q,T", [(ISING, 2, 8, 2, 2.269185), (POTTS, 3, 5, 3, 1.6),
                                             (XY, 2, 6, 0, 0.9)])
def test_record_buffer_growth(model, dim, L, q, T):
    """1500 + 700 measured sweeps: the record buffer starts with 1024 rows and
    grows twice; every record is compared."""
    say(f"[records] model={model} dim={dim} L={L}: 1500 + 700 sweeps")
    seed, beta = 41, 1.0 / T
    lat = sw.Lattice(model, dim, L, q, beta, seed)
    s0 = oracle.init_state(model, dim, L, q, seed)
    lat.sweep(1500)
    lat.sweep(700)
    ref = oracle.sweeps(model, dim, L, q, beta, seed, 0, 0, 2200, s0)
    compare_lattice(model, lat.get_state(), lat.get_labels(), lat.get_bonds(), ref)
    compare_records(model, dim, L, q, lat.series(), ref["records"])
    lat.close()


def test_labels_after_the_sweep_index_moves():
    """sw_get_labels and the cluster statistics read the last labelled sweep's
    buffer, not the one the current sweep index names."""
    say("[index] Ising 2D L=90: sweep 1, index -> 4, labels, stats, sweep 1")
    model, dim, L, q, beta, seed = ISING, 2, 90, 2, 0.44, 12
    lat = sw.Lattice(model, dim, L, q, beta, seed)
    s0 = oracle.init_state(model, dim, L, q, seed)
    lat.sweep(1)
    ref = oracle.sweeps(model, dim, L, q, beta, seed, 0, 0, 1, s0)
    for idx in (4, 7):
        lat.set_sweep_index(idx)
        np.testing.assert_array_equal(lat.get_labels(), ref["labels"])
        got = lat.measure()
        cs = oracle.cluster_stats(ref["labels"])
        assert (got["n_clusters"], got["max_cluster"], got["sum_c2"]) == (
            cs["n_clusters"], cs["max_cluster"], cs["sum_c2"])
    # the chain resumes at sweep 7 from the state the first sweep left
    lat.sweep(2)
    ref2 = oracle.sweeps(model, dim, L, q, beta, seed, 0, 7, 2, ref["state"])
    compare_lattice(model, lat.get_state(), lat.get_labels(), lat.get_bonds(), ref2)
    lat.close()


def oracle_moments(model, N, beta, rec):
    if model == ISING:
        mag = np.abs(rec["mx"])
        m2 = (rec["mx"] / N) ** 2
    elif model == POTTS:
        m2 = rec["mx"] / N ** 2
        mag = np.sqrt(np.maximum(rec["mx"], 0.0))
    else:
        m2 = (rec["mx"] ** 2 + rec["my"] ** 2) / N ** 2
        mag = np.sqrt(rec["mx"] ** 2 + rec["my"] ** 2)
    e = rec["energy"] / N
    return {"n": len(e), "abs_m": (mag / N).mean(), "m2": m2.mean(), "m4": (m2 ** 2).mean(),
            "energy": e.mean(), "energy2": (e ** 2).mean(),
            "specific_heat": beta ** 2 * N * e.var(), "binder": (m2 ** 2).mean() / m2.mean() ** 2}


@pytest.mark.parametrize("model,dim,L,q,T", [(ISING, 2, 48, 2, 2.269185), (POTTS, 2, 40, 3, 0.994972861),
                                             (ISING, 3, 12, 2, 4.5115), (XY, 3, 10, 0, 2.2019)])
def test_moments_of_the_series(model, dim, L, q, T):
    say(f"[moments] model={model} dim={dim} L={L}: 20 discarded + 200 measured sweeps")
    seed, beta, N = 8, 1.0 / T, L ** dim
    lat = sw.Lattice(model, dim, L, q, beta, seed)
    s0 = oracle.init_state(model, dim, L, q, seed)
    lat.sweep(20)
    lat.reset_measure()
    lat.sweep(200)
    got = lat.moments()
    rec = oracle.sweeps(model, dim, L, q, beta, seed, 0, 0, 220, s0)["records"]
    rec = {k: (v[20:] if v is not None else None) for k, v in rec.items()}
    want = oracle_moments(model, N, beta, rec)
    assert got["n"] == 200
    for k, v in want.items():
        assert got[k] == pytest.approx(v, rel=1e-9, abs=1e-12), k
    m = lat.measure()
    assert (m["m2"], m["m4"], m["energy"]) == pytest.approx((want["m2"], want["m4"], want["energy"]), rel=1e-12)
    lat.close()


def test_walk_cap_reports_noconv():
    """A walk cap of one step: the merge's first union already runs out, the
    kernels stop early and flag it, and the call returns SW_E_NOCONV."""
    say("[noconv] Ising 2D L=256 at T=2: walk cap 1")
    lat = sw.Lattice(ISING, 2, 256, 2, 0.5, 5)
    lat.sweep(3)
    lat.set_walk_cap(1)
    with pytest.raises(sw.SWError) as e:
        lat.sweep(2)
    assert e.value.code == -4 and "fixed point" in str(e.value)
    with pytest.raises(sw.SWError):
        lat.set_walk_cap(0)
    lat.close()
    say("[noconv] a fresh lattice afterwards still matches the oracle")
    lat = sw.Lattice(ISING, 2, 256, 2, 0.5, 5)
    lat.sweep(5)
    ref = oracle.sweeps(ISING, 2, 256, 2, 0.5, 5, 0, 0, 5, oracle.init_state(ISING, 2, 256, 2, 5))
    compare_lattice(ISING, lat.get_state(), lat.get_labels(), lat.get_bonds(), ref)
    lat.close()
