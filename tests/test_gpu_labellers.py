"""The paper's two iterative labellers for the global phase of step (2)
(Sec. 2: Hawick et al., algorithm 0, three functions with a temporary R and
atomicMin; Kalentev et al., algorithm 1, two functions on one label array
without atomics), selected per lattice like the program's `algorithm`
parameter.  Each must reach the same minimum-index labels as the oracle, so
the whole trajectory (bonds, labels, states, records) is compared site by
site, on multi-tile lattices with ragged tails, on every model and both
dimensions, and at full size from ordered states where one cluster spans the
lattice.  The iteration cap is a real bound: a cap of one scan cannot
confirm convergence and the call reports SW_E_NOCONV."""
import sys
import time

import numpy as np
import pytest

import oracle
from paper_1403_7560_amd import inputs

sw = pytest.importorskip("paper_1403_7560_amd")
pytestmark = pytest.mark.gpu

from test_gpu_parity import compare_lattice, compare_records  # noqa: E402

ISING, POTTS, XY = oracle.ISING, oracle.POTTS, oracle.XY
NAMES = {0: "Hawick", 1: "Kalentev"}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [
    (ISING, 2, 200, 2, 2.269185, 6),
    (ISING, 2, 131, 2, 1.9, 4),      # ordered phase: spanning clusters
    (POTTS, 2, 150, 3, 0.994972861, 4),
    (POTTS, 2, 70, 65, 0.5, 3),
    (ISING, 3, 40, 2, 4.5115, 4),
    (ISING, 3, 33, 2, 3.8, 3),
    (POTTS, 3, 34, 4, 1.6, 3),
    (XY, 2, 100, 0, 0.89, 4),
    (XY, 3, 20, 0, 2.2019, 3),
    (XY, 3, 33, 0, 1.8, 3),
]


@pytest.mark.parametrize("alg", [0, 1])
@pytest.mark.parametrize("model,dim,L,q,T,n", CASES)
def test_iterative_labeller_parity(alg, model, dim, L, q, T, n):
    say(f"[labeller {NAMES[alg]}] model={model} dim={dim} L={L} q={q} T={T} sweeps={n}")
    seed, beta = 500 + L, 1.0 / T
    lat = sw.Lattice(model, dim, L, q, beta, seed)
    lat.set_labeller(alg, 64)
    s0 = oracle.init_state(model, dim, L, q, seed)
    lat.sweep(n)
    ref = oracle.sweeps(model, dim, L, q, beta, seed, 0, 0, n, s0)
    compare_lattice(model, lat.get_state(), lat.get_labels(), lat.get_bonds(), ref)
    compare_records(model, dim, L, q, lat.series(), ref["records"])
    st = lat.label_stats()
    assert st["labellings"] == n and n <= st["scans"] <= 64 * n and 1 <= st["max_scans"] <= 64
    say(f"[labeller {NAMES[alg]}] scans per sweep {st['scans'] / n:.2f}, max {st['max_scans']}")
    lat.close()


@pytest.mark.parametrize("alg", [0, 1])
@pytest.mark.parametrize("name", ["C2-potts", "C2-ising", "C3"])
def test_iterative_labeller_full_size_ordered(alg, name):
    (j,), _ = inputs.workload(name)
    say(f"[labeller {NAMES[alg]} full-ordered] {name} from sweep 200, 2 sweeps")
    st = inputs.ordered_state(j["model"], j["dim"], j["L"], j["q"], seed=11)
    lat = sw.Lattice(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], j["replica"])
    lat.set_labeller(alg, 256)
    lat.set_state(st)
    lat.set_sweep_index(200)
    t0 = time.perf_counter()
    lat.sweep(2)
    say(f"[labeller {NAMES[alg]} full-ordered] {name}: 2 sweeps in {time.perf_counter() - t0:.3f} s")
    ref = oracle.sweeps(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], j["replica"], 200, 2, st)
    assert np.bincount(ref["labels"]).max() > 0.1 * ref["labels"].size
    compare_lattice(j["model"], lat.get_state(), lat.get_labels(), lat.get_bonds(), ref)
    compare_records(j["model"], j["dim"], j["L"], j["q"], lat.series(), ref["records"])
    s = lat.label_stats()
    say(f"[labeller {NAMES[alg]} full-ordered] {name}: scans {s['scans']} over 2 sweeps, max {s['max_scans']}")
    lat.close()


@pytest.mark.parametrize("alg", [0, 1])
def test_iteration_cap_reports_noconv(alg):
    say(f"[labeller {NAMES[alg]}] cap of one scan on Ising 2D L=256 at T=2")
    lat = sw.Lattice(ISING, 2, 256, 2, 0.5, 3)
    lat.set_labeller(alg, 1)
    with pytest.raises(sw.SWError) as e:
        lat.sweep(1)
    assert e.value.code == -4
    lat.close()


def test_labeller_switch_mid_chain_and_arguments():
    """The labeller may change between calls without changing the chain."""
    say("[labeller] switching union -> Hawick -> Kalentev -> union on Potts 2D L=160")
    model, dim, L, q, beta, seed = POTTS, 2, 160, 3, 1.0 / 0.994972861, 9
    lat = sw.Lattice(model, dim, L, q, beta, seed)
    for alg in (2, 0, 1, 2):
        lat.set_labeller(alg, 32)
        lat.sweep(2)
    ref = oracle.sweeps(model, dim, L, q, beta, seed, 0, 0, 8, oracle.init_state(model, dim, L, q, seed))
    compare_lattice(model, lat.get_state(), lat.get_labels(), lat.get_bonds(), ref)
    compare_records(model, dim, L, q, lat.series(), ref["records"])
    for bad in ((3, 10), (-1, 10), (1, 0), (0, 5000)):
        with pytest.raises(sw.SWError):
            lat.set_labeller(*bad)
    lat.close()
