"""GPU parity at the workloads' full sizes, in the launch configuration
bench.py times: 2D q=3 Potts and 2D Ising at L = 4096 and 3D Ising at
L = 256 in the plain form (one lattice per launch), 3D XY at L = 128 as 32
replicas in one batched launch.  Two sweeps each (the second applies the
first one's cluster decisions inside the bond kernel); every site's state,
label and bond byte and every record is compared with the oracle, which
finishes a full-size sweep in a few seconds.  Each case runs twice: from
the hot start (small clusters), and from a seeded, mostly aligned state at
sweep index 200, the regime of the timed sweeps after the warm-up, where
one cluster spans the lattice and the global merge links long chains."""
import sys

import numpy as np
import pytest

import oracle
from paper_1403_7560_amd import inputs

sw = pytest.importorskip("paper_1403_7560_amd")
pytestmark = pytest.mark.gpu

from test_gpu_parity import compare_lattice, compare_records  # noqa: E402

SWEEPS = 2
N0 = 200  # sweep index of the ordered-state windows


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_run(j, n):
    s0 = oracle.init_state(j["model"], j["dim"], j["L"], j["q"], j["seed"], j["replica"])
    return oracle.sweeps(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], j["replica"], 0, n, s0)


def ordered(j, r=0):
    return inputs.ordered_state(j["model"], j["dim"], j["L"], j["q"], seed=11 + r)


def oracle_window(j, st, n):
    ref = oracle.sweeps(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], j["replica"], N0, n, st)
    # the premise of the case: the last sweep's largest cluster spans the lattice
    assert np.bincount(ref["labels"]).max() > 0.1 * ref["labels"].size
    return ref


@pytest.mark.parametrize("name", ["C2-potts", "C2-ising", "C3"])
def test_plain_form_full_size(name):
    (j,), _ = inputs.workload(name)
    say(f"[full] {name}: model={j['model']} dim={j['dim']} L={j['L']} sweeps={SWEEPS}")
    lat = sw.Lattice(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], j["replica"])
    lat.sweep(SWEEPS)
    ref = oracle_run(j, SWEEPS)
    compare_lattice(j["model"], lat.get_state(), lat.get_labels(), lat.get_bonds(), ref)
    compare_records(j["model"], j["dim"], j["L"], j["q"], lat.series(), ref["records"])
    lat.close()


def test_batched_form_full_size():
    lats, _ = inputs.workload("C4")
    say(f"[full] C4: {len(lats)} XY 3D L={lats[0]['L']} replicas in one batch, sweeps={SWEEPS}")
    b = sw.Batch(lats)
    b.sweep(SWEEPS)
    for r in (0, 13, len(lats) - 1):
        j, m = lats[r], b.members[r]
        say(f"[full] C4 replica {r} T={1.0 / j['beta']:.5f}")
        ref = oracle_run(j, SWEEPS)
        compare_lattice(j["model"], m.get_state(), m.get_labels(), m.get_bonds(), ref)
        compare_records(j["model"], j["dim"], j["L"], j["q"], m.series(), ref["records"])
    b.close()


@pytest.mark.parametrize("name", ["C2-potts", "C2-ising", "C3"])
def test_plain_form_full_size_ordered(name):
    (j,), _ = inputs.workload(name)
    say(f"[full-ordered] {name}: model={j['model']} dim={j['dim']} L={j['L']} from sweep {N0}, sweeps={SWEEPS}")
    st = ordered(j)
    lat = sw.Lattice(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], j["replica"])
    lat.set_state(st)
    lat.set_sweep_index(N0)
    lat.sweep(SWEEPS)
    ref = oracle_window(j, st, SWEEPS)
    compare_lattice(j["model"], lat.get_state(), lat.get_labels(), lat.get_bonds(), ref)
    compare_records(j["model"], j["dim"], j["L"], j["q"], lat.series(), ref["records"])
    lat.close()


def test_batched_form_full_size_ordered():
    lats, _ = inputs.workload("C4")
    say(f"[full-ordered] C4: {len(lats)} XY 3D L={lats[0]['L']} replicas from sweep {N0}, sweeps={SWEEPS}")
    b = sw.Batch(lats)
    states = {}
    for r, m in enumerate(b.members):
        states[r] = ordered(lats[r], r)
        m.set_state(states[r])
        m.set_sweep_index(N0)
    b.sweep(SWEEPS)
    for r in (0, 13, len(lats) - 1):
        j, m = lats[r], b.members[r]
        say(f"[full-ordered] C4 replica {r} T={1.0 / j['beta']:.5f}")
        ref = oracle_window(j, states[r], SWEEPS)
        compare_lattice(j["model"], m.get_state(), m.get_labels(), m.get_bonds(), ref)
        compare_records(j["model"], j["dim"], j["L"], j["q"], m.series(), ref["records"])
    b.close()


WARM = 200  # GPU sweeps from the hot start before a resumed window


@pytest.mark.parametrize("name", ["C2-potts", "C2-ising", "C3"])
def test_plain_form_window_from_gpu_state(name):
    """200 GPU sweeps from the hot start, then a window of two more: the
    oracle resumes from the state the GPU evolved (at sweep index 200) and
    must reach the same bonds, labels, states and records."""
    (j,), _ = inputs.workload(name)
    say(f"[full-resumed] {name}: {WARM} GPU sweeps, then {SWEEPS} compared")
    lat = sw.Lattice(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], j["replica"])
    lat.sweep(WARM)
    st = lat.get_state()
    lat.reset_measure()
    lat.sweep(SWEEPS)
    ref = oracle.sweeps(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], j["replica"], WARM, SWEEPS, st)
    compare_lattice(j["model"], lat.get_state(), lat.get_labels(), lat.get_bonds(), ref)
    compare_records(j["model"], j["dim"], j["L"], j["q"], lat.series(), ref["records"])
    lat.close()


def test_batched_form_window_from_gpu_state():
    """The 32 C4 replicas sweep 200 times in one batch; replicas 0 and 31
    (the ends of the temperature grid) are compared over two more sweeps
    that the oracle resumes from their GPU-evolved states."""
    lats, _ = inputs.workload("C4")
    say(f"[full-resumed] C4: {WARM} batched sweeps of 32 replicas, then {SWEEPS} compared")
    b = sw.Batch(lats)
    b.sweep(WARM)
    states = {r: b.members[r].get_state() for r in (0, len(lats) - 1)}
    for m in b.members:
        m.reset_measure()
    b.sweep(SWEEPS)
    for r, st in states.items():
        j, m = lats[r], b.members[r]
        say(f"[full-resumed] C4 replica {r} T={1.0 / j['beta']:.5f}")
        ref = oracle.sweeps(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], j["replica"], WARM,
                            SWEEPS, st)
        compare_lattice(j["model"], m.get_state(), m.get_labels(), m.get_bonds(), ref)
        compare_records(j["model"], j["dim"], j["L"], j["q"], m.series(), ref["records"])
    b.close()
