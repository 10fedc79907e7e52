"""GPU parity at the workloads' full sizes, in the launch configuration
bench.py times: 2D q=3 Potts and 2D Ising at L = 4096 and 3D Ising at
L = 256 in the plain form (one lattice per launch), 3D XY at L = 128 as 32
replicas in one batched launch.  Every site's state, label and bond byte
and every record is compared with the oracle, which finishes a full-size
sweep in one to two seconds: ten sweeps from the hot start (small
clusters); two from a seeded, mostly aligned state at sweep index 200,
where one cluster spans the lattice and the global merge links long
chains; and three windows of five sweeps that the oracle resumes from the
states the GPU itself evolved at sweeps 200, 400 and 600 (the oracle's
windows run side by side in threads: its C calls release the GIL)."""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_1403_7560_amd import inputs

sw = pytest.importorskip("paper_1403_7560_amd")
pytestmark = pytest.mark.gpu

from test_gpu_parity import compare_lattice, compare_records  # noqa: E402

SWEEPS = 2
HOT = 10  # sweeps compared from the hot start
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
    say(f"[full] {name}: model={j['model']} dim={j['dim']} L={j['L']} sweeps={HOT}")
    lat = sw.Lattice(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], j["replica"])
    lat.sweep(HOT)
    ref = oracle_run(j, HOT)
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


WINDOWS = (200, 400, 600)  # GPU sweep indices where resumed windows start
WIN = 5  # sweeps per resumed window


def oracle_windows(j, starts):
    """The oracle's windows of WIN sweeps from (sweep index, state) pairs, in
    parallel threads."""
    def one(a):
        n0, st = a
        return oracle.sweeps(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], j["replica"], n0, WIN, st)
    with ThreadPoolExecutor(len(starts)) as ex:
        return list(ex.map(one, starts))


@pytest.mark.parametrize("name", ["C2-potts", "C2-ising", "C3"])
def test_plain_form_window_from_gpu_state(name):
    """From the hot start the GPU runs to sweeps 200, 400 and 600; at each it
    hands its state to the oracle and sweeps five more, which the oracle,
    resuming from that state, must reproduce: bonds, labels, states and
    records."""
    (j,), _ = inputs.workload(name)
    say(f"[full-resumed] {name}: windows of {WIN} sweeps at GPU sweeps {WINDOWS}")
    lat = sw.Lattice(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], j["replica"])
    got, done = [], 0
    for w0 in WINDOWS:
        lat.sweep(w0 - done)
        st = lat.get_state()
        lat.reset_measure()
        lat.sweep(WIN)
        got.append((w0, st, lat.get_state(), lat.get_labels(), lat.get_bonds(), lat.series(64)))
        done = w0 + WIN
    lat.close()
    refs = oracle_windows(j, [(w0, st) for w0, st, *_ in got])
    for (w0, _, state, labels, bonds, series), ref in zip(got, refs):
        say(f"[full-resumed] {name}: window at sweep {w0}")
        compare_lattice(j["model"], state, labels, bonds, ref)
        compare_records(j["model"], j["dim"], j["L"], j["q"], series, ref["records"])


def test_batched_form_window_from_gpu_state():
    """The 32 C4 replicas sweep 200 times in one batch; replicas 0 and 31
    (the ends of the temperature grid) are compared over five more sweeps
    that the oracle resumes from their GPU-evolved states."""
    lats, _ = inputs.workload("C4")
    w0 = WINDOWS[0]
    say(f"[full-resumed] C4: {w0} batched sweeps of 32 replicas, then {WIN} compared")
    b = sw.Batch(lats)
    b.sweep(w0)
    reps = (0, len(lats) - 1)
    states = {r: b.members[r].get_state() for r in reps}
    for m in b.members:
        m.reset_measure()
    b.sweep(WIN)
    got = {r: (b.members[r].get_state(), b.members[r].get_labels(), b.members[r].get_bonds(),
               b.members[r].series(64)) for r in reps}
    b.close()

    def one(r):
        j = lats[r]
        return oracle.sweeps(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], j["replica"], w0, WIN,
                             states[r])
    with ThreadPoolExecutor(len(reps)) as ex:
        refs = dict(zip(reps, ex.map(one, reps)))
    for r in reps:
        j = lats[r]
        say(f"[full-resumed] C4 replica {r} T={1.0 / j['beta']:.5f}")
        state, labels, bonds, series = got[r]
        compare_lattice(j["model"], state, labels, bonds, refs[r])
        compare_records(j["model"], j["dim"], j["L"], j["q"], series, refs[r]["records"])
