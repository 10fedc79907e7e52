"""Parity of the HIP path with the oracle on lattices drawn at random (a
fixed seed, so the list is the same on every run): any model, 2D or 3D, any
side from 3 up (ragged tiles on most), Potts q from 2 to 256, temperatures
around each model's critical one, any tile shape, a hot start or a seeded
random state at a later stream position.  Every site's bond byte, label and
state and every record are compared."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1403_7560_amd import inputs

sw = pytest.importorskip("paper_1403_7560_amd")
pytestmark = pytest.mark.gpu

from test_gpu_parity import compare_lattice, compare_records  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def draw_cases(n, seed=20140331):
    rng = np.random.default_rng(seed)
    cases = []
    for i in range(n):
        model = int(rng.integers(0, 3))
        dim = int(rng.integers(2, 4))
        L = int(rng.integers(3, 301)) if dim == 2 else int(rng.integers(3, 49))
        q = 2 if model == 0 else (0 if model == 2 else int(rng.choice([2, 3, 4, 5, 8, 10, 11, 16, 100, 256])))
        if model == 0:
            tc = inputs.TC_ISING_2D if dim == 2 else inputs.TC_ISING_3D
        elif model == 1:
            tc = inputs.tc_potts_2d(q) if dim == 2 else 1.8 / math.log(1.0 + math.sqrt(q))  # near the 3D values
        else:
            tc = 0.89 if dim == 2 else inputs.TC_XY_3D
        T = tc * float(rng.uniform(0.8, 1.2))
        tile = int(rng.integers(0, 4))  # reduced modulo the model's shape count below
        start = int(rng.integers(0, 2))  # 0: hot start, 1: random state at a later sweep index
        cases.append((i, model, dim, L, q, round(T, 6), tile, start, int(rng.integers(1, 1 << 30))))
    return cases


@pytest.mark.parametrize("i,model,dim,L,q,T,tile,start,seed", draw_cases(200))
def test_random_case(i, model, dim, L, q, T, tile, start, seed):
    tile %= sw.tile_count(model, dim)
    n = 3
    beta = 1.0 / T
    say(f"[random {i}] model={model} dim={dim} L={L} q={q} T={T} tile={tile} start={start} seed={seed}")
    lat = sw.Lattice(model, dim, L, q, beta, seed, tile=tile)
    if start == 0:
        s0, n0 = oracle.init_state(model, dim, L, q, seed), 0
    else:
        s0, n0 = inputs.random_state(model, dim, L, q, seed=seed + 1), 1000 + seed % 5000
        lat.set_state(s0)
        lat.set_sweep_index(n0)
    lat.sweep(n)
    ref = oracle.sweeps(model, dim, L, q, beta, seed, 0, n0, n, s0)
    compare_lattice(model, lat.get_state(), lat.get_labels(), lat.get_bonds(), ref)
    compare_records(model, dim, L, q, lat.series(), ref["records"])
    lat.close()


def draw_lattices(rng, n):
    lats = []
    for _ in range(n):
        model = int(rng.integers(0, 3))
        dim = int(rng.integers(2, 4))
        L = int(rng.integers(3, 151)) if dim == 2 else int(rng.integers(3, 33))
        q = 2 if model == 0 else (0 if model == 2 else int(rng.choice([2, 3, 4, 10, 11, 256])))
        lats.append(dict(model=model, dim=dim, L=L, q=q, beta=float(rng.uniform(0.2, 1.2)),
                         seed=int(rng.integers(1, 1 << 30)), replica=int(rng.integers(0, 8))))
    return lats


def oracle_run(j, n):
    s0 = oracle.init_state(j["model"], j["dim"], j["L"], j["q"], j["seed"], j["replica"])
    return oracle.sweeps(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], j["replica"], 0, n, s0)


@pytest.mark.parametrize("b", range(4))
def test_random_batch(b):
    """A batch of 16 random lattices, a random chunk length and uneven sweep
    counts, swept in two calls."""
    rng = np.random.default_rng(1000 + b)
    lats = draw_lattices(rng, 16)
    chunk = int(rng.choice([1, 3, 8, 32]))
    c1 = rng.integers(0, 5, len(lats))
    c2 = rng.integers(0, 4, len(lats))
    say(f"[random batch {b}] chunk={chunk} {[(j['model'], j['dim'], j['L']) for j in lats]}")
    bt = sw.Batch(lats)
    bt.set_chunk(chunk)
    bt.sweep_counts(c1)
    bt.sweep_counts(c2)
    for j, m, n in zip(lats, bt.members, c1 + c2):
        assert m.sweep_index() == n
        if n == 0:
            continue
        ref = oracle_run(j, int(n))
        compare_lattice(j["model"], m.get_state(), m.get_labels(), m.get_bonds(), ref)
        compare_records(j["model"], j["dim"], j["L"], j["q"], m.series(), ref["records"])
    bt.close()


@pytest.mark.parametrize("s", range(3))
def test_random_server(s):
    """30 random jobs through the server under a budget of a few jobs at
    once, with a random number of active jobs and chunk length."""
    rng = np.random.default_rng(2000 + s)
    jobs = draw_lattices(rng, 30)
    for j in jobs:
        j["sweeps"] = int(rng.integers(1, 12))
    budget = 4 * max(sw.footprint(j["model"], j["dim"], j["L"], j["q"]) for j in jobs)
    max_active, chunk = int(rng.choice([2, 5, 16])), int(rng.choice([1, 4, 32]))
    say(f"[random server {s}] max_active={max_active} chunk={chunk}")
    srv = sw.Server(budget, max_active=max_active, chunk=chunk)
    ids = [srv.submit(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], j["replica"], j["sweeps"])
           for j in jobs]
    left, steps = len(jobs), 0
    while left > 0:
        left = srv.step()
        steps += 1
        assert steps < 2000
    for i, j in zip(ids, jobs):
        r = srv.poll(i, j["model"], j["L"] ** j["dim"])
        assert r is not None and r["status"] == 0 and r["sweeps"] == j["sweeps"]
        ref = oracle_run(j, j["sweeps"])
        if j["model"] == 2:
            d = np.abs(r["state"].astype(np.float64) - ref["state"])
            assert np.minimum(d, 2 * np.pi - d).max() < 1e-5
        else:
            np.testing.assert_array_equal(r["state"], ref["state"])
    srv.close()
