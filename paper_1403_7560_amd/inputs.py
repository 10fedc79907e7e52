"""Seeded synthetic inputs shared by the tests and the benchmark.

Holds none of the method's arithmetic: only workload recipes (lattice shapes,
temperatures, sweep counts, the served job mix) and random configurations to
start from.  The SW chain's own random numbers are drawn inside the engine
and the oracle from the counter-based stream.
"""
import math

import numpy as np

ISING, POTTS, XY, CLOCK = 0, 1, 2, 3

TC_ISING_2D = 2.0 / math.log(1.0 + math.sqrt(2.0))  # Onsager
TC_ISING_3D = 4.5115                                 # paper, Sec. 3 (Table 1 temperature)
TC_XY_3D = 2.2019                                    # paper, Sec. 3 (near its Tc estimate)
TC_CLOCK512_3D = 2.20175                             # paper, Sec. 3 (Table 2 temperature)


def tc_potts_2d(q):
    return 1.0 / math.log(1.0 + math.sqrt(q))


def random_state(model, dim, L, q=2, seed=0):
    """A uniformly random configuration (a hot start drawn with numpy)."""
    rng = np.random.default_rng(seed)
    N = L ** dim
    if model == ISING:
        return np.where(rng.random(N) < 0.5, -1, 1).astype(np.int8)
    if model == POTTS:
        return rng.integers(0, q, N).astype(np.uint8)
    if model == CLOCK:
        return rng.integers(0, q, N).astype(np.uint16)
    th = (rng.random(N) * 2 * math.pi).astype(np.float32)
    th[th >= np.float32(2 * math.pi)] = 0.0
    return th


def ordered_state(model, dim, L, q=2, seed=0, disorder=0.05):
    """A mostly aligned configuration drawn with numpy: every site takes the
    common state (Ising +1, Potts 0, XY angle 0) except a `disorder` fraction
    that is drawn uniformly; XY angles also spread by a normal deviate of
    0.3 rad.  At the workloads' temperatures the bonds of such a state
    percolate, so the clusters span the lattice as they do once a chain has
    warmed up near Tc."""
    rng = np.random.default_rng(seed)
    N = L ** dim
    hot = random_state(model, dim, L, q, seed=seed + 1)
    flip = rng.random(N) < disorder
    if model == ISING:
        return np.where(flip, hot, 1).astype(np.int8)
    if model == POTTS:
        return np.where(flip, hot, 0).astype(np.uint8)
    if model == CLOCK:
        return np.where(flip, hot, 0).astype(np.uint16)
    th = np.mod(rng.normal(0.0, 0.3, N), 2 * math.pi).astype(np.float32)
    th[th >= np.float32(2 * math.pi)] = 0.0
    return np.where(flip, hot, th).astype(np.float32)


# The workloads: (name, list of lattices, sweeps).  A lattice is a dict of
# model/dim/L/q/beta/seed/replica.
def workload(name):
    if name == "C1":   # 2D Ising L=64 at T=2.269185, seed 1, 1000 sweeps
        return [dict(model=ISING, dim=2, L=64, q=2, beta=1 / 2.269185, seed=1, replica=0)], 1000
    if name == "C2-potts":  # 2D q=3 Potts L=4096 at its exact Tc
        return [dict(model=POTTS, dim=2, L=4096, q=3, beta=1 / tc_potts_2d(3), seed=2, replica=0)], 10000
    if name == "C2-ising":  # 2D Ising L=4096 at the exact Tc
        return [dict(model=ISING, dim=2, L=4096, q=2, beta=1 / TC_ISING_2D, seed=3, replica=0)], 10000
    if name in ("C2-potts-8192", "C2-ising-8192"):  # the C2 pair at L=8192: larger than the 256 MB Infinity Cache
        lat, _ = workload(name[:-5])
        return [dict(lat[0], L=8192)], 2000
    if name == "C3":   # 3D Ising L=256 at T=4.5115
        return [dict(model=ISING, dim=3, L=256, q=2, beta=1 / TC_ISING_3D, seed=4, replica=0)], 2000
    if name == "CLOCK-512":  # 3D 512-state clock L=256 at T=2.20175 (the paper's Table 2 shape)
        return [dict(model=CLOCK, dim=3, L=256, q=512, beta=1 / TC_CLOCK512_3D, seed=7, replica=0)], 2000
    if name == "C4":   # 3D XY L=128, 32 replicas over [0.95 Tc, 1.05 Tc]
        lats = []
        for r in range(32):
            T = TC_XY_3D * (0.95 + 0.1 * r / 31)
            lats.append(dict(model=XY, dim=3, L=128, q=0, beta=1 / T, seed=5, replica=r))
        return lats, 2000
    raise KeyError(name)


def job_mix(n_jobs, rate=200.0, seed=2014):
    """The served request mix: Poisson arrivals at `rate` jobs/s; each job
    uniform over {2D Ising, 2D Potts q in {3,4,10}, 3D Ising, 3D XY}; L
    log-uniform in [32, 2048] (2D) or [16, 192] (3D); T uniform in
    [0.9 Tc, 1.1 Tc]; sweeps uniform in [100, 5000]; its own seed."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for j in range(n_jobs):
        t += rng.exponential(1.0 / rate)
        cat = int(rng.integers(0, 4))
        if cat == 0:
            model, dim, q, tc = ISING, 2, 2, TC_ISING_2D
        elif cat == 1:
            q = int(rng.choice([3, 4, 10]))
            model, dim, tc = POTTS, 2, tc_potts_2d(q)
        elif cat == 2:
            model, dim, q, tc = ISING, 3, 2, TC_ISING_3D
        else:
            model, dim, q, tc = XY, 3, 0, TC_XY_3D
        lo, hi = (32, 2048) if dim == 2 else (16, 192)
        L = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        T = tc * rng.uniform(0.9, 1.1)
        sweeps = int(rng.integers(100, 5001))
        jobs.append(dict(arrival=t, model=model, dim=dim, L=L, q=q, beta=1.0 / T,
                         seed=int(rng.integers(1, 2**63)), replica=0, sweeps=sweeps))
    return jobs
