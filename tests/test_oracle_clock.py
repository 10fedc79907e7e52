"""Pins of the oracle's q-state clock model, the paper's own XY path (Sec. 2,
XY paragraph: a clock model with q <= 512, a random mirror direction `ispr`
per sweep and tables of the pair energy; Sec. 3 runs q = 512).

  * geometry: the mirror p -> (q/2 + r - p) mod q is the reflection
    s -> s - 2 (s.n) n of the spin vector on the axis n at angle pi r / q,
    and the folded projection table gives cos(theta - phi);
  * exact enumeration of the 3x3 q = 6 clock model (6^9 states): the
    chain's energy histogram and <E>, <m^2> against the Boltzmann ones;
  * q = 4 is two independent Ising models at half the coupling, so the
    4x4 clock chain must reproduce the convolution of two exactly enumerated
    4x4 Ising energy distributions at beta/2;
  * q = 2 is the Ising model: the 4x4 chain at T_c against its exact values;
  * q = 512 is the XY model to far better than the statistics: the chain
    against a textbook Metropolis sampler of the continuous model.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from test_oracle_enumeration import batch_mean_z, chi2_pvalue, energy_pmf, ising2d_enum
from test_oracle_physics import xy_metropolis

CLOCK = oracle.CLOCK


def vec(q, p):
    t = 2 * math.pi * np.asarray(p, dtype=np.float64) / q
    return np.stack([np.cos(t), np.sin(t)], -1)


@pytest.mark.parametrize("q", [2, 4, 6, 10, 512])
def test_mirror_and_projection_geometry(q):
    rng = np.random.default_rng(q)
    for _ in range(300):
        p, r = int(rng.integers(q)), int(rng.integers(q))
        phi = math.pi * r / q
        n = np.array([math.cos(phi), math.sin(phi)])
        s = vec(q, p)
        p2 = oracle.clock_mirror(q, p, r)
        assert 0 <= p2 < q
        np.testing.assert_allclose(vec(q, p2), s - 2 * s.dot(n) * n, atol=1e-12)
        assert oracle.clock_mirror(q, p2, r) == p  # an involution
        m, sg = oracle.clock_projection(q, p, r)
        want = float(s.dot(n))
        if sg == 0:
            assert abs(want) < 1e-12 and 2 * m == q
        else:
            assert 0 <= 2 * m < q
            assert sg * math.cos(math.pi * m / q) == pytest.approx(want, abs=1e-12)
    # every axis is drawn: r spreads uniformly over [0, q)
    rs = np.array([oracle.clock_axis(3, 0, n, q) for n in range(4000)])
    assert rs.min() >= 0 and rs.max() < q
    if q <= 10:
        assert np.all(np.bincount(rs, minlength=q) > 4000 / q * 0.7)


def test_threshold_limits():
    assert oracle.clock_threshold(8, 0.0, 0, 0) == 0
    assert oracle.clock_threshold(8, 1e6, 0, 1) == 2 ** 32 - 1
    # aligned with the axis: the Ising probability 1 - exp(-2 beta)
    b = 0.37
    assert oracle.clock_threshold(512, b, 0, 0) == oracle.threshold(oracle.ISING, b)
    # the product of projections shrinks the coupling
    assert oracle.clock_threshold(512, b, 100, 3) < oracle.clock_threshold(512, b, 10, 3)


def clock_enum(L, q):
    N = L * L
    st = np.array(list(itertools.product(range(q), repeat=N)), dtype=np.int16)
    idx = np.arange(N)
    x, y = idx % L, idx // L
    jx = (x + 1) % L + L * y
    jy = x + L * ((y + 1) % L)
    rule = np.cos(2 * math.pi * np.arange(q) / q)
    E = -(rule[(st - st[:, jx]) % q].sum(1) + rule[(st - st[:, jy]) % q].sum(1))
    t = 2 * math.pi * st / q
    M2 = np.cos(t).sum(1) ** 2 + np.sin(t).sum(1) ** 2
    return E, M2


def test_clock_q6_3x3_exact():
    L, q, beta = 3, 6, 1.1
    N = L * L
    E, M2 = clock_enum(L, q)
    assert len(E) == 6 ** 9
    w = np.exp(-beta * (E - E.min()))
    Z = w.sum()
    e_ex = float((w * E).sum() / Z) / N
    m2_ex = float((w * M2).sum() / Z) / N ** 2
    s0 = oracle.init_state(CLOCK, 2, L, q, seed=4)
    r = oracle.sweeps(CLOCK, 2, L, q, beta, 4, 0, 0, 300000, s0, last=False)["records"]
    e = r["energy"][1000:]
    m2 = (r["mx"][1000:] ** 2 + r["my"][1000:] ** 2) / N ** 2
    assert abs(batch_mean_z(e / N, e_ex)) < 5
    assert abs(batch_mean_z(m2, m2_ex)) < 5
    # energies are multiples of 1/2: histogram on 2E
    vals, pm = energy_pmf(np.rint(2 * E).astype(np.int64), w / Z)
    pv, stat, dof = chi2_pvalue(np.rint(2 * e[::5]).astype(np.int64), vals, pm)
    assert pv > 1e-6, (pv, stat, dof)


def test_clock_q4_is_two_isings_at_half_coupling():
    """Rotated by 45 degrees, the four clock states are (sigma, tau)/sqrt 2
    with two Ising spins, and s_i.s_j = (sigma_i sigma_j + tau_i tau_j)/2:
    H_clock = (H_sigma + H_tau)/2, two independent Ising models at beta/2."""
    L, q = 4, 4
    T = 0.5 * 2.0 / math.log(1.0 + math.sqrt(2.0))  # the clock-4 critical point
    beta = 1.0 / T
    N = L * L
    Ei, Mi = ising2d_enum(L)
    wi = np.exp(-(beta / 2) * (Ei - Ei.min()))
    wi /= wi.sum()
    vals_i, pm_i = energy_pmf(Ei, wi)
    # E_clock = (E_sigma + E_tau)/2: the distribution of 2 E_clock is the convolution
    conv = {}
    for a, pa in zip(vals_i, pm_i):
        for b, pb in zip(vals_i, pm_i):
            conv[a + b] = conv.get(a + b, 0.0) + pa * pb
    vals = np.array(sorted(conv))
    pm = np.array([conv[v] for v in vals])
    e_ex = float((vals * pm).sum()) / 2 / N
    m2_ex = float((wi * (Mi / N) ** 2).sum())  # |m|^2 = (m_sigma^2 + m_tau^2)/2
    s0 = oracle.init_state(CLOCK, 2, L, q, seed=9)
    r = oracle.sweeps(CLOCK, 2, L, q, beta, 9, 0, 0, 300000, s0, last=False)["records"]
    e = r["energy"][1000:]
    m2 = (r["mx"][1000:] ** 2 + r["my"][1000:] ** 2) / N ** 2
    assert abs(batch_mean_z(e / N, e_ex)) < 5
    assert abs(batch_mean_z(m2, m2_ex)) < 5
    pv, stat, dof = chi2_pvalue(np.rint(2 * e[::5]).astype(np.int64), vals, pm)
    assert pv > 1e-6, (pv, stat, dof)


def test_clock_q2_is_ising():
    L, q = 4, 2
    beta = math.log(1.0 + math.sqrt(2.0)) / 2.0
    N = L * L
    s0 = oracle.init_state(CLOCK, 2, L, q, seed=12)
    r = oracle.sweeps(CLOCK, 2, L, q, beta, 12, 0, 0, 300000, s0, last=False)["records"]
    e = r["energy"][1000:] / N
    m2 = (r["mx"][1000:] ** 2 + r["my"][1000:] ** 2) / N ** 2
    assert abs(batch_mean_z(e, -1.5656237876)) < 5
    assert abs(batch_mean_z(m2, 0.7613589086)) < 5


def test_clock_512_against_metropolis_xy():
    dim, L, beta = 2, 4, 1.0
    N = L ** dim
    E_m, m2_m = xy_metropolis(dim, L, beta, 3000, 64, seed=23)
    E_m, m2_m = E_m[500:], m2_m[500:]
    em, es = E_m.mean(0), E_m.mean(0).std(ddof=1) / math.sqrt(E_m.shape[1])
    mm, ms = m2_m.mean(0), m2_m.mean(0).std(ddof=1) / math.sqrt(m2_m.shape[1])
    s0 = oracle.init_state(CLOCK, dim, L, 512, seed=6)
    r = oracle.sweeps(CLOCK, dim, L, 512, beta, 6, 0, 0, 60000, s0, last=False)["records"]
    e = r["energy"][500:] / N
    m2 = (r["mx"][500:] ** 2 + r["my"][500:] ** 2) / N ** 2
    for sw, mean_m, err_m in [(e, em.mean(), es), (m2, mm.mean(), ms)]:
        bm = np.array([v.mean() for v in np.array_split(sw, 40)])
        err_s = bm.std(ddof=1) / math.sqrt(len(bm))
        z = (sw.mean() - mean_m) / math.sqrt(err_s ** 2 + err_m ** 2)
        assert abs(z) < 5, (sw.mean(), mean_m, err_s, err_m)


def test_planted_parity_error_is_caught():
    """Mirrors on the q state axes only (r even in units of pi/q) would keep
    the parity of p forever: the chain from a hot start must change the
    parity of sites, which the half-step axes make possible."""
    L, q = 6, 8
    s0 = oracle.init_state(CLOCK, 2, L, q, seed=2)
    out = oracle.sweeps(CLOCK, 2, L, q, 0.3, 2, 0, 0, 50, s0, last=False)["state"]
    assert np.any((out.astype(int) - s0.astype(int)) % 2 != 0)
