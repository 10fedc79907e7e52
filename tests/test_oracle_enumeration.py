"""Whole-chain pins of the oracle by exact enumeration.

The SW chain must sample the Boltzmann distribution of the paper's
Hamiltonians (Sec. 1, Eqs. (1)-(2)).  On lattices small enough to enumerate
every configuration, the exact energy distribution g(E) exp(-E/T) / Z is
computed here independently of the oracle, and the oracle's sampled energy
histogram must agree with it (chi-squared on thinned samples), together with
<E>/N, <m^2> and <m^4>.

  * 4x4 Ising at T = 2/ln(1+sqrt 2)          (2^16 states)
  * 3x3 q=3 Potts at T = 1/ln(1+sqrt 3)      (3^9 states; pins reading R2,
    p = 1 - exp(-J/T) for H = -J sum (delta - 1))
  * 3x3x3 Ising at T = 4.5115                (2^27 states, by layers)
"""
import itertools
import math

import numpy as np
import pytest
from scipy.stats import chi2

import oracle


def ising2d_enum(L):
    N = L * L
    st = np.arange(2 ** N, dtype=np.int64)
    s = 1 - 2 * ((st[:, None] >> np.arange(N)) & 1).astype(np.int64)
    idx = np.arange(N)
    x, y = idx % L, idx // L
    jx = (x + 1) % L + L * y
    jy = x + L * ((y + 1) % L)
    E = -(s * s[:, jx]).sum(1) - (s * s[:, jy]).sum(1)
    M = s.sum(1)
    return E, M


def potts2d_enum(L, q):
    N = L * L
    st = np.array(list(itertools.product(range(q), repeat=N)), dtype=np.int64)
    idx = np.arange(N)
    x, y = idx % L, idx // L
    jx = (x + 1) % L + L * y
    jy = x + L * ((y + 1) % L)
    E = (st != st[:, jx]).sum(1) + (st != st[:, jy]).sum(1)
    n = np.stack([(st == k).sum(1) for k in range(q)], 1)
    M2 = (q * (n ** 2).sum(1) - N * N) / (q - 1)
    return E, M2


def ising3d_enum_hist(L, beta):
    """Exact <E>, <m^2>, <m^4> and P(E) of the LxLxL Ising model (periodic),
    summing over one layer at a time."""
    A = L * L
    st = np.arange(2 ** A, dtype=np.int64)
    s = 1 - 2 * ((st[:, None] >> np.arange(A)) & 1).astype(np.int64)
    idx = np.arange(A)
    x, y = idx % L, idx // L
    jx = (x + 1) % L + L * y
    jy = x + L * ((y + 1) % L)
    e_in = -(s * s[:, jx]).sum(1) - (s * s[:, jy]).sum(1)
    m = s.sum(1)
    e_bt = -(s @ s.T)  # coupling of two stacked layers
    assert L == 3
    Emax = 3 * L ** 3
    Mmax = L ** 3
    hist = np.zeros((2 * Emax + 1) * (2 * Mmax + 1), dtype=np.int64)
    for a in range(2 ** A):
        E = (e_in[a] + e_in[:, None] + e_in[None, :] + e_bt[a, :, None] + e_bt + e_bt[None, :, a])
        M = m[a] + m[:, None] + m[None, :]
        hist += np.bincount(((E + Emax) * (2 * Mmax + 1) + (M + Mmax)).ravel(),
                            minlength=hist.size)
    hist = hist.reshape(2 * Emax + 1, 2 * Mmax + 1)
    Ev = np.arange(-Emax, Emax + 1)
    Mv = np.arange(-Mmax, Mmax + 1)
    assert hist.sum() == 2 ** (L ** 3)
    w = hist * np.exp(-beta * (Ev[:, None] - Ev.min()))
    Z = w.sum()
    N = L ** 3
    PE = w.sum(1) / Z
    m2 = (w * (Mv[None, :] / N) ** 2).sum() / Z
    m4 = (w * (Mv[None, :] / N) ** 4).sum() / Z
    return Ev, PE, m2, m4


def exact_from_samples(E, obs, beta):
    w = np.exp(-beta * (E - E.min()))
    Z = w.sum()
    return {k: float((w * v).sum() / Z) for k, v in obs.items()}, E, w / Z


def energy_pmf(E, p):
    vals = np.unique(E)
    pm = np.array([p[E == v].sum() for v in vals])
    return vals, pm


def chi2_pvalue(samples, vals, pm, min_exp=10.0):
    n = len(samples)
    obs = np.array([(samples == v).sum() for v in vals], dtype=float)
    assert obs.sum() == n, "sampled an energy the enumeration does not have"
    exp = pm * n
    # merge sparse bins (in energy order) until every merged bin has >= min_exp
    o_m, e_m, oa, ea = [], [], 0.0, 0.0
    for o, e in zip(obs, exp):
        oa += o
        ea += e
        if ea >= min_exp:
            o_m.append(oa)
            e_m.append(ea)
            oa = ea = 0.0
    if ea > 0:
        o_m[-1] += oa
        e_m[-1] += ea
    o_m, e_m = np.array(o_m), np.array(e_m)
    stat = float(((o_m - e_m) ** 2 / e_m).sum())
    return float(chi2.sf(stat, len(o_m) - 1)), stat, len(o_m)


def batch_mean_z(x, exact, nb=50):
    b = np.array_split(np.asarray(x, dtype=float), nb)
    means = np.array([v.mean() for v in b])
    err = means.std(ddof=1) / math.sqrt(nb)
    return (means.mean() - exact) / max(err, 1e-300)


def test_ising_4x4_exact():
    L, T = 4, 2.0 / math.log(1.0 + math.sqrt(2.0))
    beta = 1.0 / T
    E, M = ising2d_enum(L)
    N = L * L
    ex, Ev, p = exact_from_samples(E, {"e": E / N, "m2": (M / N) ** 2, "m4": (M / N) ** 4,
                                       "e2": (E / N) ** 2}, beta)
    # the enumeration itself against an independent brute-force computation of
    # the 4x4 density of states and moments at T_c
    assert len(E) == 65536 and (E.min(), E.max()) == (-32, 32)
    vals, cnt = np.unique(E, return_counts=True)
    assert list(vals) == [-32, -24, -20, -16, -12, -8, -4, 0, 4, 8, 12, 16, 20, 24, 32]
    assert list(cnt[:8]) == [2, 32, 64, 424, 1728, 6688, 13568, 20524] and list(cnt) == list(cnt[::-1])
    c_exact = beta ** 2 * N * (ex["e2"] - ex["e"] ** 2)
    assert ex["e"] == pytest.approx(-1.5656237876, abs=1e-10)
    assert ex["m2"] == pytest.approx(0.7613589086, abs=1e-10)
    assert ex["m4"] == pytest.approx(0.6656912133, abs=1e-10)
    assert c_exact == pytest.approx(0.7832668259, abs=1e-10)
    n = 400000
    s0 = oracle.init_state(oracle.ISING, 2, L, 2, seed=11)
    r = oracle.sweeps(oracle.ISING, 2, L, 2, beta, 11, 0, 0, n, s0, last=False)["records"]
    e = r["energy"][1000:]
    m = r["mx"][1000:] / N
    assert abs(batch_mean_z(e / N, ex["e"])) < 5
    assert abs(batch_mean_z(m ** 2, ex["m2"])) < 5
    assert abs(batch_mean_z(m ** 4, ex["m4"])) < 5
    # specific heat per spin (the paper's printed output): per-batch estimates
    cb = np.array([beta ** 2 * N * v.var() for v in np.array_split(e / N, 50)])
    assert abs((cb.mean() - c_exact) / (cb.std(ddof=1) / math.sqrt(50))) < 5
    vals, pm = energy_pmf(E, p)
    pv, stat, dof = chi2_pvalue(e[::5], vals, pm)
    assert pv > 1e-6, (pv, stat, dof)


def test_potts_3x3_q3_exact():
    L, q = 3, 3
    T = 1.0 / math.log(1.0 + math.sqrt(q))
    beta = 1.0 / T
    E, M2 = potts2d_enum(L, q)
    N = L * L
    assert len(E) == 3 ** 9
    ex, Ev, p = exact_from_samples(E, {"e": E / N, "m2": M2 / N ** 2, "m4": (M2 / N ** 2) ** 2},
                                   beta)
    # the enumeration against an independent brute-force computation (H of
    # Eq. (2) with states 0..q-1, M^2 of Eq. (5))
    assert ex["e"] == pytest.approx(0.2578777853, abs=1e-10)
    assert ex["m2"] == pytest.approx(0.8110566549, abs=1e-10)
    assert ex["m4"] == pytest.approx(0.7300389855, abs=1e-10)
    n = 400000
    s0 = oracle.init_state(oracle.POTTS, 2, L, q, seed=5)
    r = oracle.sweeps(oracle.POTTS, 2, L, q, beta, 5, 0, 0, n, s0, last=False)["records"]
    e = r["energy"][1000:]
    m2 = r["mx"][1000:] / N ** 2
    assert abs(batch_mean_z(e / N, ex["e"])) < 5
    assert abs(batch_mean_z(m2, ex["m2"])) < 5
    assert abs(batch_mean_z(m2 ** 2, ex["m4"])) < 5
    vals, pm = energy_pmf(E, p)
    pv, stat, dof = chi2_pvalue(e[::5], vals, pm)
    assert pv > 1e-6, (pv, stat, dof)


def test_potts_reading_rejects_doubled_coupling():
    # The alternative reading p = 1 - exp(-2J/T) is the chain at 2*beta; its
    # <E> must be far from the exact value at beta (so the pin above has power).
    L, q = 3, 3
    beta = math.log(1.0 + math.sqrt(q))
    E, M2 = potts2d_enum(L, q)
    ex1, _, _ = exact_from_samples(E, {"e": E / 9}, beta)
    ex2, _, _ = exact_from_samples(E, {"e": E / 9}, 2 * beta)
    assert ex1["e"] - ex2["e"] > 0.1


def test_ising_3x3x3_exact():
    L, T = 3, 4.5115
    beta = 1.0 / T
    Ev, PE, m2, m4 = ising3d_enum_hist(L, beta)
    N = L ** 3
    n = 300000
    s0 = oracle.init_state(oracle.ISING, 3, L, 2, seed=3)
    r = oracle.sweeps(oracle.ISING, 3, L, 2, beta, 3, 0, 0, n, s0, last=False)["records"]
    e = r["energy"][1000:]
    m = r["mx"][1000:] / N
    e_exact = float((Ev * PE).sum()) / N
    assert abs(batch_mean_z(e / N, e_exact)) < 5
    assert abs(batch_mean_z(m ** 2, m2)) < 5
    assert abs(batch_mean_z(m ** 4, m4)) < 5
    keep = PE > 0
    pv, stat, dof = chi2_pvalue(e[::5], Ev[keep], PE[keep])
    assert pv > 1e-6, (pv, stat, dof)
