"""Pins of the oracle's two XY draws against what the method fixes, not
against their own formulas: the embedding direction phi of a sweep is a
uniform angle on the circle (Sec. 2, embedded-cluster paragraph: a random
unit vector per update), independent from sweep to sweep and finer than 32
bits; the hot-start angles are uniform on [0, 2pi) and never reach 2pi.
A plausible slip (phi on [0, pi), one 32-bit word, the same word for every
sweep, a stored angle equal to 2pi) fails one of these."""
import math

import numpy as np
import pytest

import oracle


def chi2_uniform(x, lo, hi, bins):
    h, _ = np.histogram(x, bins=bins, range=(lo, hi))
    e = len(x) / bins
    return float(((h - e) ** 2 / e).sum())


def test_phi_is_uniform_on_the_circle():
    phi = np.array([oracle.xy_phi(20140328, 0, n) for n in range(40000)])
    assert phi.min() >= 0.0 and phi.max() < 2 * math.pi
    # chi^2 with 63 degrees of freedom: mean 63, sd ~11; 120 is > 5 sd
    assert chi2_uniform(phi, 0.0, 2 * math.pi, 64) < 120
    # first circular moments of a uniform angle vanish (sd 1/sqrt(2 n) ~ 0.0035)
    assert abs(np.mean(np.cos(phi))) < 0.02 and abs(np.mean(np.sin(phi))) < 0.02
    assert abs(np.mean(np.cos(2 * phi))) < 0.02


def test_phi_changes_every_sweep_and_replica():
    a = np.array([oracle.xy_phi(7, 0, n) for n in range(20000)])
    # consecutive sweeps uncorrelated
    c = np.corrcoef(np.cos(a[:-1]), np.cos(a[1:]))[0, 1]
    assert abs(c) < 0.03
    # different replicas and seeds draw different directions at the same sweep
    b = np.array([oracle.xy_phi(7, 1, n) for n in range(20000)])
    d = np.array([oracle.xy_phi(8, 0, n) for n in range(20000)])
    assert np.mean(a == b) < 1e-3 and np.mean(a == d) < 1e-3
    assert abs(np.corrcoef(np.cos(a), np.cos(b))[0, 1]) < 0.03


def test_phi_has_more_than_32_bits():
    """53 random bits: scaled back to [0, 2^53) the values are not all
    multiples of 2^21 (what a single 32-bit word would give)."""
    phi = np.array([oracle.xy_phi(11, 0, n) for n in range(2000)])
    u = phi / (2 * math.pi) * 2.0 ** 53
    frac_bits = np.mod(np.round(u), 2.0 ** 21)
    assert np.mean(frac_bits != 0) > 0.99


@pytest.mark.parametrize("dim,L", [(2, 700), (3, 80)])
def test_xy_hot_start_is_uniform(dim, L):
    th = oracle.init_state(oracle.XY, dim, L, 0, 99, 0).astype(np.float64)
    n = th.size
    assert th.min() >= 0.0 and th.max() < 2 * math.pi
    assert np.float32(th.max()) < np.float32(2 * math.pi)
    # 255 degrees of freedom: mean 255, sd ~22.6; 390 is > 5 sd
    assert chi2_uniform(th, 0.0, 2 * math.pi, 256) < 390
    tol = 6.0 / math.sqrt(2 * n)
    assert abs(np.mean(np.cos(th))) < tol and abs(np.mean(np.sin(th))) < tol
    # neighbouring sites independent (the init stream is read site by site)
    r = np.corrcoef(np.cos(th[:-1]), np.cos(th[1:]))[0, 1]
    assert abs(r) < 6.0 / math.sqrt(n)
