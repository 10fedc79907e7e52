"""Exact free energy of the periodic m x n square-lattice Ising model
(Kaufman's solution, Phys. Rev. 76, 1232 (1949)), used to pin the oracle at
finite L without any finite-size approximation.

Z = 1/2 (2 sinh 2K)^(mn/2) (Z1 + Z2 + Z3 + Z4) with
Z1, Z2 = prod_r 2cosh / 2sinh (m g_(2r+1) / 2) and Z3, Z4 = the same over
g_(2r), r = 0..n-1, where cosh g_l = cosh 2K cosh 2K* - cos(pi l / n),
K* = -ln tanh(K) / 2 and g_0 = 2 (K - K*) (signed)."""
import math

import numpy as np


def log_z(beta, m, n):
    K = beta
    Ks = -0.5 * math.log(math.tanh(K))
    l = np.arange(2 * n)
    g = np.arccosh(math.cosh(2 * K) * math.cosh(2 * Ks) - np.cos(np.pi * l / n))
    g[0] = 2 * (K - Ks)
    g_odd, g_even = g[1::2], g[0::2]
    terms = []
    for gs in (g_odd, g_even):
        terms.append((np.sum(np.log(2 * np.cosh(m * gs / 2))), 1.0))
        terms.append((np.sum(np.log(2 * np.abs(np.sinh(m * gs / 2)))), float(np.prod(np.sign(gs)))))
    top = max(t[0] for t in terms)
    total = sum(sgn * math.exp(lv - top) for lv, sgn in terms)
    return math.log(0.5) + (m * n / 2) * math.log(2 * math.sinh(2 * K)) + top + math.log(total)


def energy_per_site(beta, L, h=1e-5):
    """Exact <E>/N of the periodic L x L lattice (central difference of ln Z)."""
    return -(log_z(beta + h, L, L) - log_z(beta - h, L, L)) / (2 * h) / (L * L)
