"""Physics pins of the oracle beyond enumeration.

  * Onsager's exact energy and Yang's spontaneous magnetisation of the 2D
    Ising model, off criticality where L = 64 is effectively infinite.
  * The critical bond probability p(T_c) = 2 - sqrt 2 of the 2D Ising model.
  * The special case Potts(q = 2, beta' = 2 beta) == Ising(beta): with the
    same seed the two chains are the same trajectory, bond for bond and
    label for label (Sec. 1: the 2-state Potts model is Ising up to the
    energy unit).
  * Swendsen-Wang identities: E[#active] = p E[#aligned], and the improved
    estimator E[M^2 | clusters] = sum_C |C|^2, which also holds for the Potts
    M^2 of Eq. (5).
  * XY: the reflection maps the projection sigma to -sigma and keeps the
    perpendicular component; the SW chain agrees with a textbook
    single-site Metropolis sampler (written here) on <E>/N and <m^2>.
"""
import math

import numpy as np
import pytest
from scipy.special import ellipk

import oracle
from exact_ising2d import energy_per_site
from test_oracle_enumeration import batch_mean_z


def onsager_u(beta):
    k = 2.0 * math.sinh(2 * beta) / math.cosh(2 * beta) ** 2
    K = ellipk(k * k)
    return -1.0 / math.tanh(2 * beta) * (1 + 2.0 / math.pi * (2 * math.tanh(2 * beta) ** 2 - 1) * K)


def yang_m(beta):
    return (1.0 - math.sinh(2 * beta) ** -4) ** 0.125


@pytest.mark.parametrize("T", [2.0, 3.0])
def test_onsager_energy(T):
    L, beta = 64, 1.0 / T
    N = L * L
    s0 = oracle.init_state(oracle.ISING, 2, L, 2, seed=21)
    r = oracle.sweeps(oracle.ISING, 2, L, 2, beta, 21, 0, 0, 2200, s0, last=False)["records"]
    e = r["energy"][200:] / N
    # at L = 64 and these temperatures the finite-size correction is < 1e-9
    assert abs(energy_per_site(beta, L) - onsager_u(beta)) < 1e-8
    assert abs(batch_mean_z(e, onsager_u(beta), nb=20)) < 5
    assert abs(e.mean() - onsager_u(beta)) < 5e-3
    if T < 2.269:
        m = np.abs(r["mx"][200:]) / N
        assert abs(m.mean() - yang_m(beta)) < 5e-3


def test_kaufman_matches_enumeration():
    from test_oracle_enumeration import exact_from_samples, ising2d_enum
    E, _ = ising2d_enum(4)
    for beta in (0.3, math.log(1 + math.sqrt(2)) / 2, 0.5):
        ex, _, _ = exact_from_samples(E, {"e": E / 16}, beta)
        assert energy_per_site(beta, 4) == pytest.approx(ex["e"], abs=1e-8)


@pytest.mark.parametrize("L,T", [(16, 2.0), (16, 2.0 / math.log(1 + math.sqrt(2))), (12, 3.0)])
def test_kaufman_finite_lattice(L, T):
    """The chain's energy against the exact finite-L value (no finite-size
    approximation), at high statistics."""
    beta = 1.0 / T
    N = L * L
    zs = []
    for seed in (1, 2):
        s0 = oracle.init_state(oracle.ISING, 2, L, 2, seed)
        r = oracle.sweeps(oracle.ISING, 2, L, 2, beta, seed, 0, 0, 60000, s0, last=False)["records"]
        zs.append(batch_mean_z(r["energy"][1000:] / N, energy_per_site(beta, L), nb=50))
    assert all(abs(z) < 5 for z in zs), zs
    assert abs(sum(zs) / math.sqrt(len(zs))) < 5


def test_critical_threshold():
    beta_c = math.log(1.0 + math.sqrt(2.0)) / 2.0
    thr = oracle.threshold(oracle.ISING, beta_c)
    assert abs(thr - (2.0 - math.sqrt(2.0)) * 2 ** 32) <= 2
    assert oracle.threshold(oracle.ISING, 0.0) == 0
    assert oracle.threshold(oracle.POTTS, 0.0) == 0
    assert oracle.threshold(oracle.ISING, 1e3) == 2 ** 32
    assert oracle.threshold(oracle.POTTS, 0.7) == oracle.threshold(oracle.ISING, 0.35)


@pytest.mark.parametrize("dim,L", [(2, 9), (2, 16), (3, 5), (3, 8)])
def test_potts2_is_ising(dim, L):
    beta = 0.37 if dim == 2 else 0.2
    seed = 99
    si = oracle.init_state(oracle.ISING, dim, L, 2, seed)
    sp = oracle.init_state(oracle.POTTS, dim, L, 2, seed)
    np.testing.assert_array_equal(si, 1 - 2 * sp.astype(np.int8))
    for n in range(12):
        bi, ai = oracle.bonds(oracle.ISING, dim, L, 2, beta, seed, 0, n, si)
        bp, ap = oracle.bonds(oracle.POTTS, dim, L, 2, 2 * beta, seed, 0, n, sp)
        np.testing.assert_array_equal(bi, bp)
        lab = oracle.labels_uf(dim, L, bi)
        si = oracle.set_clusters(oracle.ISING, dim, L, 2, seed, 0, n, lab, si)
        sp = oracle.set_clusters(oracle.POTTS, dim, L, 2, seed, 0, n, lab, sp)
        np.testing.assert_array_equal(si, 1 - 2 * sp.astype(np.int8))
        mi = oracle.measure(oracle.ISING, dim, L, 2, si)
        mp = oracle.measure(oracle.POTTS, dim, L, 2, sp)
        # Ising E = -(aligned - unlike), Potts E = unlike: E_I = 2 E_P - dN
        assert mi["energy"] == 2 * mp["energy"] - dim * L ** dim
        assert mp["mx"] == pytest.approx(mi["mx"] ** 2, rel=1e-12, abs=1e-9)


@pytest.mark.parametrize("model,dim,L,q,beta", [(oracle.ISING, 2, 16, 2, 0.44),
                                               (oracle.ISING, 3, 8, 2, 0.2216),
                                               (oracle.POTTS, 2, 16, 3, 1.0),
                                               (oracle.POTTS, 3, 8, 4, 0.6)])
def test_sw_identities(model, dim, L, q, beta):
    seed = 4242
    p = (-math.expm1(-2 * beta)) if model == oracle.ISING else (-math.expm1(-beta))
    s = oracle.init_state(model, dim, L, q, seed)
    N = L ** dim
    act, ali, diff = [], [], []
    for n in range(1500):
        m = oracle.measure(model, dim, L, q, s)
        b, na = oracle.bonds(model, dim, L, q, beta, seed, 0, n, s)
        act.append(na)
        ali.append(m["aligned"])
        lab = oracle.labels_uf(dim, L, b)
        s = oracle.set_clusters(model, dim, L, q, seed, 0, n, lab, s)
        m2 = oracle.measure(model, dim, L, q, s)["mx"]
        if model == oracle.ISING:
            m2 = m2 * m2
        diff.append((m2 - oracle.cluster_stats(lab)["sum_c2"]) / N ** 2)
    act, ali = np.array(act[100:], float), np.array(ali[100:], float)
    # each aligned bond is active independently with probability p
    z = (act.sum() - p * ali.sum()) / math.sqrt(p * (1 - p) * ali.sum())
    assert abs(z) < 5
    assert abs(batch_mean_z(np.array(diff[100:]), 0.0, nb=20)) < 5


def test_xy_reflection_geometry():
    L, dim = 12, 2
    N = L * L
    rng = np.random.default_rng(3)
    th = (rng.random(N) * 2 * math.pi).astype(np.float32)
    th[:4] = [0.0, np.float32(2 * math.pi) - np.float32(1e-6), np.float32(math.pi), 1e-7]
    labels = np.arange(N, dtype=np.int32)  # every site its own cluster
    for sweep in range(3):
        phi = oracle.xy_phi(8, 0, sweep)
        new = oracle.set_clusters(oracle.XY, dim, L, 0, 8, 0, sweep, labels, th)
        flip = np.array([oracle.cluster_decision(oracle.XY, 0, 8, 0, sweep, dim, L, i) for i in range(N)])
        assert 0.35 < flip.mean() < 0.65
        assert np.all((new >= 0) & (new < np.float32(2 * math.pi)))
        np.testing.assert_array_equal(new[flip == 0], th[flip == 0])
        a, b = th.astype(np.float64) - phi, new.astype(np.float64) - phi
        f = flip == 1
        np.testing.assert_allclose(np.cos(b[f]), -np.cos(a[f]), atol=2e-6)
        np.testing.assert_allclose(np.sin(b[f]), np.sin(a[f]), atol=2e-6)


def xy_metropolis(dim, L, beta, sweeps, chains, seed):
    """Checkerboard single-site Metropolis for the XY model (textbook)."""
    rng = np.random.default_rng(seed)
    shape = (chains,) + (L,) * dim
    th = rng.random(shape) * 2 * math.pi
    grids = np.indices((L,) * dim).sum(0) % 2
    E_rec, m2_rec = [], []
    axes = list(range(1, dim + 1))
    N = L ** dim
    for sw in range(sweeps):
        for color in (0, 1):
            mask = (grids == color)[None]
            prop = th + rng.uniform(-2.0, 2.0, shape)
            nb = [np.roll(th, sh, ax) for ax in axes for sh in (1, -1)]
            d_old = sum(np.cos(th - t) for t in nb)
            d_new = sum(np.cos(prop - t) for t in nb)
            dE = -(d_new - d_old)
            acc = (rng.random(shape) < np.exp(-beta * dE)) & mask
            th = np.where(acc, prop, th)
        E = -sum(np.cos(th - np.roll(th, 1, ax)).sum(axis=tuple(axes)) for ax in axes)
        mx = np.cos(th).sum(axis=tuple(axes))
        my = np.sin(th).sum(axis=tuple(axes))
        E_rec.append(E / N)
        m2_rec.append((mx * mx + my * my) / N ** 2)
    return np.array(E_rec), np.array(m2_rec)


@pytest.mark.parametrize("dim,L,beta", [(2, 4, 1.0), (3, 4, 0.45)])
def test_xy_against_metropolis(dim, L, beta):
    N = L ** dim
    E_m, m2_m = xy_metropolis(dim, L, beta, 3000, 64, seed=17)
    E_m, m2_m = E_m[500:], m2_m[500:]
    # per-chain means are independent: error of the grand mean from their spread
    em, es = E_m.mean(0), E_m.mean(0).std(ddof=1) / math.sqrt(E_m.shape[1])
    mm, ms = m2_m.mean(0), m2_m.mean(0).std(ddof=1) / math.sqrt(m2_m.shape[1])
    s0 = oracle.init_state(oracle.XY, dim, L, 0, seed=31)
    r = oracle.sweeps(oracle.XY, dim, L, 0, beta, 31, 0, 0, 60000, s0, last=False)["records"]
    e = r["energy"][500:] / N
    m2 = (r["mx"][500:] ** 2 + r["my"][500:] ** 2) / N ** 2
    for sw, mt, mean_m, err_m in [(e, None, em.mean(), es), (m2, None, mm.mean(), ms)]:
        b = np.array_split(sw, 40)
        bm = np.array([v.mean() for v in b])
        err_s = bm.std(ddof=1) / math.sqrt(len(bm))
        z = (sw.mean() - mean_m) / math.sqrt(err_s ** 2 + err_m ** 2)
        assert abs(z) < 5, (sw.mean(), mean_m, err_s, err_m)


def test_xy_high_temperature():
    # at small beta the bond energy tends to -I1(beta)/I0(beta) per bond
    from scipy.special import iv
    L, dim, beta = 16, 2, 0.1
    N = L * L
    s0 = oracle.init_state(oracle.XY, dim, L, 0, seed=2)
    r = oracle.sweeps(oracle.XY, dim, L, 0, beta, 2, 0, 0, 6000, s0, last=False)["records"]
    e_bond = r["energy"][100:] / (dim * N)
    want = -iv(1, beta) / iv(0, beta)
    # the first loop correction on the square lattice is O(beta^3) ~ 1e-3 relative
    assert abs(e_bond.mean() - want) < 2e-3
    assert abs(batch_mean_z(e_bond, want, nb=20)) < 6


def test_xy_bond_margins_near_ties():
    """How close the XY bond test comes to a tie: u = U 2^-32 against
    p = -expm1(-(2 beta s_i) s_j) with s = cos(theta - phi), recomputed with
    numpy's libm on every bond of a 3D lattice and two sweeps' directions.
    A bond whose |u - p| is below 1e-12 could flip if two libms disagreed in
    the last bits of cos or expm1; none may occur, and the decisions must be
    the oracle's.  The smallest margin is printed (the libm margin the GPU
    parity of the XY bonds relies on)."""
    import math
    L, dim, beta, seed = 20, 3, 1 / 2.2019, 3
    st = oracle.init_state(oracle.XY, dim, L, 0, seed)
    N = L ** dim
    g = np.arange(N)
    x, y, z = g % L, (g // L) % L, g // (L * L)
    nbr = [((x + 1) % L) + L * (y + L * z), x + L * (((y + 1) % L) + L * z), x + L * (y + L * ((z + 1) % L))]
    smallest, ties = 1.0, 0
    for n in (0, 1):
        phi = oracle.xy_phi(seed, 0, n)
        b, _ = oracle.bonds(oracle.XY, dim, L, 0, beta, seed, 0, n, st)
        s = np.cos(st.astype(np.float64) - phi)
        for mu in range(dim):
            sj = s[nbr[mu]]
            p = -np.expm1(-(2.0 * beta * s) * sj)
            u = np.array([oracle.bond_uniform(seed, 0, n, dim, L, i, mu) for i in range(N)], dtype=np.float64)
            u *= 2.0 ** -32
            want = (s * sj > 0) & (u < p)
            np.testing.assert_array_equal(((b >> mu) & 1).astype(bool), want)
            m = np.abs(u - p)[s * sj > 0]
            smallest = min(smallest, float(m.min()))
            ties += int((m < 1e-12).sum())
    print(f"XY bond margins: smallest |u - p| = {smallest:.3e} over {2 * dim * N} bonds")
    assert ties == 0 and smallest > 0.0
    assert math.isfinite(smallest)
