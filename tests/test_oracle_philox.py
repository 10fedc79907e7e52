"""Pins of the oracle's random-number layer.

Philox4x32-10 (Salmon et al., SC'11) is checked against an independent
implementation, rocRAND's Philox header, run as a tool: for random (key,
counter) pairs the four output words must agree exactly.  rocRAND's counter
for (subsequence s, offset 4b) is (b mod 2^32, b div 2^32, s mod 2^32,
s div 2^32) and its key is the 64-bit seed, so all four counter words and
both key words are exercised.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_kat(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND known-answer tool")
    exe = str(tmp_path_factory.mktemp("kat") / "kat")
    subprocess.run([hipcc, "-O1", "-o", exe, os.path.join(HERE, "rocrand_philox_kat.cpp")],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(rocrand_kat):
    rng = np.random.default_rng(20140329)
    cases = []
    for k in range(400):
        seed = int(rng.integers(0, 2**64, dtype=np.uint64))
        sub = int(rng.integers(0, 2**64, dtype=np.uint64))
        blk = int(rng.integers(0, 2**40, dtype=np.uint64))
        if k % 4 == 0:
            sub &= 0xFFFF
            blk &= 0xFFFF
        cases.append((seed, sub, blk))
    cases += [(0, 0, 0), (2**64 - 1, 2**64 - 1, 2**64 // 4 - 1), (1, 0, 0)]
    inp = "".join(f"{s} {u} {b}\n" for s, u, b in cases)
    out = subprocess.run([rocrand_kat], input=inp, capture_output=True, text=True, check=True)
    lines = out.stdout.strip().split("\n")
    assert len(lines) == len(cases)
    for (seed, sub, blk), line in zip(cases, lines):
        want = [int(v) for v in line.split()]
        ctr = [blk & 0xFFFFFFFF, (blk >> 32) & 0xFFFFFFFF, sub & 0xFFFFFFFF, sub >> 32]
        key = [seed & 0xFFFFFFFF, seed >> 32]
        got = [int(v) for v in oracle.philox(ctr, key)]
        assert got == want, (seed, sub, blk)


def test_word_layout():
    # word w of stream (tag, n) for replica r = lane w%4 of block (w//4, n, tag, r)
    seed = 0x0123456789ABCDEF
    for (rep, tag, n, w) in [(0, 0, 0, 0), (3, 2, 17, 5), (31, 5, 0, 4097), (7, 3, 999, 2**31 - 1)]:
        blk = oracle.philox([w >> 2, n, tag, rep], [seed & 0xFFFFFFFF, seed >> 32])
        assert oracle.word(seed, rep, tag, n, w) == int(blk[w & 3])


def test_philox_uniformity():
    # chi^2 of the top byte and balance of every bit over 2^16 consecutive words
    words = np.array([oracle.word(1, 0, oracle.TAG_BOND, 0, w) for w in range(1 << 16)],
                     dtype=np.uint64)
    counts = np.bincount((words >> 24).astype(np.int64), minlength=256)
    exp = len(words) / 256
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    # 255 dof: mean 255, sd 22.6; 6 sd bounds
    assert 120 < chi2 < 400
    for bit in range(32):
        ones = int(((words >> bit) & 1).sum())
        assert abs(ones - len(words) / 2) < 6 * np.sqrt(len(words) / 4)


def test_bond_uniform_layout():
    # U(g, mu) = P << 16 | S.  Bond primaries are laid out by columns: the
    # Philox block x + L (y//4 + ceil(L/4) z) of BOND holds the words of sites
    # (x, 4 (y//4) + 0..3, z), x primary high, y primary low; z primaries come
    # two per word from BOND_Z blocks of eight rows; secondaries from the tie
    # stream at the row-major bond index
    seed, rep, n = 0x5EED, 2, 7
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for dim, L in ((2, 6), (2, 13), (3, 5), (3, 11)):
        N = L ** dim
        for g in sorted({0, 1, 2, 3, 4, 5, L, L + 1, 3 * L - 1, N // 2, N - 1}):
            x, y, z = g % L, (g // L) % L, g // (L * L)
            blk = oracle.philox([x + L * (y // 4 + -(-L // 4) * z), n, oracle.TAG_BOND, rep], key)
            w = int(blk[y % 4])
            for mu in range(dim):
                u = oracle.bond_uniform(seed, rep, n, dim, L, g, mu)
                if mu < 2:
                    p = (w >> 16) if mu == 0 else (w & 0xFFFF)
                else:
                    zb = oracle.philox([x + L * (y // 8 + -(-L // 8) * z), n, oracle.TAG_BOND_Z, rep], key)
                    wz = int(zb[(y % 8) // 2])
                    p = (wz & 0xFFFF) if (y & 1) else (wz >> 16)
                s_ = oracle.word(seed, rep, oracle.TAG_BOND_TIE, n, dim * g + mu) >> 16
                assert u == (p << 16) | s_, (dim, L, g, mu)


def test_column_layout_is_a_bijection():
    """Every 16-bit half of the BOND words that fall on a site (and of the
    BOND_Z words in 3D) is the primary of exactly one bond of the oracle:
    the sorted primaries that swo_bond_uniform hands out equal the sorted
    halves of the stream's words, so no two bonds share a primary and none
    is left out (sizes that are not multiples of 4 or 8 included)."""
    seed, rep, n = 5, 2, 9
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for dim, L in ((2, 10), (3, 6), (3, 5)):
        N = L ** dim
        got_xy = sorted(oracle.bond_uniform(seed, rep, n, dim, L, g, mu) >> 16 for g in range(N) for mu in (0, 1))
        q4, q8, nz = -(-L // 4), -(-L // 8), (L if dim == 3 else 1)
        want_xy = []
        for b in range(L * q4 * nz):
            yb = (b // L) % q4
            w = oracle.philox([b, n, oracle.TAG_BOND, rep], key)
            for lane in range(4):
                if 4 * yb + lane < L:  # the word of a site
                    want_xy += [int(w[lane]) >> 16, int(w[lane]) & 0xFFFF]
        assert got_xy == sorted(want_xy), (dim, L)
        if dim == 3:
            got_z = sorted(oracle.bond_uniform(seed, rep, n, dim, L, g, 2) >> 16 for g in range(N))
            want_z = []
            for b in range(L * q8 * L):
                yb = (b // L) % q8
                w = oracle.philox([b, n, oracle.TAG_BOND_Z, rep], key)
                for half in range(8):  # y = 8 yb + half: lane half // 2, high half for even y
                    if 8 * yb + half < L:
                        v = int(w[half // 2])
                        want_z.append((v >> 16) if half % 2 == 0 else (v & 0xFFFF))
            assert got_z == sorted(want_z), (dim, L)


def test_bond_uniform_is_uniform():
    L = 28
    u = np.array([oracle.bond_uniform(9, 0, 3, 3, L, i, mu) for i in range(L ** 3) for mu in range(3)],
                 dtype=np.uint64)
    for shift in (28, 12):  # a primary nibble and a secondary nibble
        counts = np.bincount(((u >> shift) & 15).astype(np.int64), minlength=16)
        exp = len(u) / 16
        chi2 = float(((counts - exp) ** 2 / exp).sum())
        assert chi2 < 60  # 15 dof
    d = np.array([oracle.cluster_decision(0, 2, 9, 0, 3, 2, 200, g) for g in range(20000)])
    assert abs(d.mean() - 0.5) < 0.02
    d = np.array([oracle.cluster_decision(1, 5, 9, 0, 3, 2, 200, g) for g in range(20000)])
    assert np.all(np.bincount(d, minlength=5) > 3600)


def test_potts_decision_layout():
    # Potts q >= 3: the new state of the cluster rooted at g is floor(w q / 2^32)
    # for the CLUSTER word of site g in the column layout
    seed, rep, n, q = 77, 1, 4, 7
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for dim, L in ((2, 9), (3, 7)):
        for g in (0, 5, L + 3, L ** dim - 1):
            x, y, z = g % L, (g // L) % L, g // (L * L)
            blk = oracle.philox([x + L * (y // 4 + -(-L // 4) * z), n, oracle.TAG_CLUSTER, rep], key)
            want = (int(blk[y % 4]) * q) >> 32
            assert oracle.cluster_decision(oracle.POTTS, q, seed, rep, n, dim, L, g) == want
