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
    # U(i, mu) = P << 16 | S: primaries packed two per BOND word (x high, y low),
    # z primaries two per BOND_Z word, secondaries from the tie stream
    seed, rep, n = 0x5EED, 2, 7
    for dim in (2, 3):
        for i in (0, 1, 2, 3, 4, 5, 1001, 2**20 + 3):
            for mu in range(dim):
                u = oracle.bond_uniform(seed, rep, n, dim, i, mu)
                if mu < 2:
                    w = oracle.word(seed, rep, oracle.TAG_BOND, n, i)
                    p = (w >> 16) if mu == 0 else (w & 0xFFFF)
                else:
                    w = oracle.word(seed, rep, oracle.TAG_BOND_Z, n, i >> 1)
                    p = (w & 0xFFFF) if (i & 1) else (w >> 16)
                s = oracle.word(seed, rep, oracle.TAG_BOND_TIE, n, dim * i + mu) >> 16
                assert u == (p << 16) | s


def test_bond_uniform_is_uniform():
    u = np.array([oracle.bond_uniform(9, 0, 3, 3, i, mu) for i in range(20000) for mu in range(3)],
                 dtype=np.uint64)
    for shift in (28, 12):  # a primary nibble and a secondary nibble
        counts = np.bincount(((u >> shift) & 15).astype(np.int64), minlength=16)
        exp = len(u) / 16
        chi2 = float(((counts - exp) ** 2 / exp).sum())
        assert chi2 < 60  # 15 dof
    d = np.array([oracle.cluster_decision(0, 2, 9, 0, 3, g) for g in range(20000)])
    assert abs(d.mean() - 0.5) < 0.02
    d = np.array([oracle.cluster_decision(1, 5, 9, 0, 3, g) for g in range(20000)])
    assert np.all(np.bincount(d, minlength=5) > 3600)
