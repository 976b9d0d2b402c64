"""Pins of the oracle's counter-based generator (Philox, Salmon et al. SC'11).

The 4x32 variant the method uses is pinned by the generator authors' published
known-answer vectors (tests/golden/philox4x32_10_kat.txt): a swapped
multiplier, Weyl constant or output word fails them.  The 4x64 variant shares
the round structure and key schedule; it is pinned against numpy's independent
Philox4x64-10 bit generator.  The 32-bit Weyl constants are also checked
against their definitions (golden ratio and sqrt(3) - 1).
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest


def _kat_rows():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "philox4x32_10_kat.txt")
    rows = []
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].split()
            if line:
                rows.append([int(w, 16) for w in line])
    return rows


def test_philox4x32_known_answers(orc):
    rows = _kat_rows()
    assert len(rows) == 3
    for r in rows:
        ctr, key, want = r[0:4], r[4:6], r[6:10]
        got = [int(x) for x in orc.philox4x32(ctr, key)]
        assert got == want, ([hex(x) for x in got], [hex(x) for x in want])


@pytest.mark.parametrize("ctr,key", [
    ([0, 0, 0, 0], [0, 0]),
    ([5, 0, 0, 0], [1, 2]),
    ([123456789, 987654321, 42, 7], [0xDEADBEEFCAFEBABE, 0x0123456789ABCDEF]),
    ([2**64 - 2, 2**63, 1, 2**40 + 3], [2**64 - 1, 17]),
])
def test_philox4x64_matches_numpy(orc, ctr, key):
    # numpy increments the 256-bit counter before producing a block
    # pass uint64 arrays: a Python list of large ints is converted through float64
    bg = np.random.Philox(counter=np.array(ctr, np.uint64), key=np.array(key, np.uint64))
    ref = bg.random_raw(8)
    c1 = list(ctr)
    for blk in range(2):
        # counter + 1 + blk as a 256-bit little-endian integer
        val = sum(int(c) << (64 * i) for i, c in enumerate(ctr)) + 1 + blk
        c1 = [(val >> (64 * i)) & (2**64 - 1) for i in range(4)]
        got = orc.philox4x64(c1, key)
        assert [int(x) for x in got] == [int(x) for x in ref[4 * blk:4 * blk + 4]]


def test_weyl_constants_from_definition():
    # the 32-bit key increments are floor(2^32 * (golden ratio - 1)) and
    # floor(2^32 * (sqrt(3) - 1)); the 64-bit ones carry more bits of the same numbers
    phi_frac = (math.sqrt(5) - 1) / 2
    assert int(phi_frac * 2**32) == 0x9E3779B9
    assert int((math.sqrt(3) - 1) * 2**32) == 0xBB67AE85
    # top halves of the 64-bit constants (checked against numpy above) agree
    assert 0x9E3779B97F4A7C15 >> 32 == 0x9E3779B9
    assert 0xBB67AE8584CAA73B >> 32 == 0xBB67AE85


def test_philox4x32_key_and_counter_sensitivity(orc):
    base = orc.philox4x32([1, 2, 3, 4], [5, 6])
    for i in range(4):
        c = [1, 2, 3, 4]
        c[i] ^= 1
        other = orc.philox4x32(c, [5, 6])
        # avalanche: about half the 128 output bits flip for a one-bit input change
        flips = sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(base, other))
        assert 30 < flips < 98
    for i in range(2):
        k = [5, 6]
        k[i] ^= 1 << 31
        other = orc.philox4x32([1, 2, 3, 4], k)
        flips = sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(base, other))
        assert 30 < flips < 98


def test_philox4x32_uniformity(orc):
    # chi-square on the top 4 bits of 40,000 words
    ws = np.array([orc.word(99, e, 3, 7, 11) for e in range(40000)], np.uint64)
    counts = np.bincount((ws >> 28).astype(np.int64), minlength=16)
    exp = len(ws) / 16
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 45.0  # 15 dof, p ~ 1e-4


def test_word_layout(orc):
    # element e is word (e & 3) of block (e >> 2); counter = (block, t, particle, swarm)
    seed = 0x1234567890ABCDEF
    blk = orc.philox4x32([3, 9, 5, 2], [seed & 0xFFFFFFFF, seed >> 32])
    for w in range(4):
        assert orc.word(seed, 12 + w, 9, 5, 2) == int(blk[w])


def test_u01_and_bounded(orc):
    assert orc.u01(0) == 0.0
    assert orc.u01(0xFFFFFFFF) == float(Fraction(2**24 - 1, 2**24))
    assert orc.u01(0xFFFFFFFF) < 1.0
    assert orc.u01(0x80000000) == 0.5
    # the low 8 bits are dropped, so the value is exact in binary32
    for w in [1, 255, 256, 0xABCDEF12]:
        assert np.float32(orc.u01(w)) == orc.u01(w)
    assert orc.bounded(0, 7) == 0
    assert orc.bounded(0xFFFFFFFF, 7) == 6
    assert orc.bounded(0x80000000, 10) == 5
    # bounded maps the 2^32 words onto [0, m) in m nearly equal runs
    for m in [1, 2, 3, 150, 1000]:
        edges = [orc.bounded(w, m) for w in (0, 2**32 // m - 1, 2**32 // m + 1, 2**32 - 1)]
        assert edges[0] == 0 and edges[-1] == m - 1
        assert all(0 <= e < m for e in edges)
