"""Pins of the oracle's random-number contract (CPU only).

The generator is Philox4x32-10 (Salmon et al., SC'11).  Its published
known-answer vectors pin the round function, multipliers and key schedule;
the transforms are pinned by exact end points, by Python-integer evaluation
of the bit formulas and by distribution tests against SciPy.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

from oracle import philox as P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            assert parts[0] == "10"
            vals = [int(v, 16) for v in parts[1:]]
            rows.append((vals[0:4], vals[4:6], vals[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(ctr, key, expect):
    out = P.philox4x32_10(np.array(ctr, dtype=np.uint32), np.array(key, dtype=np.uint32))
    assert [int(v) for v in out] == expect


def test_philox_vectorised_matches_scalar():
    g = np.random.default_rng(0)
    ctr = g.integers(0, 2 ** 32, size=(50, 4), dtype=np.uint64).astype(np.uint32)
    key = g.integers(0, 2 ** 32, size=(50, 2), dtype=np.uint64).astype(np.uint32)
    batch = P.philox4x32_10(ctr, key)
    for r in range(50):
        assert np.array_equal(batch[r], P.philox4x32_10(ctr[r], key[r]))


def test_key_and_counter_layout():
    seed = 0x0123456789ABCDEF
    k = P.key_of(seed, 5)
    assert int(k[0]) == 0x89ABCDEF and int(k[1]) == (0x01234567 ^ 5)
    w = P.words(seed, 5, 7, 11, 13, P.NEW_Z, 2)
    direct = P.philox4x32_10(np.array([7, 11, 13, (P.NEW_Z << 24) | 2], dtype=np.uint32), k)
    assert np.array_equal(w, direct)


def test_u24_exact_endpoints_and_formula():
    assert P.u24(0) == 2.0 ** -24
    assert P.u24(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    g = np.random.default_rng(1)
    w = g.integers(0, 2 ** 32, size=1000, dtype=np.uint64)
    got = P.u24(w)
    for wi, gi in zip(w[:50], got[:50]):
        assert gi == (2 * (int(wi) >> 9) + 1) / 2 ** 24
    # exactly representable in float32
    assert np.array_equal(got.astype(np.float32).astype(np.float64), got)


def test_u53_formula_and_range():
    assert P.u53(0, 0) == 0.0
    assert P.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    g = np.random.default_rng(2)
    w0 = g.integers(0, 2 ** 32, size=200, dtype=np.uint64)
    w1 = g.integers(0, 2 ** 32, size=200, dtype=np.uint64)
    got = P.u53(w0, w1)
    for a, b, v in zip(w0, w1, got):
        assert v == ((int(a) << 21) | (int(b) >> 11)) / 2 ** 53


def test_uniforms_are_uniform():
    u = P.uniform53(42, 3, 9, np.arange(200000), P.CAND_U)
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    w = P.words(42, 3, 9, np.arange(50000), 1, P.LA_X, 0)
    for s in range(4):
        assert stats.kstest(P.u24(w[:, s]), "uniform").pvalue > 1e-3


def test_normals_distribution_and_independence():
    n = P.normals(7, 0, 3, np.arange(40000)[:, None], np.arange(4)[None, :], P.LA_Z, 6)
    flat = n.reshape(-1, 6)
    for d in range(6):
        assert stats.kstest(flat[:, d], "norm").pvalue > 1e-3
    c = np.corrcoef(flat.T)
    assert np.max(np.abs(c - np.eye(6))) < 0.02
    # normal d of a draw comes from block d // 4: the 5th normal uses block 1
    w1 = P.words(7, 0, 3, 5, 2, P.LA_Z, 1)
    r = np.sqrt(-2 * np.log(P.u24(w1[0])))
    assert np.isclose(n[5, 2, 4], r * np.cos(2 * np.pi * P.u24(w1[1])), rtol=0, atol=1e-15)
    assert np.isclose(n[5, 2, 5], r * np.sin(2 * np.pi * P.u24(w1[1])), rtol=0, atol=1e-15)


def test_packed_normals_distribution_and_independence():
    """Ten normals per two blocks: the remnant pairs (normals 8, 9, 18, 19)
    are standard normal and uncorrelated with the word normals of the same
    blocks and with each other."""
    n = P.normals(11, 2, 5, np.arange(30000)[:, None], np.arange(2)[None, :], P.NEW_Z, 20)
    flat = n.reshape(-1, 20)
    for d in range(20):
        assert stats.kstest(flat[:, d], "norm").pvalue > 1e-3, d
    c = np.corrcoef(flat.T)
    assert np.max(np.abs(c - np.eye(20))) < 0.02
    # squares too: a remnant built from bits shared with U24 would couple radii
    c2 = np.corrcoef((flat ** 2).T)
    assert np.max(np.abs(c2 - np.eye(20))) < 0.03


def test_packed_layout_from_raw_words():
    """Normals 0-7 of a packed draw are blocks 0 and 1 in slot order (the
    block-aligned layout); normals 8, 9 come from the two blocks' remnant
    uniforms, here rebuilt bit by bit with Python integers; normals 10-13
    come from block 2."""
    D = 14
    n = P.normals(5, 1, 9, 3, 7, P.LA_X, D)
    nb = P.normals_blocked(5, 1, 9, 3, 7, P.LA_X, 8)
    assert np.array_equal(n[:8], nb)
    w0 = [int(v) for v in P.words(5, 1, 9, 3, 7, P.LA_X, 0)]
    w1 = [int(v) for v in P.words(5, 1, 9, 3, 7, P.LA_X, 1)]
    w2 = [int(v) for v in P.words(5, 1, 9, 3, 7, P.LA_X, 2)]

    def rem(w):
        bits = [(w[0] >> k) & 1 for k in range(9)] + [(w[1] >> k) & 1 for k in range(9)] + \
            [(w[2] >> k) & 1 for k in range(5)]
        v = sum(b << k for k, b in enumerate(bits))
        return (2 * v + 1) / 2.0 ** 24

    a, b = rem(w0), rem(w1)
    r = math.sqrt(-2 * math.log(a))
    assert math.isclose(n[8], r * math.cos(2 * math.pi * b), rel_tol=0, abs_tol=1e-14)
    assert math.isclose(n[9], r * math.sin(2 * math.pi * b), rel_tol=0, abs_tol=1e-14)
    r2 = math.sqrt(-2 * math.log((2 * (w2[0] >> 9) + 1) / 2.0 ** 24))
    assert math.isclose(n[10], r2 * math.cos(2 * math.pi * (2 * (w2[1] >> 9) + 1) / 2.0 ** 24), abs_tol=1e-14)
    # a shorter draw is a prefix of a longer one
    assert np.array_equal(P.normals(5, 1, 9, 3, 7, P.LA_X, 9), n[:9])


def test_streams_differ_by_every_key_field():
    base = P.words(1, 0, 1, 2, 3, P.LA_X, 0)
    for args in [(2, 0, 1, 2, 3, P.LA_X, 0), (1, 1, 1, 2, 3, P.LA_X, 0),
                 (1, 0, 2, 2, 3, P.LA_X, 0), (1, 0, 1, 3, 3, P.LA_X, 0),
                 (1, 0, 1, 2, 4, P.LA_X, 0), (1, 0, 1, 2, 3, P.LA_Z, 0),
                 (1, 0, 1, 2, 3, P.LA_X, 1)]:
        assert not np.array_equal(base, P.words(*args))
