"""Pins of the oracle's systematic resampling (CPU only).

Systematic resampling is fixed by its definition: the offspring count of
particle i is the number of points (k+u)/n * C in [C_{i-1}, C_i), which is
floor or ceil of n * wbar_i, and whose expectation over u in [0, 1) is
exactly n * wbar_i.  The expectation is computed here by enumerating every
breakpoint of u (the points where an index changes), not by sampling.
"""
import numpy as np
import pytest

import dpf_synth as S
from oracle.resample import (logsumexp, normalise_log, offspring_counts, systematic,
                             systematic_log, weights_from_log)

KINDS = ["lognormal", "equal", "dominant", "zeros", "tiny", "single"]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", [1, 7, 50, 100, 4096])
def test_invariants(kind, n):
    for seed in range(5):
        w = S.weight_corpus(seed, n, kind)
        u = np.random.default_rng(seed).random()
        A = systematic(w, n, u)
        assert A.shape == (n,)
        assert np.all(np.diff(A) >= 0)
        assert np.all(w[A] > 0)
        O = offspring_counts(A, n)
        assert O.sum() == n
        wb = w / w.sum()
        assert np.all(O >= np.floor(n * wb - 1e-9)) and np.all(O <= np.ceil(n * wb + 1e-9))


def _breakpoints(w, n_out):
    C = np.cumsum(w)
    bps = set([0.0, 1.0])
    for k in range(n_out):
        for c in C:
            u = c * n_out / C[-1] - k
            if 0.0 < u < 1.0:
                bps.add(u)
    return np.array(sorted(bps))


@pytest.mark.parametrize("n,n_out", [(3, 3), (5, 5), (8, 3), (4, 9), (12, 12)])
def test_expected_counts_exact(n, n_out):
    g = np.random.default_rng(n * 31 + n_out)
    for _ in range(10):
        w = g.random(n) ** 3
        w[g.random(n) < 0.2] = 0.0
        if w.sum() == 0:
            w[0] = 1.0
        bps = _breakpoints(w, n_out)
        E = np.zeros(n)
        for lo, hi in zip(bps[:-1], bps[1:]):
            if hi - lo <= 1e-14:
                continue
            A = systematic(w, n_out, 0.5 * (lo + hi))
            E += (hi - lo) * np.bincount(A, minlength=n)
        assert np.allclose(E, n_out * w / w.sum(), atol=1e-9)


def test_single_draw_is_inverse_cdf():
    g = np.random.default_rng(3)
    for _ in range(200):
        w = g.random(6)
        u = g.random()
        C = np.cumsum(w)
        expect = int(np.argmax(C > u * C[-1]))
        assert systematic(w, 1, u)[0] == expect


def test_strict_rule_on_exact_ties():
    # equal weights, u = 0: points are exactly 0, 1, ..., n-1 and C_i = i + 1,
    # so the first index strictly above point k is k.
    n = 10
    A = systematic(np.ones(n), n, 0.0)
    assert np.array_equal(A, np.arange(n))
    # zeros between positive weights are skipped even when a point sits on a boundary
    w = np.array([1.0, 0.0, 0.0, 1.0])
    assert np.array_equal(systematic(w, 4, 0.0), [0, 0, 3, 3])


def test_point_at_total_clamps_to_last_positive():
    w = np.array([0.5, 0.25, 0.25, 0.0, 0.0])
    u = 1.0 - 2.0 ** -53
    A = systematic(w, 5, u)
    assert A[-1] == 2
    assert np.all(w[A] > 0)


def test_log_weights_and_degenerate_fallback():
    lw = np.array([0.0, -np.inf, np.nan, 1.0])
    w, deg, nonf = weights_from_log(lw)
    assert not deg and nonf
    assert np.allclose(w, [np.exp(-1.0), 0.0, 0.0, 1.0])
    w, deg, nonf = weights_from_log(np.array([-np.inf, -np.inf]))
    assert deg and not nonf and np.array_equal(w, [1.0, 1.0])
    A, deg, _ = systematic_log(np.full(4, np.nan), 4, 0.3)
    assert deg and np.array_equal(A, [0, 1, 2, 3])


def test_logsumexp_and_normalise():
    g = np.random.default_rng(4)
    a = g.normal(size=(5, 7)) * 30
    from scipy.special import logsumexp as sp_lse
    assert np.allclose(logsumexp(a), sp_lse(a, axis=1), rtol=1e-13)
    lam, deg = normalise_log(a)
    assert not deg.any()
    assert np.allclose(np.exp(lam).sum(axis=1), 1.0, atol=1e-12)
    lam, deg = normalise_log(np.full((1, 4), -np.inf))
    assert deg[0] and np.allclose(np.exp(lam), 0.25)
