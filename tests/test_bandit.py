"""Hedge and Exp3 (Section 3, Fig. 5) and the reward of Section 4.3, pinned
against values worked out by hand from the algorithms' definitions."""
import math

import numpy as np
import pytest

from paper_1203_2394_amd import bandit as B


def test_reward_is_alpha_over_alpha_plus_squared_error():
    assert B.reward(0.0) == 1.0
    assert math.isclose(float(B.reward(0.1)), 0.001 / (0.001 + 0.01))
    assert math.isclose(float(B.reward(-2.0, alpha=0.5)), 0.5 / 4.5)
    r = B.reward(np.linspace(-5, 5, 101))
    assert np.all((r > 0) & (r <= 1))


def test_hedge_probabilities_by_hand():
    # eta = 0.5, K = 2; rewards (0.2, 0.6) then (1.0, 0.1)
    h = B.Hedge(2, 0.5)
    assert np.allclose(h.probs(), [0.5, 0.5])
    h.update([0.2, 0.6])
    # exp(0.1) = 1.1051709181, exp(0.3) = 1.3498588076
    assert np.allclose(h.probs(), [1.1051709181 / 2.4550297257, 1.3498588076 / 2.4550297257], atol=1e-10)
    h.update([1.0, 0.1])
    # G = (1.2, 0.7): exp(0.6) = 1.8221188004, exp(0.35) = 1.4190675486
    assert np.allclose(h.probs(), [1.8221188004 / 3.2411863490, 1.4190675486 / 3.2411863490], atol=1e-10)
    # the draw is the inverse CDF of the probabilities
    assert h.choose(0.5) == 0 and h.choose(0.57) == 1


def test_exp3_updates_by_hand():
    # gamma = 0.2, eta = 0.5, K = 2
    e = B.Exp3(2, 0.5, 0.2)
    assert np.allclose(e.probs(), [0.5, 0.5])
    i = e.choose(0.3)                         # p^ = (0.5, 0.5): action 0
    assert i == 0
    e.update(i, 0.4)                          # r^ = (0.4 / 0.5, 0) = (0.8, 0)
    assert np.allclose(e.hedge.G, [0.8, 0.0])
    # p = (exp(0.4), 1) / (exp(0.4) + 1), exp(0.4) = 1.4918246976
    p0 = 1.4918246976 / 2.4918246976
    assert np.allclose(e.hedge.probs(), [p0, 1 - p0], atol=1e-10)
    assert np.allclose(e.probs(), [0.8 * p0 + 0.1, 0.8 * (1 - p0) + 0.1], atol=1e-10)
    i = e.choose(0.99)                        # action 1
    assert i == 1
    ph1 = 0.8 * (1 - p0) + 0.1
    e.update(i, 1.0)                          # r^ = (0, 1 / p^_1)
    assert np.allclose(e.hedge.G, [0.8, 1.0 / ph1], atol=1e-12)


def test_run_helpers_follow_the_step_rules():
    g = np.random.default_rng(3)
    R = g.random((50, 3))
    u = g.random(50)
    acts, P = B.run_hedge(R, 0.7, u)
    h = B.Hedge(3, 0.7)
    for t in range(50):
        assert np.allclose(P[t], h.probs())
        assert acts[t] == h.choose(u[t])
        h.update(R[t])
    acts, P, Ph = B.run_exp3(R, 0.7, 0.3, u)
    e = B.Exp3(3, 0.7, 0.3)
    for t in range(50):
        assert np.allclose(Ph[t], e.probs()) and np.allclose(P[t], e.hedge.probs())
        i = e.choose(u[t])
        assert acts[t] == i
        e.update(i, R[t, i])


def test_exp3_finds_the_better_action_and_adapts_after_a_change():
    """Rewards drawn around 0.3 and 0.7; the better action swaps at t = 1500.
    Exp3 (gamma = 0.2, eta = 0.05) puts most of its weight on the better action
    before the change and moves it over afterwards; gamma keeps every
    action's probability at least gamma / K."""
    T, tc = 4000, 1500
    g = np.random.default_rng(11)
    base = np.where(np.arange(T)[:, None] < tc, [0.3, 0.7], [0.7, 0.3])
    R = np.clip(base + 0.05 * g.normal(size=(T, 2)), 0, 1)
    acts, P, Ph = B.run_exp3(R, 0.05, 0.2, B.uniforms(5, T))
    assert Ph.min() >= 0.1 - 1e-12
    assert P[tc - 1, 1] > 0.95
    assert P[-1, 0] > 0.95
    assert np.mean(acts[-500:] == 0) > 0.8


def test_long_runs_do_not_overflow():
    T = 20000
    R = np.ones((T, 2))
    R[:, 1] = 0.0
    acts, P, Ph = B.run_exp3(R, 0.5, 0.2, B.uniforms(1, T))
    assert np.all(np.isfinite(P)) and P[-1, 0] > 1 - 1e-12
    acts, P = B.run_hedge(R, 0.5, B.uniforms(2, T))
    assert np.all(np.isfinite(P))


@pytest.mark.parametrize("bad", [(0, 0.5), (2, 0.0)])
def test_hedge_rejects_bad_parameters(bad):
    with pytest.raises(ValueError):
        B.Hedge(*bad)
    with pytest.raises(ValueError):
        B.Exp3(2, 0.5, 0.0)
